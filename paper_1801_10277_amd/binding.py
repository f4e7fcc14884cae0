"""ctypes binding of libceleste.so (argument marshalling only).

Every entry point of include/celeste.h is exposed under the same name; `Plan` wraps a
plan built from a synthetic `Field` and takes torch float64 CUDA tensors for device
buffers and the current torch stream for ordering.  All arithmetic runs in the HIP
library: if it is missing, importing this module raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libceleste.so")

CELESTE_OK = 0
CELESTE_EINVAL = -1
CELESTE_ECONFLICT = -2
CELESTE_EHIP = -3
CELESTE_ENOMEM = -4
CELESTE_EDOMAIN = -5
CELESTE_ESCRATCH = -6
CELESTE_PLAIN = 0
CELESTE_BATCHED = 1
CELESTE_INCLUDE_KL = 1
CELESTE_INCLUDE_LGAMMA = 2
CELESTE_COLOR_MIXTURE = 4
ROW = 48              # theta / gradient row width
EXPORTS = ["celeste_plan_create", "celeste_plan_destroy", "celeste_plan_get_info", "celeste_elbo",
           "celeste_elbo_grad", "celeste_hvp", "celeste_hessian", "celeste_newton", "celeste_total_elbo",
           "celeste_color_batches", "celeste_sweep", "celeste_plan_set_launch", "celeste_autotune",
           "celeste_plan_use_graph", "celeste_plan_profile", "celeste_plan_status", "celeste_last_hip_error",
           "celeste_status_string", "celeste_version", "celeste_debug_math", "celeste_conflict_graph",
           "celeste_cyclades_batches", "celeste_plan_set_hessian_mode", "celeste_elbo_grad_noalloc",
           "celeste_work_counts"]


class celeste_image(C.Structure):
    _fields_ = [("band", C.c_int32), ("H", C.c_int32), ("W", C.c_int32), ("reserved", C.c_int32),
                ("pix_offset", C.c_int64), ("sky", C.c_double), ("iota", C.c_double),
                ("origin_x", C.c_double), ("origin_y", C.c_double), ("psf", C.c_double * 18),
                ("sky_map", C.c_void_p), ("wcs", C.c_double * 4)]


class celeste_box(C.Structure):
    _fields_ = [("img", C.c_int32), ("r0", C.c_int32), ("c0", C.c_int32), ("h", C.c_int32),
                ("w", C.c_int32)]


class celeste_problem_desc(C.Structure):
    _fields_ = [("n_img", C.c_int32), ("n_src", C.c_int32), ("images", C.POINTER(celeste_image)),
                ("x", C.c_void_p), ("n_pix", C.c_int64), ("patch_ptr", C.POINTER(C.c_int32)),
                ("boxes", C.POINTER(celeste_box)),
                ("exp_alpha", C.c_double * 6), ("exp_nu", C.c_double * 6),
                ("dev_alpha", C.c_double * 8), ("dev_nu", C.c_double * 8),
                ("prior_phi", C.c_double), ("prior_r", C.c_double * 4), ("prior_c", C.c_double * 16),
                ("flags", C.c_uint32), ("reserved", C.c_int32),
                ("color_mix_w", C.c_double * 16), ("color_mix_mean", C.c_double * 64),
                ("color_mix_cov", C.c_double * 256)]


class celeste_tr_params(C.Structure):
    _fields_ = [("radius0", C.c_double), ("radius_max", C.c_double), ("eta_accept", C.c_double),
                ("gtol", C.c_double), ("newton_steps", C.c_int32), ("reserved", C.c_int32)]


class celeste_plan_info(C.Structure):
    _fields_ = [("n_visits", C.c_int64), ("n_pairs", C.c_int64), ("n_items", C.c_int64),
                ("n_tiles", C.c_int64), ("n_nbr", C.c_int64), ("chunk", C.c_int32),
                ("waves_per_block", C.c_int32), ("grid_blocks", C.c_int32), ("tile_h", C.c_int32),
                ("tile_w", C.c_int32), ("dynamic_queue", C.c_int32), ("strip_rows", C.c_int32),
                ("render_mode", C.c_int32), ("n_classes", C.c_int32), ("n_params", C.c_int32),
                ("workspace_bytes", C.c_int64)]


_lib = None


def lib():
    """Load libceleste.so (built in-tree by paper_1801_10277_amd.csrc.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libceleste.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1801_10277_amd.csrc.build)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)
    L.celeste_plan_create.argtypes = [C.POINTER(celeste_problem_desc), C.POINTER(vp)]
    L.celeste_plan_destroy.argtypes = [vp]
    L.celeste_plan_destroy.restype = None
    L.celeste_plan_get_info.argtypes = [vp, C.POINTER(celeste_plan_info)]
    L.celeste_elbo.argtypes = [vp, dp, dp, C.c_int, dp, vp]
    L.celeste_elbo_grad.argtypes = [vp, dp, dp, C.c_int, dp, dp, vp]
    L.celeste_elbo_grad_noalloc.argtypes = [vp, dp, dp, dp, dp, vp]
    L.celeste_hvp.argtypes = [vp, dp, dp, dp, dp, vp]
    L.celeste_hessian.argtypes = [vp, dp, ip, C.c_int, dp, vp]
    L.celeste_newton.argtypes = [vp, dp, ip, C.c_int, C.c_int, C.POINTER(celeste_tr_params), dp, dp, vp]
    L.celeste_total_elbo.argtypes = [vp, dp, dp, vp]
    L.celeste_work_counts.argtypes = [vp, dp, C.POINTER(C.c_int64), vp]
    L.celeste_color_batches.argtypes = [vp, C.c_uint64, ip, ip, ip]
    L.celeste_sweep.argtypes = [vp, dp, ip, ip, C.c_int, C.c_int, C.POINTER(celeste_tr_params), dp, vp]
    L.celeste_plan_set_hessian_mode.argtypes = [vp, C.c_int]
    L.celeste_conflict_graph.argtypes = [vp, ip, ip, C.c_int64, C.POINTER(C.c_int64)]
    L.celeste_cyclades_batches.argtypes = [C.c_int32, ip, ip, ip, C.c_int32, ip, ip, ip, ip]
    L.celeste_plan_set_launch.argtypes = [vp] + [C.c_int] * 8
    L.celeste_autotune.argtypes = [vp, dp, C.c_int, C.POINTER(C.c_double), vp]
    L.celeste_plan_use_graph.argtypes = [vp, C.c_int]
    L.celeste_plan_profile.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    L.celeste_plan_status.argtypes = [vp, vp]
    L.celeste_last_hip_error.restype = C.c_char_p
    L.celeste_debug_math.argtypes = [C.c_int, dp, dp, C.c_int, vp]
    L.celeste_status_string.argtypes = [C.c_int]
    L.celeste_status_string.restype = C.c_char_p
    _lib = L
    return L


class CelesteError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().celeste_status_string(code).decode()
        if code == CELESTE_EHIP:
            msg += " (" + lib().celeste_last_hip_error().decode() + ")"
        super().__init__("%s failed: %s [%d]" % (what, msg, code))
        self.code = code


def check(code, what):
    if code != CELESTE_OK:
        raise CelesteError(code, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def tr_params(radius0=1.0, radius_max=1e3, eta_accept=0.1, gtol=1e-8, newton_steps=10):
    p = celeste_tr_params()
    p.radius0, p.radius_max, p.eta_accept, p.gtol = radius0, radius_max, eta_accept, gtol
    p.newton_steps = newton_steps
    return p


FN_EXP, FN_LOG, FN_RCP = 0, 1, 2


def _i32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def cyclades_batches(adj_ptr, adj, order, sample_size):
    """celeste_cyclades_batches on host arrays (no GPU needed): (batch_ptr, batch_src,
    n_components)."""
    adj_ptr = np.ascontiguousarray(adj_ptr, np.int32)
    adj = np.ascontiguousarray(adj, np.int32)
    order = np.ascontiguousarray(order, np.int32)
    n = len(adj_ptr) - 1
    if len(order) != n:
        raise CelesteError(CELESTE_EINVAL, "celeste_cyclades_batches")
    bp = np.zeros(n + 1, np.int32)
    bs = np.zeros(max(n, 1), np.int32)
    nb, nc = C.c_int32(), C.c_int32()
    check(lib().celeste_cyclades_batches(n, _i32p(adj_ptr), _i32p(adj) if len(adj) else None,
                                         _i32p(order) if n else None, sample_size, _i32p(bp), _i32p(bs),
                                         C.byref(nb), C.byref(nc)), "celeste_cyclades_batches")
    return bp[:nb.value + 1].copy(), bs[:n].copy(), nc.value



def debug_math(fn, x):
    """The strip kernels' table-driven exp (FN_EXP), table-driven log (FN_LOG) or Newton
    reciprocal (FN_RCP) on a float64 CUDA tensor."""
    import torch
    y = torch.empty_like(x)
    check(lib().celeste_debug_math(fn, _ptr(x), _ptr(y), x.numel(), _stream()), "celeste_debug_math")
    return y


class Plan:
    """A libceleste plan for one synthetic Field; pixel data lives in a torch CUDA tensor."""

    def __init__(self, f, device="cuda", flags=None, check_status=True):
        import torch
        L = lib()
        self.field = f
        self.S = f.n_src
        self.check_status = check_status
        self.x = torch.as_tensor(np.ascontiguousarray(f.x, np.float64)).to(device)
        smap = getattr(f, "sky_map", None)
        self.sky_map = None if smap is None else torch.as_tensor(np.ascontiguousarray(smap, np.float64)).to(device)
        n = f.n_img
        imgs = (celeste_image * n)()
        for i in range(n):
            im = imgs[i]
            im.band, im.H, im.W = int(f.img_band[i]), int(f.img_H[i]), int(f.img_W[i])
            im.pix_offset = int(f.img_off[i])
            im.sky, im.iota = float(f.img_sky[i]), float(f.img_iota[i])
            im.origin_x, im.origin_y = float(f.img_origin[i, 0]), float(f.img_origin[i, 1])
            for k, v in enumerate(np.asarray(f.img_psf[i], np.float64).reshape(-1)):
                im.psf[k] = float(v)
            for k, v in enumerate(np.asarray(f.wcs(i), np.float64).reshape(-1)):
                im.wcs[k] = float(v)
            if self.sky_map is not None:
                im.sky_map = self.sky_map.data_ptr() + 8 * int(f.img_off[i])
        ptr = np.ascontiguousarray(f.patch_ptr, np.int32)
        nb = int(ptr[-1])
        boxes = (celeste_box * max(nb, 1))()
        for b in range(nb):
            boxes[b].img, boxes[b].r0, boxes[b].c0, boxes[b].h, boxes[b].w = (int(v) for v in f.boxes[b])
        d = celeste_problem_desc()
        d.n_img, d.n_src = n, f.n_src
        d.images = C.cast(imgs, C.POINTER(celeste_image))
        d.x = self.x.data_ptr()
        d.n_pix = int(self.x.numel())
        self._ptr = ptr
        d.patch_ptr = ptr.ctypes.data_as(C.POINTER(C.c_int32))
        d.boxes = C.cast(boxes, C.POINTER(celeste_box))
        for name in ("exp_alpha", "exp_nu", "dev_alpha", "dev_nu"):
            arr = getattr(d, name)
            for k, v in enumerate(getattr(f, name)):
                arr[k] = float(v)
        d.prior_phi = float(f.prior_phi)
        for k, v in enumerate(np.asarray(f.prior_r).reshape(-1)):
            d.prior_r[k] = float(v)
        for k, v in enumerate(np.asarray(f.prior_c).reshape(-1)):
            d.prior_c[k] = float(v)
        d.flags = int(f.flags if flags is None else flags)
        if d.flags & CELESTE_COLOR_MIXTURE:
            for name in ("color_mix_w", "color_mix_mean", "color_mix_cov"):
                arr = getattr(d, name)
                for k, v in enumerate(np.asarray(getattr(f, name), np.float64).reshape(-1)):
                    arr[k] = float(v)
        self.n_params = 43 if d.flags & CELESTE_COLOR_MIXTURE else 27
        self.desc = d
        h = C.c_void_p()
        check(L.celeste_plan_create(C.byref(d), C.byref(h)), "celeste_plan_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.celeste_plan_destroy(self.h)
            self.h = None

    # ---- helpers
    def _status(self, what):
        if self.check_status:
            check(lib().celeste_plan_status(self.h, _stream()), what + " (device status)")

    def _theta(self, theta):
        import torch
        assert theta.dtype == torch.float64 and theta.is_cuda and theta.is_contiguous()
        assert theta.shape == (self.S, ROW)
        return theta

    def info(self):
        i = celeste_plan_info()
        check(lib().celeste_plan_get_info(self.h, C.byref(i)), "celeste_plan_get_info")
        return {k: getattr(i, k) for k, _ in i._fields_}

    # ---- entry points
    def elbo(self, theta, mode=CELESTE_BATCHED, active=None, out=None):
        import torch
        self._theta(theta)
        out = torch.zeros(self.S, dtype=torch.float64, device=theta.device) if out is None else out
        check(lib().celeste_elbo(self.h, _ptr(theta), _ptr(active), mode, _ptr(out), _stream()), "celeste_elbo")
        self._status("celeste_elbo")
        return out

    def elbo_grad(self, theta, mode=CELESTE_BATCHED, active=None, elbo=None, grad=None):
        import torch
        self._theta(theta)
        elbo = torch.zeros(self.S, dtype=torch.float64, device=theta.device) if elbo is None else elbo
        grad = torch.zeros(self.S, ROW, dtype=torch.float64, device=theta.device) if grad is None else grad
        check(lib().celeste_elbo_grad(self.h, _ptr(theta), _ptr(active), mode, _ptr(elbo), _ptr(grad),
                                      _stream()), "celeste_elbo_grad")
        self._status("celeste_elbo_grad")
        return elbo, grad

    def elbo_grad_noalloc(self, theta, active=None, elbo=None, grad=None):
        """celeste_elbo_grad_noalloc: the batched ELBO + gradient with the library's static
        scratch instead of plan memory (the call itself allocates nothing)."""
        import torch
        self._theta(theta)
        elbo = torch.zeros(self.S, dtype=torch.float64, device=theta.device) if elbo is None else elbo
        grad = torch.zeros(self.S, ROW, dtype=torch.float64, device=theta.device) if grad is None else grad
        check(lib().celeste_elbo_grad_noalloc(self.h, _ptr(theta), _ptr(active), _ptr(elbo), _ptr(grad),
                                              _stream()), "celeste_elbo_grad_noalloc")
        self._status("celeste_elbo_grad_noalloc")
        return elbo, grad

    def hvp(self, theta, v, with_grad=False):
        import torch
        self._theta(theta)
        hv = torch.zeros(self.S, ROW, dtype=torch.float64, device=theta.device)
        g = torch.zeros(self.S, ROW, dtype=torch.float64, device=theta.device) if with_grad else None
        check(lib().celeste_hvp(self.h, _ptr(theta), _ptr(v.contiguous()), _ptr(hv), _ptr(g), _stream()),
              "celeste_hvp")
        self._status("celeste_hvp")
        return (hv, g) if with_grad else hv

    def hessian(self, theta, src):
        import torch
        self._theta(theta)
        src = np.ascontiguousarray(src, np.int32)
        H = torch.zeros(len(src), self.n_params, self.n_params, dtype=torch.float64, device=theta.device)
        check(lib().celeste_hessian(self.h, _ptr(theta), src.ctypes.data_as(C.POINTER(C.c_int32)), len(src),
                                    _ptr(H), _stream()), "celeste_hessian")
        self._status("celeste_hessian")
        return H

    def newton(self, theta, src, n_steps, params=None, radius=None, elbo_out=True):
        import torch
        self._theta(theta)
        params = params or tr_params()
        src = np.ascontiguousarray(src, np.int32)
        if radius is None:
            radius = torch.full((self.S,), params.radius0, dtype=torch.float64, device=theta.device)
        e = torch.zeros(self.S, dtype=torch.float64, device=theta.device) if elbo_out else None
        check(lib().celeste_newton(self.h, _ptr(theta), src.ctypes.data_as(C.POINTER(C.c_int32)), len(src),
                                   n_steps, C.byref(params), _ptr(radius), _ptr(e), _stream()),
              "celeste_newton")
        self._status("celeste_newton")
        return e, radius

    def total_elbo(self, theta):
        import torch
        self._theta(theta)
        out = torch.zeros(1, dtype=torch.float64, device=theta.device)
        check(lib().celeste_total_elbo(self.h, _ptr(theta), _ptr(out), _stream()), "celeste_total_elbo")
        self._status("celeste_total_elbo")
        return out

    WORK_KEYS = ("strips", "visits", "group_strips", "star_strips", "galaxy_strips", "pad_strips",
                 "star_visits", "galaxy_visits", "pad_visits")

    def work_counts(self, theta):
        """Work of the strip passes at theta under the component culling (dict of
        WORK_KEYS); synchronises the stream."""
        out = (C.c_int64 * len(self.WORK_KEYS))()
        check(lib().celeste_work_counts(self.h, _ptr(self._theta(theta)), out, _stream()), "celeste_work_counts")
        return dict(zip(self.WORK_KEYS, (int(v) for v in out)))

    def color_batches(self, seed=0):
        ptr = np.zeros(self.S + 1, np.int32)
        src = np.zeros(self.S, np.int32)
        nb = C.c_int32()
        check(lib().celeste_color_batches(self.h, seed, ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                                          src.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nb)),
              "celeste_color_batches")
        return ptr[:nb.value + 1].copy(), src

    def set_hessian_mode(self, mode):
        """0: closed-form position / shape Hessian rows (default); 1: tangent passes."""
        check(lib().celeste_plan_set_hessian_mode(self.h, mode), "celeste_plan_set_hessian_mode")

    def conflict_graph(self):
        """Box-overlap conflict graph as host CSR (adj_ptr [S + 1], adj)."""
        ptr = np.zeros(self.S + 1, np.int32)
        n = C.c_int64()
        code = lib().celeste_conflict_graph(self.h, _i32p(ptr), None, 0, C.byref(n))
        if code != CELESTE_EINVAL or n.value == 0:
            check(code, "celeste_conflict_graph")
        adj = np.zeros(max(n.value, 1), np.int32)
        check(lib().celeste_conflict_graph(self.h, _i32p(ptr), _i32p(adj), len(adj), C.byref(n)),
              "celeste_conflict_graph")
        return ptr, adj[:n.value].copy()

    def cyclades_batches(self, seed, sample_size, graph=None):
        """Cyclades schedule of one epoch: the sampling order is a seeded permutation of the
        sources; `graph` is conflict_graph()'s result, fetched when None.  Returns
        (batch_ptr, batch_src, n_components, order)."""
        order = np.random.default_rng(seed).permutation(self.S).astype(np.int32)
        ptr, adj = self.conflict_graph() if graph is None else graph
        bp, bs, nc = cyclades_batches(ptr, adj, order, sample_size)
        return bp, bs, nc, order

    def sweep(self, theta, batch_ptr, batch_src, n_sweeps, params=None):
        import torch
        self._theta(theta)
        params = params or tr_params()
        bp = np.ascontiguousarray(batch_ptr, np.int32)
        bs = np.ascontiguousarray(batch_src, np.int32)
        trace = torch.zeros(n_sweeps + 1, dtype=torch.float64, device=theta.device)
        check(lib().celeste_sweep(self.h, _ptr(theta), bp.ctypes.data_as(C.POINTER(C.c_int32)),
                                  bs.ctypes.data_as(C.POINTER(C.c_int32)), len(bp) - 1, n_sweeps,
                                  C.byref(params), _ptr(trace), _stream()), "celeste_sweep")
        self._status("celeste_sweep")
        return trace

    def set_launch(self, chunk=64, waves_per_block=4, grid_blocks=0, dynamic=0, tile_h=16, tile_w=16,
                   strip_rows=16, render_mode=2):
        check(lib().celeste_plan_set_launch(self.h, chunk, waves_per_block, grid_blocks, dynamic, tile_h,
                                            tile_w, strip_rows, render_mode), "celeste_plan_set_launch")

    def autotune(self, theta, reps=5):
        ms = C.c_double()
        check(lib().celeste_autotune(self.h, _ptr(self._theta(theta)), reps, C.byref(ms), _stream()),
              "celeste_autotune")
        return ms.value

    def profile(self, enable=True, reset=True):
        """Enable/disable phase timing; returns (ms[4] summed since last reset, calls)."""
        ms = (C.c_double * 4)()
        n = C.c_int64()
        check(lib().celeste_plan_profile(self.h, 1 if enable else 0, ms, C.byref(n), 1 if reset else 0),
              "celeste_plan_profile")
        return list(ms), n.value

    def use_graph(self, enable=True):
        check(lib().celeste_plan_use_graph(self.h, 1 if enable else 0), "celeste_plan_use_graph")
