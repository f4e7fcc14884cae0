"""ctypes front end of the FP64 CPU oracle (celeste_oracle.cpp).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline leg of
bench.py.  It never touches the HIP library and the HIP library never touches it.

Functions take a `Field` from paper_1801_10277_amd.synth (plain numpy arrays) and an
optional theta override.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "celeste_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=False):
    """Compile the oracle with g++ (-O2, no FMA contraction, OpenMP for the batch call)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class OImage(C.Structure):
    _fields_ = [("band", C.c_int32), ("H", C.c_int32), ("W", C.c_int32), ("pad", C.c_int32),
                ("off", C.c_int64), ("sky", C.c_double), ("iota", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("psf", C.c_double * 18),
                ("sky_map", C.POINTER(C.c_double)), ("wcs", C.c_double * 4)]


class OProblem(C.Structure):
    _fields_ = [("n_img", C.c_int32), ("n_src", C.c_int32),
                ("img", C.POINTER(OImage)), ("x", C.POINTER(C.c_double)),
                ("patch_ptr", C.POINTER(C.c_int32)), ("box", C.POINTER(C.c_int32)),
                ("theta", C.POINTER(C.c_double)),
                ("exp_alpha", C.c_double * 6), ("exp_nu", C.c_double * 6),
                ("dev_alpha", C.c_double * 8), ("dev_nu", C.c_double * 8),
                ("prior_phi", C.c_double), ("prior_r", C.c_double * 4),
                ("prior_c", C.c_double * 16), ("flags", C.c_int32), ("pad", C.c_int32),
                ("mix_w", C.c_double * 16), ("mix_mean", C.c_double * 64), ("mix_cov", C.c_double * 256)]


ROW = 48          # theta row width
FLAG_MIX = 4      # colour prior as a Gaussian mixture (16 responsibilities in the row)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.POINTER(OProblem)
        dp = C.POINTER(C.c_double)
        L.oracle_source_value.argtypes = [P, C.c_int, dp]
        L.oracle_source_grad.argtypes = [P, C.c_int, dp, dp, dp]
        L.oracle_source_hvp.argtypes = [P, C.c_int, dp, dp, dp]
        L.oracle_source_hessian.argtypes = [P, C.c_int, dp, dp]
        L.oracle_render.argtypes = [P, C.c_int, dp, dp]
        L.oracle_source_light.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.oracle_profiles.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double, dp]
        L.oracle_flux_moments.argtypes = [P, C.c_int, C.c_int, C.c_int, dp]
        L.oracle_kl.argtypes = [P, C.c_int]
        L.oracle_kl.restype = C.c_double
        L.oracle_total_elbo.argtypes = [P]
        L.oracle_total_elbo.restype = C.c_double
        L.oracle_grad_many.argtypes = [P, C.c_int, C.POINTER(C.c_int32), dp, dp]
        L.oracle_n_params.argtypes = [P]
        assert L.oracle_sizeof_image() == C.sizeof(OImage)
        assert L.oracle_sizeof_problem() == C.sizeof(OProblem)
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, f, theta=None, flags=None):
        n = f.n_img
        imgs = (OImage * n)()
        for i in range(n):
            im = imgs[i]
            im.band, im.H, im.W = int(f.img_band[i]), int(f.img_H[i]), int(f.img_W[i])
            im.off = int(f.img_off[i])
            im.sky, im.iota = float(f.img_sky[i]), float(f.img_iota[i])
            im.ox, im.oy = float(f.img_origin[i, 0]), float(f.img_origin[i, 1])
            for k, v in enumerate(np.asarray(f.img_psf[i], np.float64).reshape(-1)):
                im.psf[k] = float(v)
            A = f.wcs(i)
            for k, v in enumerate(np.asarray(A, np.float64).reshape(-1)):
                im.wcs[k] = float(v)
        self.imgs = imgs
        # per-pixel sky maps: same layout as x
        self.sky_map = None
        if getattr(f, "sky_map", None) is not None:
            self.sky_map = np.ascontiguousarray(f.sky_map, np.float64)
            for i in range(n):
                imgs[i].sky_map = C.cast(C.c_void_p(self.sky_map.ctypes.data + 8 * int(f.img_off[i])),
                                         C.POINTER(C.c_double))
        self.x = np.ascontiguousarray(f.x, np.float64)
        self.ptr = np.ascontiguousarray(f.patch_ptr, np.int32)
        self.box = np.ascontiguousarray(f.boxes, np.int32).reshape(-1)
        th = f.theta if theta is None else theta
        self.theta = np.ascontiguousarray(th, np.float64).reshape(-1, ROW)
        p = OProblem()
        p.n_img, p.n_src = n, self.theta.shape[0]
        p.img = C.cast(imgs, C.POINTER(OImage))
        p.x = _dp(self.x)
        p.patch_ptr = self.ptr.ctypes.data_as(C.POINTER(C.c_int32))
        p.box = self.box.ctypes.data_as(C.POINTER(C.c_int32))
        p.theta = _dp(self.theta)
        for name in ("exp_alpha", "exp_nu", "dev_alpha", "dev_nu"):
            arr = getattr(p, name)
            for k, v in enumerate(getattr(f, name)):
                arr[k] = float(v)
        p.prior_phi = float(f.prior_phi)
        for k, v in enumerate(np.asarray(f.prior_r).reshape(-1)):
            p.prior_r[k] = float(v)
        for k, v in enumerate(np.asarray(f.prior_c).reshape(-1)):
            p.prior_c[k] = float(v)
        p.flags = int(f.flags if flags is None else flags)
        if p.flags & FLAG_MIX:
            for name, arr in (("mix_w", f.color_mix_w), ("mix_mean", f.color_mix_mean),
                              ("mix_cov", f.color_mix_cov)):
                dst = getattr(p, name)
                for k, v in enumerate(np.asarray(arr, np.float64).reshape(-1)):
                    dst[k] = float(v)
        self.n = 43 if p.flags & FLAG_MIX else 27
        self.p = p
        self.ref = C.byref(p)


def source_value(prob, s):
    """(pixel sum, -KL, sum |pixel terms|) of source s."""
    out = np.zeros(3)
    lib().oracle_source_value(prob.ref, s, _dp(out))
    return out


def source_elbo(prob, s):
    v = source_value(prob, s)
    return v[0] + v[1]


def n_params(prob):
    """Parameters of a source's ELBO: 27, or 43 with the colour-prior mixture."""
    return prob.n


def source_grad(prob, s):
    """Returns (value3, grad[n], gabs[n]) of source s (value3 as source_value; n =
    n_params)."""
    val = np.zeros(3)
    g = np.zeros(prob.n)
    ga = np.zeros(prob.n)
    lib().oracle_source_grad(prob.ref, s, _dp(val), _dp(g), _dp(ga))
    return val, g, ga


def source_hvp(prob, s, v):
    v = np.ascontiguousarray(np.asarray(v, np.float64)[:prob.n])
    hv = np.zeros(prob.n)
    ha = np.zeros(prob.n)
    lib().oracle_source_hvp(prob.ref, s, _dp(v), _dp(hv), _dp(ha))
    return hv, ha


def source_hessian(prob, s, with_abs=False):
    """n x n Hessian of ELBO_s (n = n_params; columns: Hessian-vector products along unit
    vectors, in parallel); with_abs also returns the per-entry sums of |per-visit terms|."""
    H = np.zeros((prob.n, prob.n))
    Ha = np.zeros((prob.n, prob.n))
    lib().oracle_source_hessian(prob.ref, s, _dp(H), _dp(Ha))
    return (H, Ha) if with_abs else H


def render(prob, f, n):
    H, W = int(f.img_H[n]), int(f.img_W[n])
    E = np.zeros((H, W))
    V = np.zeros((H, W))
    lib().oracle_render(prob.ref, n, _dp(E), _dp(V))
    return E, V


def source_light(prob, f, s, n):
    H, W = int(f.img_H[n]), int(f.img_W[n])
    E = np.zeros((H, W))
    V = np.zeros((H, W))
    lib().oracle_source_light(prob.ref, s, n, _dp(E), _dp(V))
    return E, V


def profiles(prob, s, n, px, py):
    out = np.zeros(2)
    lib().oracle_profiles(prob.ref, s, n, float(px), float(py), _dp(out))
    return out


def flux_moments(prob, s, a, b):
    out = np.zeros(2)
    lib().oracle_flux_moments(prob.ref, s, a, b, _dp(out))
    return out


def kl(prob, s):
    return lib().oracle_kl(prob.ref, s)


def total_elbo(prob):
    return lib().oracle_total_elbo(prob.ref)


def grad_many(prob, srcs):
    srcs = np.ascontiguousarray(srcs, np.int32)
    val = np.zeros((len(srcs), 3))
    g = np.zeros((len(srcs), prob.n))
    lib().oracle_grad_many(prob.ref, len(srcs), srcs.ctypes.data_as(C.POINTER(C.c_int32)),
                           _dp(val), _dp(g))
    return val, g
