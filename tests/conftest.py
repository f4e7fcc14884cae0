import copy
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def synth():
    from paper_1801_10277_amd import synth as s
    return s


@pytest.fixture(scope="session")
def O():
    from oracle import oracle as o
    o.build()
    return o


def clone(f):
    return copy.deepcopy(f)


def _boxes_meet(a, b):
    return (a[0] == b[0] and a[1] < b[1] + b[3] and b[1] < a[1] + a[3] and a[2] < b[2] + b[4]
            and b[2] < a[2] + a[4])


def neighbourhood(f, s, theta=None):
    """Source s with every source that has a box meeting one of s's boxes (same image), in
    their original order, over the same images: (sub-field, index of s in it).  Pixels of
    s's boxes see exactly these sources, so s's ELBO, gradient and Newton steps (others
    fixed) are those of the full field."""
    th = f.theta if theta is None else theta
    ptr = np.asarray(f.patch_ptr)
    mine = f.boxes[ptr[s]:ptr[s + 1]]
    keep = []
    for t in range(f.n_src):
        if t == s or any(_boxes_meet(a, b) for a in mine for b in f.boxes[ptr[t]:ptr[t + 1]]):
            keep.append(t)
    g = copy.copy(f)
    g.theta = np.ascontiguousarray(th[keep])
    g.boxes = np.ascontiguousarray(np.concatenate([f.boxes[ptr[t]:ptr[t + 1]] for t in keep]))
    counts = [ptr[t + 1] - ptr[t] for t in keep]
    g.patch_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    g.truth = {}
    return g, keep.index(s)


def single_source(synth, size=41, side=None, star=True, q=None, seed=3, psf_sigmas=None,
                  psf_weights=None, center=None, shape=None, sky=150.0, n_bands=1, band0=2,
                  r_var=0.01, c_var=0.01):
    """A one-source field built by hand: square image(s), box = whole image by default."""
    f = synth.tiny(S=1, n_bands=n_bands, size=size, side=size if side is None else side,
                   seed=seed)
    f.flags = synth.FLAG_INCLUDE_KL
    f.img_band = np.arange(band0, band0 + n_bands, dtype=np.int32) % 5
    f.img_sky[:] = sky
    if psf_sigmas is not None:
        f.img_psf[:, :, 3] = np.asarray(psf_sigmas) ** 2
        f.img_psf[:, :, 5] = np.asarray(psf_sigmas) ** 2
        f.img_psf[:, :, 4] = 0.0
        f.img_psf[:, :, 1:3] = 0.0
    if psf_weights is not None:
        f.img_psf[:, :, 0] = psf_weights
    c = (size - 1) / 2.0 if center is None else center
    f.theta[0, 0] = c
    f.theta[0, 1] = c
    if shape is not None:
        f.theta[0, 2:6] = shape
    if q is not None:
        f.theta[0, 6] = q
    for base in (7, 17):
        f.theta[0, base + 1] = r_var
        f.theta[0, base + 6:base + 10] = c_var
    if side is None:
        f.boxes = np.array([[n, 0, 0, size, size] for n in range(n_bands)], np.int32)
    else:
        cc = int(np.floor(c + 0.5))
        h = side // 2
        r0, r1 = max(cc - h, 0), min(cc + h + 1, size)
        f.boxes = np.array([[n, r0, r0, r1 - r0, r1 - r0] for n in range(n_bands)], np.int32)
    f.patch_ptr = np.array([0, n_bands], np.int32)
    return f
