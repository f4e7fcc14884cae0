"""The culling rule of the strip kernels, restated on the host and checked by brute force.

A work item covers strips start .. start + count - 1 of a box of width w (strip s: column
s mod w, rows L (s / w) .. L (s / w) + L - 1 clipped to the box height h).  The kernels
leave a Gaussian (centre c, precision P positive definite) out of the item when, on each
of the at most three rectangles its strips cover, x^2 det P / P_yy or y^2 det P / P_xx
exceeds 100 at the rectangle's offsets nearest the centre.  Minimising the quadratic form
over one coordinate gives both bounds, so a culled Gaussian's form exceeds 100 on every
pixel of the item; this test enumerates the pixels of random items and checks exactly
that, and that the rectangles cover every strip's pixels and nothing outside the box.
"""
import numpy as np
import pytest

CULL_Q = 100.0


def item_rectangles(start, count, w, h, L):
    """(c0, c1, r0, r1) inclusive, box-relative, as the kernels form them."""
    s0, s1 = start, start + count - 1
    rb0, rb1 = s0 // w, s1 // w
    band_end = lambda rb: min(rb * L + L, h) - 1
    rects = [(s0 - rb0 * w, w - 1 if rb1 > rb0 else s1 - rb0 * w, rb0 * L, band_end(rb0))]
    if rb1 > rb0:
        rects.append((0, s1 - rb1 * w, rb1 * L, band_end(rb1)))
        if rb1 > rb0 + 1:
            rects.append((0, w - 1, (rb0 + 1) * L, rb1 * L - 1))
    return rects


def culled(cx, cy, a, b, d, rects, bx, by):
    det = a * d - b * b
    if not (a > 0 and det > 0):
        return False
    m = np.inf
    for (ca, cb, ra, rb) in rects:
        x0, x1 = bx + ca - cx, bx + cb - cx
        y0, y1 = by + ra - cy, by + rb - cy
        ux, uy = max(x0, -x1, 0.0), max(y0, -y1, 0.0)
        m = min(m, max(ux * ux * det - CULL_Q * d, uy * uy * det - CULL_Q * a))
    return m > 0


def item_pixels(start, count, w, h, L):
    px = set()
    for s in range(start, start + count):
        rb, col = divmod(s, w)
        for r in range(rb * L, min(rb * L + L, h)):
            px.add((col, r))
    return px


@pytest.mark.parametrize("L", [4, 8, 16])
def test_rectangles_cover_exactly_the_item(L):
    rng = np.random.default_rng(L)
    for _ in range(300):
        w, h = int(rng.integers(1, 90)), int(rng.integers(1, 90))
        n = w * -(-h // L)
        start = int(rng.integers(0, n))
        count = int(rng.integers(1, min(n - start, 1024) + 1))
        want = item_pixels(start, count, w, h, L)
        got = set()
        for (ca, cb, ra, rb) in item_rectangles(start, count, w, h, L):
            assert 0 <= ca <= cb < w and 0 <= ra <= rb < h
            got |= {(c, r) for c in range(ca, cb + 1) for r in range(ra, rb + 1)}
        assert got == want


@pytest.mark.parametrize("L", [8, 16])
def test_culled_gaussians_stay_below_the_threshold_on_every_pixel(L):
    rng = np.random.default_rng(100 + L)
    n_culled = 0
    for _ in range(400):
        w, h = int(rng.integers(20, 100)), int(rng.integers(20, 100))
        bx, by = float(rng.integers(0, 500)), float(rng.integers(0, 500))
        n = w * -(-h // L)
        start = int(rng.integers(0, n))
        count = int(rng.integers(1, min(n - start, 64) + 1))
        rects = item_rectangles(start, count, w, h, L)
        pix = np.array(sorted(item_pixels(start, count, w, h, L)), float)
        X, Y = bx + pix[:, 0], by + pix[:, 1]
        for _ in range(8):
            # covariance with axis ratio down to 0.05 and scales 0.3 .. 12 px
            sig = rng.uniform(0.3, 12.0) * np.array([1.0, rng.uniform(0.05, 1.0)])
            th = rng.uniform(0, np.pi)
            R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
            P = np.linalg.inv(R @ np.diag(sig ** 2) @ R.T)
            a, b, d = P[0, 0], P[0, 1], P[1, 1]
            cx, cy = bx + rng.uniform(-40, w + 40), by + rng.uniform(-40, h + 40)
            if culled(cx, cy, a, b, d, rects, bx, by):
                n_culled += 1
                dx, dy = X - cx, Y - cy
                q = a * dx * dx + 2 * b * dx * dy + d * dy * dy
                assert q.min() > CULL_Q, (q.min(), cx, cy, a, b, d, rects)
    assert n_culled > 200   # the rule does fire on these draws


def test_non_positive_definite_is_never_culled():
    rects = [(0, 9, 0, 9)]
    assert not culled(1e4, 1e4, 1.0, 2.0, 1.0, rects, 0.0, 0.0)     # det < 0
    assert not culled(1e4, 1e4, -1.0, 0.0, -1.0, rects, 0.0, 0.0)   # negative definite
    assert culled(1e4, 1e4, 1.0, 0.0, 1.0, rects, 0.0, 0.0)
