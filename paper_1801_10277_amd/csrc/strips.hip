// Strip kernels: the batched render, the fused forward + adjoint and the per-visit
// background, all walking vertical strips of L pixels.
//
// Along a column the exponent of a Gaussian is a quadratic in the row offset, so the
// value at the next row is the current one times a ratio that itself shrinks by the
// constant factor exp(-P_yy) per row.  A lane therefore pays two exps per Gaussian per
// strip (value and first ratio at the strip's top row) and two multiplies per further
// row, instead of one exp per Gaussian per pixel; the result equals the direct
// evaluation up to a few ulps per row.  In the adjoint the per-row derivative terms are
// polynomials of degree <= 2 in the row offset, so each Gaussian contributes through
// three moments sum_k g_k, sum_k g_k k, sum_k g_k k^2 of its weighted values.
//
// Work item = a run of up to `chunk` strips of one box (strip s of a box of width w:
// column s mod w, rows L (s / w) ... L (s / w) + L - 1 clipped to the box).  Lane j of a
// wave takes strips start + j, start + j + 64, ...; consecutive lanes hold consecutive
// columns, so pixel loads of one row are contiguous.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "model.h"

namespace cel {

__device__ __forceinline__ double clamp_arg(double v) { return v < 700.0 ? v : 700.0; }
__device__ __forceinline__ dual clamp_arg(dual v) { return v.v < 700.0 ? v : mkd(700.0, 0.0); }

__device__ __forceinline__ void strip_geometry(const PairDev& p, int s, int L, int& c, int& r0, int& nrow) {
    const int rb = s / p.w;
    c = p.c0 + (s - rb * p.w);
    r0 = p.r0 + rb * L;
    nrow = min(L, p.h - rb * L);
}

// Value and first row ratio of component e at column px, top row py0.
template <class T>
__device__ __forceinline__ void strip_seed(const T* e, double px, double py0, T& n, T& rt, T& pdx0, T& pdy0,
                                           const double* __restrict__ t2) {
    const T dx = px - e[F_CX], dy = py0 - e[F_CY];
    pdx0 = e[F_PXX] * dx + e[F_PXY] * dy;
    pdy0 = e[F_PXY] * dx + e[F_PYY] * dy;
    n = fexp(e[F_LOGW] - 0.5 * (dx * pdx0 + dy * pdy0), t2);
    rt = fexp(clamp_arg(-(pdy0 + 0.5 * e[F_PYY])), t2);
}

// Pass A: star and galaxy profile values down the strip.
// SGN: also fgd[k] = sum of the de Vaucouleurs minus the exponential components (d fg /
// d frac_dev).
// live (with CULL): the components to evaluate (item_live); the others are skipped.
template <class T, int L, bool SGN = false, bool CULL = false>
__device__ __forceinline__ void strip_values(const T* __restrict__ tab, double px, double py0, T* fs, T* fg,
                                             const double* __restrict__ t2, T* fgd = nullptr,
                                             uint64_t live = ~0ull) {
    const T zero = scalar_traits<T>::make(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < L; ++k) fs[k] = fg[k] = zero;
    if constexpr (SGN) {
#pragma unroll
        for (int k = 0; k < L; ++k) fgd[k] = zero;
    }
#pragma unroll
    for (int c = 0; c < NPSF; ++c) {
        if (CULL && !((live >> c) & 1)) continue;
        const T* e = tab + c * CST;
        T n, rt, pdx0, pdy0;
        strip_seed(e, px, py0, n, rt, pdx0, pdy0, t2);
        const T rdy = e[F_RDY];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            fs[k] += n;
            if (k + 1 < L) {
                n = n * rt;
                rt = rt * rdy;
            }
        }
    }
#pragma unroll scalar_traits<T>::gal_unroll
    for (int c = NPSF; c < NCOMP; ++c) {
        if (CULL && !((live >> c) & 1)) continue;
        const T* e = tab + c * CST;
        T n, rt, pdx0, pdy0;
        strip_seed(e, px, py0, n, rt, pdx0, pdy0, t2);
        const T rdy = e[F_RDY], wt = e[F_WT];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            fg[k] += n * wt;
            if constexpr (SGN) fgd[k] += n * e[F_SGN];
            if (k + 1 < L) {
                n = n * rt;
                rt = rt * rdy;
            }
        }
    }
}

// Pass B: d/d(position, frac_dev, shape covariance) accumulated with per-row weights
// Gs (star) and Gg (galaxy).
template <class T, int L, bool CULL = false>
__device__ __forceinline__ void strip_adjoint(const T* __restrict__ tab, double px, double py0, const T* Gs,
                                              const T* Gg, T* acc, const double* __restrict__ t2,
                                              uint64_t live = ~0ull) {
    // Row moments by repeated running sums: with t_k = G_k value_k and u = L - k,
    //   A = sum t,  B = sum_k (sum_{i<=k} t_i) = sum t u,  C = sum_k (B after row k) = sum t u(u+1)/2,
    // so about the strip centre KC = (L-1)/2 (h = KC + 1 = (L+1)/2):
    //   m0 = sum t = A,  m1 = sum t (k-KC) = h A - B,  m2 = sum t (k-KC)^2 = h^2 A - (2h+1) B + 2C.
    // One fused multiply-add and two adds per row instead of a product and three accumulations.
    constexpr double KC = 0.5 * (L - 1);
    constexpr double H = KC + 1.0;
    const T zero = scalar_traits<T>::make(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NPSF; ++c) {
        if (CULL && !((live >> c) & 1)) continue;
        const T* e = tab + c * CST;
        T n, rt, pdx0, pdy0;
        strip_seed(e, px, py0, n, rt, pdx0, pdy0, t2);
        const T rdy = e[F_RDY];
        T A = zero, B = zero;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            A += Gs[k] * n;
            B += A;
            if (k + 1 < L) {
                n = n * rt;
                rt = rt * rdy;
            }
        }
        const T m0 = A, m1 = H * A - B;
        const T pdxc = pdx0 + e[F_PXY] * KC, pdyc = pdy0 + e[F_PYY] * KC;
        acc[A_UX] += pdxc * m0 + e[F_PXY] * m1;
        acc[A_UY] += pdyc * m0 + e[F_PYY] * m1;
    }
#pragma unroll scalar_traits<T>::gal_unroll
    for (int c = NPSF; c < NCOMP; ++c) {
        if (CULL && !((live >> c) & 1)) continue;
        const T* e = tab + c * CST;
        T n, rt, pdx0, pdy0;
        strip_seed(e, px, py0, n, rt, pdx0, pdy0, t2);
        const T rdy = e[F_RDY];
        T A = zero, B = zero, C = zero;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            A += Gg[k] * n;
            B += A;
            C += B;
            if (k + 1 < L) {
                n = n * rt;
                rt = rt * rdy;
            }
        }
        const T m0 = A, m1 = H * A - B, m2 = (H * H) * A - (2.0 * H + 1.0) * B + 2.0 * C;
        const T a = e[F_PXX], b = e[F_PXY], d = e[F_PYY];
        const T pdxc = pdx0 + b * KC, pdyc = pdy0 + d * KC;
        const T wt = e[F_WT], wnu = e[F_WNU];
        acc[A_FDEV] += e[F_SGN] * m0;
        acc[A_UX] += wt * (pdxc * m0 + b * m1);
        acc[A_UY] += wt * (pdyc * m0 + d * m1);
        acc[A_SXX] += wnu * ((pdxc * pdxc - a) * m0 + 2.0 * (pdxc * b) * m1 + (b * b) * m2);
        acc[A_SXY] += wnu * ((pdxc * pdyc - b) * m0 + (pdxc * d + pdyc * b) * m1 + (b * d) * m2);
        acc[A_SYY] += wnu * ((pdyc * pdyc - d) * m0 + 2.0 * (pdyc * d) * m1 + (d * d) * m2);
    }
}

// Pass B of the value-gradient adjoint from a box table staged in LDS.
// The star component and the 14 galaxy components of one PSF component share their centre
// (the source position plus that PSF component's offset), so the offsets dx = px - cx,
// dy = py0 - cy and their products are formed once per group and strip.  With
// P = [[a, b], [b, d]] and j = py0 + k - cy the row offset from the centre, a component's
// exponent is LW - (a dx^2 + 2 b dx dy + d dy^2) / 2 and its first row ratio
// exp(-(b dx + d dy) - d / 2), and every intermediate's contribution is a combination of
// the raw row moments M_i = sum_k t_k j^i (t_k = row weight x value).  With
// U = a dx M0 + b M1, U' = b dx M0 + d M1 (the sums of t (P (m - mu))_x and _y),
// W = a dx M1 + b M2 and W' = b dx M1 + d M2:
//   position:  wt U, wt U';    frac_dev: sgn M0;
//   shape xx:  wnu (a (dx U - M0) + b W),   xy: wnu (b (dx U - M0) + d W),
//   shape yy:  wnu (b dx U' + d (W' - M0)),
// (the sums of t ((P (m - mu))_x^2 - a), t ((P (m - mu))_x (P (m - mu))_y - b) and
// t ((P (m - mu))_y^2 - d)).  The moments come from the running sums A, B, C of the strip
// recurrence through the row-moment identity about a centre c with L - c = e = L + dy:
// M0 = A, M1 = e A - B, M2 = e^2 A - (2e + 1) B + 2C.  Per galaxy component this takes 29
// operations after the rows, against about 38 for the same fold about the strip centre with
// per-lane products of the precision, and the seed 6 instead of 12.
// Staged table: field-major, [NDF][NCP] (lane c writes component c's fields at stride NCP,
// no bank conflicts; every lane then reads the same words); stars at slots 0..2, galaxy
// group g at 4 + 14 g, so that the pairs of the unrolled galaxy loop are 16-byte aligned.
constexpr int NCP = 46;
enum DerivedField { D_CX = 0, D_CY, D_LW, D_RDY, D_A, D_B, D_D, D_WT, D_WNU, D_SGN, NDF };

__device__ __forceinline__ int staged_slot(int c) { return c < NPSF ? c : c + 1; }

// One wave writes the staged table of a box into its LDS slot (lane c: component c).  Lane
// NCOMP fills the spare slot NPSF with a component that is zero everywhere (log weight -1000,
// flat, every weight 0): the loops over the live components below pair an odd one with it.
__device__ __forceinline__ void stage_derived(const double* __restrict__ tab, double* my, int lane) {
    if (lane < NCOMP) {
        const double* e = tab + lane * CST;
        double* o = my + staged_slot(lane);
        o[D_CX * NCP] = e[F_CX];
        o[D_CY * NCP] = e[F_CY];
        o[D_LW * NCP] = e[F_LOGW];
        o[D_RDY * NCP] = e[F_RDY];
        o[D_A * NCP] = e[F_PXX];
        o[D_B * NCP] = e[F_PXY];
        o[D_D * NCP] = e[F_PYY];
        o[D_WT * NCP] = e[F_WT];
        o[D_WNU * NCP] = e[F_WNU];
        o[D_SGN * NCP] = e[F_SGN];
    } else if (lane == NCOMP) {
        double* o = my + NPSF;
        o[D_CX * NCP] = 0.0;
        o[D_CY * NCP] = 0.0;
        o[D_LW * NCP] = -1000.0;   // exp underflows to exactly 0
        o[D_RDY * NCP] = 1.0;
        o[D_A * NCP] = 0.0;
        o[D_B * NCP] = 0.0;
        o[D_D * NCP] = 0.0;
        o[D_WT * NCP] = 0.0;
        o[D_WNU * NCP] = 0.0;
        o[D_SGN * NCP] = 0.0;
    }
}

// Components that are negligible on every pixel of a work item are left out of its strips.
// The item's strips cover at most three rectangles of its box: the rest of its first band,
// whole bands, the start of its last band.  For P = [[a, b], [b, d]] positive definite,
// minimising the quadratic form over one coordinate gives
// (x, y) P (x, y)^T >= x^2 det P / d  and  >= y^2 det P / a,
// so a component whose form exceeds CULL_Q on each rectangle by one of these bounds stays
// below exp(-CULL_Q / 2) (< 2e-22) of its own peak on the whole item: far below the
// rounding of any pixel's expected count, which holds the sky.  Returns the live
// components as a wave-uniform bit set (bit c: table component c); lane c tests component c.
constexpr double CULL_Q = 100.0;

template <class T>
__device__ __forceinline__ uint64_t item_live(const T* __restrict__ tab, const PairDev& p, const Item& it, int L,
                                              int lane) {
    bool cull = false;
    if (lane < NCOMP) {
        const T* e = tab + lane * CST;
        const double cx = value_of(e[F_CX]), cy = value_of(e[F_CY]), a = value_of(e[F_PXX]),
                     b = value_of(e[F_PXY]), d = value_of(e[F_PYY]);
        const double det = fma(a, d, -(b * b));
        const double qa = CULL_Q * a, qd = CULL_Q * d;
        // > 0 if the form exceeds CULL_Q on columns ca..cb, rows ra..rb of the box
        auto far = [&](int ca, int cb, int ra, int rb) {
            const double x0 = (double)(p.c0 + ca) - cx, x1 = (double)(p.c0 + cb) - cx;
            const double y0 = (double)(p.r0 + ra) - cy, y1 = (double)(p.r0 + rb) - cy;
            const double ux = fmax(fmax(x0, -x1), 0.0), uy = fmax(fmax(y0, -y1), 0.0);
            return fmax(fma(ux * ux, det, -qd), fma(uy * uy, det, -qa));
        };
        const int s0 = it.start, s1 = it.start + it.count - 1;
        const int rb0 = s0 / p.w, rb1 = s1 / p.w;
        double m = far(s0 - rb0 * p.w, rb1 > rb0 ? p.w - 1 : s1 - rb0 * p.w, rb0 * L, min(rb0 * L + L, p.h) - 1);
        if (rb1 > rb0) {
            m = fmin(m, far(0, s1 - rb1 * p.w, rb1 * L, min(rb1 * L + L, p.h) - 1));
            if (rb1 > rb0 + 1) m = fmin(m, far(0, p.w - 1, (rb0 + 1) * L, rb1 * L - 1));
        }
        cull = a > 0.0 && det > 0.0 && m > 0.0 && cx - cx == 0.0 && cy - cy == 0.0;
    }
    return ~__builtin_amdgcn_ballot_w64(cull) & ((1ull << NCOMP) - 1);
}

// Staged slots of the live galaxy components of PSF group grp, two at a time (an odd last
// one paired with the zero component in slot NPSF).
template <class F>
__device__ __forceinline__ void for_live_pairs(uint64_t live, int grp, F&& f) {
    uint32_t gm = (uint32_t)(live >> (NPSF + grp * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1);
    const int base = NPSF + 1 + grp * NGAL_PER_PSF;
    while (gm) {
        const int s0 = base + __builtin_ctz(gm);
        gm &= gm - 1;
        int s1 = NPSF;
        if (gm) {
            s1 = base + __builtin_ctz(gm);
            gm &= gm - 1;
        }
        f(s0, s1);
    }
}

// One galaxy component's rows and fold (strip_adjoint_staged), in its PSF group's frame.
template <int L>
__device__ __forceinline__ void gal_adjoint_staged(const double* __restrict__ e, const double* Gg, double dx,
                                                   double h2x, double mxy, double h2y, double mdx, double mdyh,
                                                   double ev, double ev2, double e21, double* acc,
                                                   const double* __restrict__ t2) {
    const double a = e[D_A * NCP], b = e[D_B * NCP], d = e[D_D * NCP];
    double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, e[D_LW * NCP]))), t2);
    double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
    const double rdy = e[D_RDY * NCP];
    double A = 0.0, B = 0.0, C = 0.0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        A = fma(Gg[k], n, A);
        B += A;
        C += B;
        if (k + 1 < L) {
            n = n * rt;
            rt = rt * rdy;
        }
    }
    const double M1 = fma(ev, A, -B), M2 = fma(ev2, A, fma(-e21, B, C + C));
    const double X1 = dx * A, Y1 = dx * M1;
    const double U = fma(a, X1, b * M1), Up = fma(b, X1, d * M1);
    const double W = fma(a, Y1, b * M2), Wp = fma(b, Y1, d * M2);
    const double dU = fma(dx, U, -A), dUp = dx * Up, Wm = Wp - A;
    const double wt = e[D_WT * NCP], wnu = e[D_WNU * NCP];
    const double wna = wnu * a, wnb = wnu * b, wnd = wnu * d;
    acc[A_FDEV] = fma(e[D_SGN * NCP], A, acc[A_FDEV]);
    acc[A_UX] = fma(wt, U, acc[A_UX]);
    acc[A_UY] = fma(wt, Up, acc[A_UY]);
    acc[A_SXX] = fma(wna, dU, fma(wnb, W, acc[A_SXX]));
    acc[A_SXY] = fma(wnb, dU, fma(wnd, W, acc[A_SXY]));
    acc[A_SYY] = fma(wnb, dUp, fma(wnd, Wm, acc[A_SYY]));
}

// live: the components to evaluate (item_live); the others are skipped.
template <int L>
__device__ __forceinline__ void strip_adjoint_staged(const double* __restrict__ lt, double px, double py0,
                                                     const double* Gs, const double* Gg, double* acc,
                                                     const double* __restrict__ t2, uint64_t live) {
#pragma unroll 1
    for (int grp = 0; grp < NPSF; ++grp) {
        const bool star = (live >> grp) & 1;
        if (!star && !((live >> (NPSF + grp * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1))) continue;
        const double* es = lt + grp;
        const double dx = px - es[D_CX * NCP], dy = py0 - es[D_CY * NCP];
        const double h2x = -0.5 * (dx * dx), mxy = -(dx * dy), h2y = -0.5 * (dy * dy);
        const double mdx = -dx, mdyh = -(dy + 0.5);
        const double ev = (double)L + dy;
        const double ev2 = ev * ev, e21 = 2.0 * ev + 1.0;
        if (star) {
            const double a = es[D_A * NCP], b = es[D_B * NCP], d = es[D_D * NCP];
            double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, es[D_LW * NCP]))), t2);
            double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
            const double rdy = es[D_RDY * NCP];
            double A = 0.0, B = 0.0;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                A = fma(Gs[k], n, A);
                B += A;
                if (k + 1 < L) {
                    n = n * rt;
                    rt = rt * rdy;
                }
            }
            const double M1 = fma(ev, A, -B), X1 = dx * A;
            acc[A_UX] = fma(a, X1, fma(b, M1, acc[A_UX]));
            acc[A_UY] = fma(b, X1, fma(d, M1, acc[A_UY]));
        }
        for_live_pairs(live, grp, [&](int s0, int s1) {
            gal_adjoint_staged<L>(lt + s0, Gg, dx, h2x, mxy, h2y, mdx, mdyh, ev, ev2, e21, acc, t2);
            gal_adjoint_staged<L>(lt + s1, Gg, dx, h2x, mxy, h2y, mdx, mdyh, ev, ev2, e21, acc, t2);
        });
    }
}

// Pass A of the render's strip pass from the box table staged in LDS (strip_adjoint_staged's
// layout): star and galaxy profile values down the strip, the offsets from each PSF group's
// shared centre formed once per group.
// SGN: also fgd[k] = sum of the de Vaucouleurs minus the exponential components (d fg /
// d frac_dev).
template <int L, bool SGN>
__device__ __forceinline__ void gal_values_staged(const double* __restrict__ e, double h2x, double mxy, double h2y,
                                                  double mdx, double mdyh, double* fg, double* fgd,
                                                  const double* __restrict__ t2) {
    const double a = e[D_A * NCP], b = e[D_B * NCP], d = e[D_D * NCP];
    double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, e[D_LW * NCP]))), t2);
    double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
    const double rdy = e[D_RDY * NCP], wt = e[D_WT * NCP];
    const double sgn = SGN ? e[D_SGN * NCP] : 0.0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        fg[k] = fma(n, wt, fg[k]);
        if constexpr (SGN) fgd[k] = fma(n, sgn, fgd[k]);
        if (k + 1 < L) {
            n = n * rt;
            rt = rt * rdy;
        }
    }
}

template <int L, bool SGN = false>
__device__ __forceinline__ void strip_values_staged(const double* __restrict__ lt, double px, double py0,
                                                    double* fs, double* fg, const double* __restrict__ t2,
                                                    uint64_t live, double* fgd = nullptr) {
#pragma unroll
    for (int k = 0; k < L; ++k) fs[k] = fg[k] = 0.0;
    if constexpr (SGN) {
#pragma unroll
        for (int k = 0; k < L; ++k) fgd[k] = 0.0;
    }
#pragma unroll 1
    for (int grp = 0; grp < NPSF; ++grp) {
        const bool star = (live >> grp) & 1;
        if (!star && !((live >> (NPSF + grp * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1))) continue;
        const double* es = lt + grp;
        const double dx = px - es[D_CX * NCP], dy = py0 - es[D_CY * NCP];
        const double h2x = -0.5 * (dx * dx), mxy = -(dx * dy), h2y = -0.5 * (dy * dy);
        const double mdx = -dx, mdyh = -(dy + 0.5);
        if (star) {
            const double a = es[D_A * NCP], b = es[D_B * NCP], d = es[D_D * NCP];
            double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, es[D_LW * NCP]))), t2);
            double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
            const double rdy = es[D_RDY * NCP];
#pragma unroll
            for (int k = 0; k < L; ++k) {
                fs[k] += n;
                if (k + 1 < L) {
                    n = n * rt;
                    rt = rt * rdy;
                }
            }
        }
        for_live_pairs(live, grp, [&](int s0, int s1) {
            gal_values_staged<L, SGN>(lt + s0, h2x, mxy, h2y, mdx, mdyh, fg, fgd, t2);
            gal_values_staged<L, SGN>(lt + s1, h2x, mxy, h2y, mdx, mdyh, fg, fgd, t2);
        });
    }
}

// Pixel term of one row: accumulates the value and d/dk1..k4 and returns the row
// weights d l / d f_star and d l / d f_gal.
// (The -log(x!) constant is not added here: each box's sum of it is precomputed once.)
template <class T, bool DERIV>
__device__ __forceinline__ void strip_pixel(double x, T E, T V, T fs, T fg, const T* k, T* acc, T& Gs, T& Gg,
                                            const double2* __restrict__ tl) {
    const T Es = k[C_K1] * fs + k[C_K2] * fg;
    const T inv = frcp(E);
    const T r = V * inv * inv;
    acc[A_VAL] += x * (flog(E, tl) - 0.5 * r) - E;
    if (DERIV) {
        const T lE = x * inv * (1.0 + r) - 1.0;
        const T lV = -0.5 * x * (inv * inv);
        const T A = lE - 2.0 * Es * lV;
        acc[A_K1] += A * fs;
        acc[A_K2] += A * fg;
        acc[A_K3] += lV * (fs * fs);
        acc[A_K4] += lV * (fg * fg);
        Gs = A * k[C_K1] + 2.0 * lV * (k[C_K3] * fs);
        Gg = A * k[C_K2] + 2.0 * lV * (k[C_K4] * fg);
    }
}

// Second derivatives of one pixel term in the box's brightness factors k1..k4, added into
// h[NKK]: with l_EE = -x/E^2 - 3xV/E^4, l_EV = x/E^3, l_V = -x/(2E^2) (l_VV = 0), dE/dk =
// (fs, fg, 0, 0) and dV/dk = (-2 Es fs, -2 Es fg, fs^2, fg^2), d2V/dk1dk1 = -2 fs^2,
// d2V/dk1dk2 = -2 fs fg, d2V/dk2dk2 = -2 fg^2:
// h_ij = l_EE E_i E_j + l_EV (E_i V_j + V_i E_j) + l_V V_ij.
// frac_dev f enters only through the galaxy profile, fg = f fgd_dev + (1 - f) fg_exp, so
// dfg/df = fgd (the dev minus the exp profile) and, with E_f = k2 fgd,
// V_f = 2 fgd (k4 fg - Es k2), V_ff = 2 fgd^2 (k4 - k2^2), V_f1 = -2 fs k2 fgd,
// V_f2 = -2 (fg k2 + Es) fgd, V_f4 = 2 fg fgd, E_f2 = fgd:
// h_fi = l_EE E_f E_i + l_EV (E_f V_i + V_f E_i) + l_V V_fi + l_E E_fi.
__device__ __forceinline__ void pixel_kk(double x, double E, double V, double fs, double fg, double fgd,
                                         const double* k, double* h) {
    const double inv = frcp(E);
    const double inv2 = inv * inv;
    const double r = V * inv2;
    const double lE = x * inv * (1.0 + r) - 1.0;
    const double lEE = -x * inv2 * (1.0 + 3.0 * r);
    const double lEV = x * inv2 * inv;
    const double lV = -0.5 * x * inv2;
    const double Es = k[C_K1] * fs + k[C_K2] * fg;
    const double Q = lEE - 4.0 * lEV * Es - 2.0 * lV;
    const double a = lEV * fs, b = lEV * fg;
    h[KK_11] += Q * (fs * fs);
    h[KK_12] += Q * (fs * fg);
    h[KK_22] += Q * (fg * fg);
    h[KK_13] += a * (fs * fs);
    h[KK_14] += a * (fg * fg);
    h[KK_23] += b * (fs * fs);
    h[KK_24] += b * (fg * fg);
    const double Ef = k[C_K2] * fgd;
    const double Vf = 2.0 * fgd * (k[C_K4] * fg - Es * k[C_K2]);
    h[KK_F1] += lEE * (Ef * fs) + lEV * (Ef * (-2.0 * Es * fs) + Vf * fs) + lV * (-2.0 * fs * k[C_K2] * fgd);
    h[KK_F2] += lEE * (Ef * fg) + lEV * (Ef * (-2.0 * Es * fg) + Vf * fg) +
                lV * (-2.0 * (fg * k[C_K2] + Es) * fgd) + lE * fgd;
    h[KK_F3] += lEV * Ef * (fs * fs);
    h[KK_F4] += lEV * Ef * (fg * fg) + lV * (2.0 * fg * fgd);
    h[KK_FF] += lEE * (Ef * Ef) + 2.0 * lEV * (Ef * Vf) + lV * (2.0 * fgd * fgd * (k[C_K4] - k[C_K2] * k[C_K2]));
}

// Sky plus the light of every other box of the image that covers each row of the strip.
template <int L>
__device__ __forceinline__ void strip_background(const PairDev& p, const PairDev* __restrict__ pairs,
                                                 const int32_t* __restrict__ nbr, const double* __restrict__ tabv,
                                                 const double* __restrict__ coefv, const celeste_image& im, int c,
                                                 int r0, double* Eb, double* Vb, const double* __restrict__ t2) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
        Eb[k] = r0 + k < im.H ? sky_at(im, r0 + k, c) : im.sky;
        Vb[k] = 0.0;
    }
    for (int q = p.nbr_begin; q < p.nbr_end; ++q) {
        const int pi = __builtin_amdgcn_readfirstlane(nbr[q]);
        const PairDev o = pairs[pi];
        if (c < o.c0 || c >= o.c0 + o.w || r0 + L <= o.r0 || r0 >= o.r0 + o.h) continue;
        double fs[L], fg[L];
        strip_values<double, L>(tabv + (size_t)pi * NCOMP * CST, (double)c, (double)r0, fs, fg, t2);
        const double* kk = coefv + (size_t)pi * NCOEF;
        const double k1 = kk[C_K1], k2 = kk[C_K2], k3 = kk[C_K3], k4 = kk[C_K4];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int r = r0 + k;
            if (r < o.r0 || r >= o.r0 + o.h) continue;
            const double Et = k1 * fs[k] + k2 * fg[k];
            Eb[k] += Et;
            Vb[k] += k3 * fs[k] * fs[k] + k4 * fg[k] * fg[k] - Et * Et;
        }
    }
}

// Sky plus the light of every other box of the image covering each row of the strip, from
// the boxes' stored own profile values (ascending box order).
template <int L>
__device__ __forceinline__ void strip_background_fg(const PairDev& p, const PairDev* __restrict__ pairs,
                                                    const int32_t* __restrict__ nbr,
                                                    const double* __restrict__ coefv,
                                                    const double* __restrict__ fgm, const celeste_image& im, int c, int r0,
                                                    double* Eb, double* Vb) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
        Eb[k] = r0 + k < im.H ? sky_at(im, r0 + k, c) : im.sky;
        Vb[k] = 0.0;
    }
    for (int q = p.nbr_begin; q < p.nbr_end; ++q) {
        const int pi = __builtin_amdgcn_readfirstlane(nbr[q]);
        const PairDev o = pairs[pi];
        if (c < o.c0 || c >= o.c0 + o.w || r0 + L <= o.r0 || r0 >= o.r0 + o.h) continue;
        const double* kk = coefv + (size_t)pi * NCOEF;
        const double k1 = kk[C_K1], k2 = kk[C_K2], k3 = kk[C_K3], k4 = kk[C_K4];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int r = r0 + k;
            if (r < o.r0 || r >= o.r0 + o.h) continue;
            const size_t vi = (size_t)o.visit_off + (size_t)(r - o.r0) * o.w + (c - o.c0);
            const double fs = fgm[2 * vi], fg = fgm[2 * vi + 1];
            const double Et = k1 * fs + k2 * fg;
            Eb[k] += Et;
            Vb[k] += k3 * fs * fs + k4 * fg * fg - Et * Et;
        }
    }
}

// The next item of the dynamic queue for the whole wave (called with every lane active, so
// the first active lane is lane 0); wave-uniform, so the item loop stays scalar.
__device__ inline int next_item_s(int* counter, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(counter, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

// ----------------------------------------------------------------------- planes
__global__ void __launch_bounds__(256) k_fill_planes(const celeste_image* __restrict__ images,
                                                     double* __restrict__ E, double* __restrict__ V,
                                                     const int* status) {
    if (*status) return;
    const celeste_image& im = images[blockIdx.y];
    const int64_t npix = (int64_t)im.H * im.W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
        E[im.pix_offset + i] = im.sky_map ? im.sky_map[i] : im.sky;
        V[im.pix_offset + i] = 0.0;
    }
}

// Adds the light of the boxes of one conflict-free class to the planes (no two boxes of a
// class share a pixel, so the read-modify-write needs no atomics; classes run in order).
template <int L>
__global__ void __launch_bounds__(256) k_render_strips(Sel sel, const Item* __restrict__ items,
                                                       const PairDev* __restrict__ pairs,
                                                       const celeste_image* __restrict__ images,
                                                       const double* __restrict__ tab,
                                                       const double* __restrict__ coef, double* __restrict__ E,
                                                       double* __restrict__ V, const int* status) {
    if (*status) return;
    __shared__ double t2[EXP_TAB];
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int j = blockIdx.x * wpb + (threadIdx.x >> 6); j < sel.n; j += nw) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(sel, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        const celeste_image& im = images[p.img];
        const double* tb = tab + (size_t)it.pair * NCOMP * CST;
        const double* kp = coef + (size_t)it.pair * NCOEF;
        const double k1 = kp[C_K1], k2 = kp[C_K2], k3 = kp[C_K3], k4 = kp[C_K4];
        for (int q = lane; q < it.count; q += 64) {
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            double fs[L], fg[L];
            strip_values<double, L>(tb, (double)c, (double)r0, fs, fg, t2);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k >= nrow) break;
                const size_t gi = (size_t)im.pix_offset + (size_t)(r0 + k) * im.W + c;
                const double Et = k1 * fs[k] + k2 * fg[k];
                E[gi] += Et;
                V[gi] += k3 * fs[k] * fs[k] + k4 * fg[k] * fg[k] - Et * Et;
            }
        }
    }
}

// ----------------------------------------------------------------------- adjoint
// KK (double gradient passes over planes, stored backgrounds or stored values only): also
// the brightness-factor block of each box's intermediate Hessian, per item into a.kk.
// At least two waves per SIMD: the dual-number variants would otherwise take 256 VGPRs
// plus accumulation registers and run one wave per SIMD; with the bound they spill a few
// hundred bytes per lane and run 17% faster (the value variants fit without spilling).
// Three for the value-gradient pass over stored own values (the hot path): it needs 191
// VGPRs unbounded and 168 with the bound (two registers spilled).
template <class T, int BASE, bool DERIV, int L, bool FGM, bool KK>
__global__ void __launch_bounds__(256, (FGM && DERIV && std::is_same<T, double>::value) ? 3 : 2) k_adjoint_strips(AdjArgs a, const Item* __restrict__ items,
                                                        const PairDev* __restrict__ pairs,
                                                        const celeste_image* __restrict__ images,
                                                        const int32_t* __restrict__ nbr,
                                                        const double* __restrict__ xs, const double* __restrict__ Ep,
                                                        const double* __restrict__ Vp, const double* __restrict__ bg,
                                                        const double* __restrict__ tabp,
                                                        const double* __restrict__ coefp,
                                                        const double* __restrict__ tabv,
                                                        const double* __restrict__ coefv,
                                                        const uint8_t* __restrict__ active,
                                                        const double* __restrict__ fgm,
                                                        double* __restrict__ partials) {
    if (*a.status) return;
    __shared__ double t2[EXP_TAB];
    __shared__ double2 tl[128];
    // The value-gradient pass over stored own values (the hot path) reads each box's table
    // from LDS, staged by the wave at the start of each item in the derived form of
    // strip_adjoint_staged: the per-component loads of the galaxy loop then wait on LDS
    // instead of missing the scalar cache (38% of the scalar loads missed with the table read
    // from global memory), the table leaves the scalar registers (no spills), and the
    // coefficients every lane shares are formed once per box instead of once per strip.
    constexpr bool LDS_TAB = DERIV && std::is_same<T, double>::value &&
                             (FGM ? (BASE == BASE_PLANES || BASE == BASE_FG) : (BASE == BASE_PLANES || BASE == BASE_BG));
    extern __shared__ double ltab[];   // LDS_TAB: [waves per block][NDF][NCP], sized at launch
    fill_log_table(tl);
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const T zero = scalar_traits<T>::make(0.0, 0.0);
    int j = a.dynamic ? next_item_s(a.counter, lane) : blockIdx.x * wpb + (threadIdx.x >> 6);
    while (j < a.items.n) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        if (!active || active[p.src]) {
            const celeste_image& im = images[p.img];
            const T* tab = reinterpret_cast<const T*>(tabp) + (size_t)it.pair * NCOMP * CST;
            // dual passes (HVP, Hessian tangents) read the table directly; they cull too
            constexpr bool CULL_T = !LDS_TAB && std::is_same<T, dual>::value;
            uint64_t live = 0;
            if constexpr (CULL_T) live = item_live(tab, p, it, L, lane);
            if constexpr (LDS_TAB) {
                // the wave's previous item has finished reading its copy (in-order LDS)
                double* my = ltab + (threadIdx.x >> 6) * (NCP * NDF);
                __builtin_amdgcn_wave_barrier();
                stage_derived(reinterpret_cast<const double*>(tab), my, lane);
                live = item_live(reinterpret_cast<const double*>(tab), p, it, L, lane);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            const T* kp = reinterpret_cast<const T*>(coefp) + (size_t)it.pair * NCOEF;
            const T k[NCOEF] = {kp[0], kp[1], kp[2], kp[3]};
            T acc[NACC];
#pragma unroll
            for (int f = 0; f < NACC; ++f) acc[f] = zero;
            double kh[NKK_USED];
#pragma unroll
            for (int f = 0; f < NKK_USED; ++f) kh[f] = 0.0;
            for (int q = lane; q < it.count; q += 64) {
                int c, r0, nrow;
                strip_geometry(p, it.start + q, L, c, r0, nrow);
                const double px = (double)c, py0 = (double)r0;
                if constexpr (FGM && DERIV && (BASE == BASE_PLANES || BASE == BASE_FG)) {
                    // Rows streamed one at a time, the next row's loads in flight, so that only
                    // the row weights (and for BASE_FG the neighbours' background) stay live
                    // into pass B.
                    double Eb[L], Vb[L];
                    if constexpr (BASE == BASE_FG)
                        strip_background_fg<L>(p, pairs, nbr, coefv, fgm, im, c, r0, Eb, Vb);
                    // Row addresses as 32-bit byte offsets from wave-uniform bases (the image's
                    // planes, the box's stored values; plan creation bounds images below 2^29
                    // pixels and boxes below 2^28 visits): one add and one select per row.
                    const char* xb = reinterpret_cast<const char*>(xs + im.pix_offset);
                    const char* eb = reinterpret_cast<const char*>(Ep + im.pix_offset);
                    const char* vb = reinterpret_cast<const char*>(Vp + im.pix_offset);
                    const char* fb = reinterpret_cast<const char*>(fgm + 2 * p.visit_off);
                    const uint32_t W8 = (uint32_t)im.W * 8u, w16 = (uint32_t)p.w * 16u;
                    const uint32_t go = (uint32_t)(r0 * im.W + c) * 8u;
                    const uint32_t vo = (uint32_t)((r0 - p.r0) * p.w + (c - p.c0)) * 16u;
                    // row rr of the strip if `in`, else its top row (a row past the box)
                    auto row_load = [&](int rr, bool in, double& x_, double& e_, double& v_, double& s_,
                                        double& g_) {
                        const uint32_t gr = go + (in ? (uint32_t)rr * W8 : 0u);
                        const uint32_t vr = vo + (in ? (uint32_t)rr * w16 : 0u);
                        x_ = *reinterpret_cast<const double*>(xb + gr);
                        if constexpr (BASE == BASE_PLANES) {
                            e_ = *reinterpret_cast<const double*>(eb + gr);
                            v_ = *reinterpret_cast<const double*>(vb + gr);
                        }
                        const double2 sg = *reinterpret_cast<const double2*>(fb + vr);
                        s_ = sg.x;
                        g_ = sg.y;
                    };
                    T Gs[L], Gg[L];
                    double cx_, ce_ = 0.0, cv_ = 0.0, cs_, cg_;
                    row_load(0, true, cx_, ce_, cv_, cs_, cg_);
#pragma unroll
                    for (int kk = 0; kk < L; ++kk) {
                        double nx_ = 0.0, ne_ = 0.0, nv_ = 0.0, ns_ = 0.0, ng_ = 0.0;
                        if (kk + 1 < L) row_load(kk + 1, kk + 1 < nrow, nx_, ne_, nv_, ns_, ng_);
                        T gs = zero, gg = zero;
                        if (kk < nrow && cx_ == cx_) {
                            const T fsk = scalar_traits<T>::make(cs_, 0.0), fgk = scalar_traits<T>::make(cg_, 0.0);
                            T E, V;
                            if constexpr (BASE == BASE_PLANES) {
                                E = scalar_traits<T>::make(ce_, 0.0);
                                V = scalar_traits<T>::make(cv_, 0.0);
                            } else {
                                const T Es = k[C_K1] * fsk + k[C_K2] * fgk;
                                const T Vs = k[C_K3] * (fsk * fsk) + k[C_K4] * (fgk * fgk) - Es * Es;
                                E = Eb[kk] + Es;
                                V = Vb[kk] + Vs;
                            }
                            strip_pixel<T, true>(cx_, E, V, fsk, fgk, k, acc, gs, gg, tl);
                        }
                        Gs[kk] = gs;
                        Gg[kk] = gg;
                        cx_ = nx_;
                        ce_ = ne_;
                        cv_ = nv_;
                        cs_ = ns_;
                        cg_ = ng_;
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (LDS_TAB)
                        strip_adjoint_staged<L>(ltab + (threadIdx.x >> 6) * (NCP * NDF), px, py0, Gs, Gg,
                                                acc, t2, live);
                    else
                        strip_adjoint<T, L>(tab, px, py0, Gs, Gg, acc, t2);
                    continue;
                }
                if constexpr (DERIV && !FGM && (BASE == BASE_PLANES || BASE == BASE_BG)) {
                    // Own values from pass A, then the pixel rows streamed as above.
                    T fs[L], fg[L], fgd[KK ? L : 1];
                    if constexpr (LDS_TAB)
                        strip_values_staged<L, KK>(ltab + (threadIdx.x >> 6) * (NCP * NDF), px, py0, fs, fg, t2,
                                                   live, fgd);
                    else
                        strip_values<T, L, KK, CULL_T>(tab, px, py0, fs, fg, t2, fgd, live);
                    const double* xs_i = xs + im.pix_offset;
                    auto row_load = [&](int rr, double& x_, double& e_, double& v_) {
                        const size_t gi = (size_t)(r0 + rr) * im.W + c;
                        x_ = xs_i[gi];
                        if constexpr (BASE == BASE_PLANES) {
                            e_ = Ep[im.pix_offset + gi];
                            v_ = Vp[im.pix_offset + gi];
                        } else {
                            const size_t vi = (size_t)p.visit_off + (size_t)(r0 + rr - p.r0) * p.w + (c - p.c0);
                            e_ = bg[2 * vi];
                            v_ = bg[2 * vi + 1];
                        }
                    };
                    double cx_, ce_, cv_;
                    row_load(0, cx_, ce_, cv_);
#pragma unroll
                    for (int kk = 0; kk < L; ++kk) {
                        double nx_ = 0.0, ne_ = 0.0, nv_ = 0.0;
                        if (kk + 1 < L) row_load(kk + 1 < nrow ? kk + 1 : 0, nx_, ne_, nv_);
                        T gs = zero, gg = zero;
                        if constexpr (KK) {
                            // own values for the closed-form Hessian pass that follows
                            if (a.fg_out && kk < nrow) {
                                const size_t vi = (size_t)p.visit_off + (size_t)(r0 + kk - p.r0) * p.w + (c - p.c0);
                                a.fg_out[2 * vi] = fs[kk];
                                a.fg_out[2 * vi + 1] = fg[kk];
                            }
                        }
                        if (kk < nrow && cx_ == cx_) {
                            const T Es = k[C_K1] * fs[kk] + k[C_K2] * fg[kk];
                            const T Vs = k[C_K3] * (fs[kk] * fs[kk]) + k[C_K4] * (fg[kk] * fg[kk]) - Es * Es;
                            T E, V;
                            if constexpr (BASE == BASE_PLANES) {
                                E = value_with_tangent(ce_, Es);
                                V = value_with_tangent(cv_, Vs);
                            } else {
                                E = ce_ + Es;
                                V = cv_ + Vs;
                            }
                            strip_pixel<T, true>(cx_, E, V, fs[kk], fg[kk], k, acc, gs, gg, tl);
                            if constexpr (KK) pixel_kk(cx_, E, V, fs[kk], fg[kk], fgd[kk], k, kh);
                        }
                        fs[kk] = gs;
                        fg[kk] = gg;
                        cx_ = nx_;
                        ce_ = ne_;
                        cv_ = nv_;
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (LDS_TAB)
                        strip_adjoint_staged<L>(ltab + (threadIdx.x >> 6) * (NCP * NDF), px, py0, fs, fg, acc, t2,
                                                live);
                    else
                        strip_adjoint<T, L, CULL_T>(tab, px, py0, fs, fg, acc, t2, live);
                    continue;
                }
                double x[L], Eb[L], Vb[L];
                if (BASE == BASE_NBR) {
                    strip_background<L>(p, pairs, nbr, tabv, coefv, im, c, r0, Eb, Vb, t2);
                } else if (BASE == BASE_FG) {
                    strip_background_fg<L>(p, pairs, nbr, coefv, fgm, im, c, r0, Eb, Vb);
                }
#pragma unroll
                for (int kk = 0; kk < L; ++kk) {
                    const int rr = kk < nrow ? kk : 0;   // rows past the box reuse row 0 (masked below)
                    const size_t gi = (size_t)im.pix_offset + (size_t)(r0 + rr) * im.W + c;
                    x[kk] = kk < nrow ? xs[gi] : __builtin_nan("");
                    if (BASE == BASE_PLANES) {
                        Eb[kk] = Ep[gi];
                        Vb[kk] = Vp[gi];
                    } else if (BASE == BASE_BG) {
                        const size_t vi = (size_t)p.visit_off + (size_t)(r0 + rr - p.r0) * p.w + (c - p.c0);
                        Eb[kk] = bg[2 * vi];
                        Vb[kk] = bg[2 * vi + 1];
                    }
                }
                if (BASE == BASE_PLANES && !DERIV) {
                    // value only: the planes already hold the totals
#pragma unroll
                    for (int kk = 0; kk < L; ++kk) {
                        if (!(x[kk] == x[kk])) continue;
                        T gs, gg;
                        strip_pixel<T, false>(x[kk], scalar_traits<T>::make(Eb[kk], 0.0),
                                              scalar_traits<T>::make(Vb[kk], 0.0), zero, zero, k, acc, gs, gg, tl);
                    }
                    continue;
                }
                T fs[L], fg[L];
                if (FGM) {
                    // own profile values stored by the render's strip pass
#pragma unroll
                    for (int kk = 0; kk < L; ++kk) {
                        const int rr = kk < nrow ? kk : 0;
                        const size_t vi = (size_t)p.visit_off + (size_t)(r0 + rr - p.r0) * p.w + (c - p.c0);
                        fs[kk] = scalar_traits<T>::make(fgm[2 * vi], 0.0);
                        fg[kk] = scalar_traits<T>::make(fgm[2 * vi + 1], 0.0);
                    }
                } else {
                    strip_values<T, L>(tab, px, py0, fs, fg, t2);
                }
                // fs, fg become the row weights of pass B
#pragma unroll
                for (int kk = 0; kk < L; ++kk) {
                    T gs = zero, gg = zero;
                    if (x[kk] == x[kk]) {
                        const T Es = k[C_K1] * fs[kk] + k[C_K2] * fg[kk];
                        const T Vs = k[C_K3] * (fs[kk] * fs[kk]) + k[C_K4] * (fg[kk] * fg[kk]) - Es * Es;
                        T E, V;
                        if (BASE == BASE_PLANES) {
                            E = value_with_tangent(Eb[kk], Es);
                            V = value_with_tangent(Vb[kk], Vs);
                        } else {
                            E = Eb[kk] + Es;
                            V = Vb[kk] + Vs;
                        }
                        strip_pixel<T, DERIV>(x[kk], E, V, fs[kk], fg[kk], k, acc, gs, gg, tl);
                    }
                    fs[kk] = gs;
                    fg[kk] = gg;
                    // one row at a time: interleaving the rows' log/division chains would
                    // multiply the live registers without adding useful parallelism
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (DERIV) strip_adjoint<T, L>(tab, px, py0, fs, fg, acc, t2);
            }
            T* out = reinterpret_cast<T*>(partials) + (size_t)ii * NACC;
#pragma unroll
            for (int f = 0; f < NACC; ++f) {
                const T s = wave_sum(acc[f]);
                if (lane == 0) out[f] = s;
            }
            if constexpr (KK) {
#pragma unroll
                for (int f = 0; f < NKK_USED; ++f) {
                    const double s = wave_sum(kh[f]);
                    if (lane == 0) a.kk[(size_t)ii * NKK + f] = s;
                }
            }
        }
        j = a.dynamic ? next_item_s(a.counter, lane) : j + nw;
    }
}

// ------------------------------------------------- closed-form geometric Hessian block
// Second derivatives of a box's pixel sum in its position, frac_dev and shape intermediates
// (the exact Hessians of Section IV-D), evaluated pixel by pixel in closed form.  For a
// component n = w N(m; mu, C) with z = P (m - mu), P = C^-1 = [[a, b], [b, d]] and
// D_ij = z_i z_j - P_ij, and with the operators d/du_i (position) and s_ij = c_ij d/dS_ij
// (c = 2 on the diagonal: the accumulator scaling of the gradient pass) on a galaxy
// component of covariance C = nu S + PSF:
//   d n/du_i = n z_i,                 d2 n/du_i du_j = n D_ij,
//   s_ij n = nu n D_ij,               d/du_i s_kl n = nu n (z_i D_kl - P_ki z_l - P_li z_k),
//   s_ij s_kl n = nu^2 n (D_ij D_kl - T_ij,kl),
// where, from s_ij z = -nu P E_ij z and s_ij P = -nu P E_ij P (E_xx = 2 e_x e_x^T,
// E_xy = e_x e_y^T + e_y e_x^T, E_yy = 2 e_y e_y^T), T_ij,kl is y_k z_l + z_k y_l - Q_kl with
// y = P E_ij z and Q = P E_ij P, linear in D:
//   T_xx,xx = 4a Dxx + 2a^2,  T_xx,xy = 2a Dxy + 2b Dxx + 2ab,  T_xx,yy = 4b Dxy + 2b^2,
//   T_xy,xy = a Dyy + 2b Dxy + d Dxx + ad + b^2,  T_xy,yy = 2b Dyy + 2d Dxy + 2bd,
//   T_yy,yy = 4d Dyy + 2d^2.
// frac_dev enters the galaxy profile linearly (weight +1 de Vaucouleurs, -1 exponential).
// With the pixel term l(E, V), E = Eb + k1 fs + k2 fg, V = Vb + k3 fs^2 + k4 fg^2 - Es^2
// (Es = k1 fs + k2 fg), l_VV = 0 and the row weights Gs, Gg of the gradient pass, the entry
// between geometric intermediates g, h is
//   (l_EE - 2 l_V) E_g E_h + l_EV (E_g V_h + V_g E_h) + 2 l_V (k3 fs_g fs_h + k4 fg_g fg_h)
//   + Gs fs_gh + Gg fg_gh,
// and the entry between g and k_i follows from dE/dk = (fs, fg, 0, 0) and
// dV/dk = (-2 Es fs, -2 Es fg, fs^2, fg^2).  Entry layout: see HGField.
// The terms Gs fs_gh + Gg fg_gh are summed per strip from row moments (k_hess_second);
// k_hess_geom adds the products of first derivatives and the k-block entries.

// ---------------------------------------------- closed-form Hessian: second-derivative terms
// The second-derivative terms of the geometric block (each pixel's row weight Gs or Gg times a
// profile's second derivatives in position, frac_dev and shape) are, per Gaussian, the
// weighted pixel sum of n times a polynomial of degree <= 4 in z = P (m - mu).  Down a strip
// z is affine in the row: z_k = z_c + (b, d) s_k with z_c its value at the strip centre and
// s_k = k - (L - 1)/2, so with the strip recurrence for n and the exact centred row moments
// U_m = sum_k t_k s_k^m (t_k = row weight x value, m <= 4; s_k^m are compile-time constants)
// the sums N_pq = sum_k t_k zx_k^p zy_k^q follow by applying the maps
// (X V)_m = zx_c V_m + b V_(m+1) and (Y V)_m = zy_c V_m + d V_(m+1) to U: N_pq = (X^p Y^q U)_0.
// With the moments about the strip centre, every term of these expansions is bounded by the
// strip's own values of |z|^4, so no cancellation beyond a small factor arises.  The entries
// (galaxy component, weights wt, sgn, wnu = wt nu):
//   XX, XY, YY: wt (N20 - a N00, N11 - b N00, N02 - d N00);   XF, YF: sgn N10, sgn N01;
//   F_Sxx, F_Sxy, F_Syy: sgn nu times the same three as XX, XY, YY;
//   X_Sxx: wnu (N30 - 3a N10);   X_Sxy = Y_Sxx: wnu (N21 - 2b N10 - a N01);
//   X_Syy = Y_Sxy: wnu (N12 - d N10 - 2b N01);   Y_Syy: wnu (N03 - 3d N01);
//   Sxx_Sxx: wnu nu (N40 - 6a N20 + 3a^2 N00);   Sxx_Sxy: wnu nu (N31 - 3b N20 - 3a N11 + 3ab N00);
//   Sxx_Syy = Sxy_Sxy: wnu nu (N22 - d N20 - a N02 - 4b N11 + (ad + 2b^2) N00);
//   Sxy_Syy: wnu nu (N13 - 3d N11 - 3b N02 + 3bd N00);   Syy_Syy: wnu nu (N04 - 6d N02 + 3d^2 N00)
// (the expansions of the per-pixel formulas of hess_pixels), and for a star (weight Gs):
// XX, XY, YY: N20 - a N00, N11 - b N00, N02 - d N00.  One pass over the components per strip
// (two exps per component), against one exp and about 55 operations per pixel and component
// for the same terms pixel by pixel.
enum HessStagedField { H_CX = 0, H_CY, H_LW, H_RDY, H_A, H_B, H_D, H_WT, H_WNU, H_SGN, H_NU, NDH };

// One wave writes the staged table of a box (field-major [NDH][NCP], slots as in
// stage_derived) into its LDS slot; nu[g]: nu of galaxy component g.
__device__ __forceinline__ void stage_hess(const double* __restrict__ tab, const double* __restrict__ nu,
                                           double* my, int lane) {
    if (lane < NCOMP) {
        const double* e = tab + lane * CST;
        double* o = my + staged_slot(lane);
        o[H_CX * NCP] = e[F_CX];
        o[H_CY * NCP] = e[F_CY];
        o[H_LW * NCP] = e[F_LOGW];
        o[H_RDY * NCP] = e[F_RDY];
        o[H_A * NCP] = e[F_PXX];
        o[H_B * NCP] = e[F_PXY];
        o[H_D * NCP] = e[F_PYY];
        o[H_WT * NCP] = e[F_WT];
        o[H_WNU * NCP] = e[F_WNU];
        o[H_SGN * NCP] = e[F_SGN];
        o[H_NU * NCP] = lane < NPSF ? 0.0 : nu[lane - NPSF];
    } else if (lane == NCOMP) {   // the zero component (stage_derived)
        double* o = my + NPSF;
#pragma unroll
        for (int f = 0; f < NDH; ++f) o[f * NCP] = 0.0;
        o[H_LW * NCP] = -1000.0;
        o[H_RDY * NCP] = 1.0;
    }
}

template <int L>
__device__ __forceinline__ void hess_second_strip(const double* __restrict__ lt, double px, double py0,
                                                  const double* Gs, const double* Gg, double* H,
                                                  const double* __restrict__ t2, uint64_t live) {
    constexpr double KC = 0.5 * (L - 1);
#pragma unroll 1
    for (int grp = 0; grp < NPSF; ++grp) {
        const bool star = (live >> grp) & 1;
        if (!star && !((live >> (NPSF + grp * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1))) continue;
        const double* es = lt + grp;
        const double dx = px - es[H_CX * NCP], dy = py0 - es[H_CY * NCP];
        const double h2x = -0.5 * (dx * dx), mxy = -(dx * dy), h2y = -0.5 * (dy * dy);
        const double mdx = -dx, mdyh = -(dy + 0.5), dyc = dy + KC;
        if (star) {
            const double a = es[H_A * NCP], b = es[H_B * NCP], d = es[H_D * NCP];
            double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, es[H_LW * NCP]))), t2);
            double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
            const double rdy = es[H_RDY * NCP];
            double U0 = 0.0, U1 = 0.0, U2 = 0.0;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const double sk = (double)k - KC;
                const double t = Gs[k] * n;
                U0 += t;
                U1 = fma(sk, t, U1);
                U2 = fma(sk * sk, t, U2);
                if (k + 1 < L) {
                    n = n * rt;
                    rt = rt * rdy;
                }
            }
            const double zx = fma(a, dx, b * dyc), zy = fma(b, dx, d * dyc);
            const double X10 = fma(zx, U0, b * U1), X11 = fma(zx, U1, b * U2);
            const double Y10 = fma(zy, U0, d * U1), Y11 = fma(zy, U1, d * U2);
            const double N20 = fma(zx, X10, b * X11), N11 = fma(zy, X10, d * X11), N02 = fma(zy, Y10, d * Y11);
            H[HG_XX] += fma(-a, U0, N20);
            H[HG_XY] += fma(-b, U0, N11);
            H[HG_YY] += fma(-d, U0, N02);
        }
        auto gal = [&](const double* __restrict__ e) {
            const double a = e[H_A * NCP], b = e[H_B * NCP], d = e[H_D * NCP];
            double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, e[H_LW * NCP]))), t2);
            double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
            const double rdy = e[H_RDY * NCP];
            double U[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const double sk = (double)k - KC;
                const double t = Gg[k] * n;
                U[0] += t;
                U[1] = fma(sk, t, U[1]);
                U[2] = fma(sk * sk, t, U[2]);
                U[3] = fma(sk * sk * sk, t, U[3]);
                U[4] = fma(sk * sk * sk * sk, t, U[4]);
                if (k + 1 < L) {
                    n = n * rt;
                    rt = rt * rdy;
                }
            }
            const double zx = fma(a, dx, b * dyc), zy = fma(b, dx, d * dyc);
            // Y^q U for q = 1..4, then X^p on each: N_pq = (X^p Y^q U)_0
            double Y1[4], Y2[3], Y3[2];
#pragma unroll
            for (int m = 0; m < 4; ++m) Y1[m] = fma(zy, U[m], d * U[m + 1]);
#pragma unroll
            for (int m = 0; m < 3; ++m) Y2[m] = fma(zy, Y1[m], d * Y1[m + 1]);
#pragma unroll
            for (int m = 0; m < 2; ++m) Y3[m] = fma(zy, Y2[m], d * Y2[m + 1]);
            const double N04 = fma(zy, Y3[0], d * Y3[1]);
            double X1[4], X2[3], X3[2];
#pragma unroll
            for (int m = 0; m < 4; ++m) X1[m] = fma(zx, U[m], b * U[m + 1]);
#pragma unroll
            for (int m = 0; m < 3; ++m) X2[m] = fma(zx, X1[m], b * X1[m + 1]);
#pragma unroll
            for (int m = 0; m < 2; ++m) X3[m] = fma(zx, X2[m], b * X2[m + 1]);
            const double N40 = fma(zx, X3[0], b * X3[1]);
            const double N00 = U[0], N10 = X1[0], N20 = X2[0], N30 = X3[0];
            const double XY1a = fma(zx, Y1[0], b * Y1[1]), XY1b = fma(zx, Y1[1], b * Y1[2]),
                         XY1c = fma(zx, Y1[2], b * Y1[3]);
            const double XXY1a = fma(zx, XY1a, b * XY1b), XXY1b = fma(zx, XY1b, b * XY1c);
            const double N01 = Y1[0], N11 = XY1a, N21 = XXY1a, N31 = fma(zx, XXY1a, b * XXY1b);
            const double XY2a = fma(zx, Y2[0], b * Y2[1]), XY2b = fma(zx, Y2[1], b * Y2[2]);
            const double N02 = Y2[0], N12 = XY2a, N22 = fma(zx, XY2a, b * XY2b);
            const double N03 = Y3[0], N13 = fma(zx, Y3[0], b * Y3[1]);
            const double wt = e[H_WT * NCP], sg = e[H_SGN * NCP], wnu = e[H_WNU * NCP], nu = e[H_NU * NCP];
            const double snu = sg * nu, vnu = wnu * nu;
            const double e20 = fma(-a, N00, N20), e11 = fma(-b, N00, N11), e02 = fma(-d, N00, N02);
            H[HG_XX] = fma(wt, e20, H[HG_XX]);
            H[HG_XY] = fma(wt, e11, H[HG_XY]);
            H[HG_YY] = fma(wt, e02, H[HG_YY]);
            H[HG_XF] = fma(sg, N10, H[HG_XF]);
            H[HG_YF] = fma(sg, N01, H[HG_YF]);
            H[HG_F_SXX] = fma(snu, e20, H[HG_F_SXX]);
            H[HG_F_SXY] = fma(snu, e11, H[HG_F_SXY]);
            H[HG_F_SYY] = fma(snu, e02, H[HG_F_SYY]);
            const double x1 = fma(-3.0 * a, N10, N30);
            const double x2 = fma(-2.0 * b, N10, fma(-a, N01, N21));
            const double x3 = fma(-d, N10, fma(-2.0 * b, N01, N12));
            const double x4 = fma(-3.0 * d, N01, N03);
            H[HG_X_SXX] = fma(wnu, x1, H[HG_X_SXX]);
            H[HG_X_SXY] = fma(wnu, x2, H[HG_X_SXY]);
            H[HG_Y_SXX] = fma(wnu, x2, H[HG_Y_SXX]);
            H[HG_X_SYY] = fma(wnu, x3, H[HG_X_SYY]);
            H[HG_Y_SXY] = fma(wnu, x3, H[HG_Y_SXY]);
            H[HG_Y_SYY] = fma(wnu, x4, H[HG_Y_SYY]);
            const double s1 = fma(-6.0 * a, N20, fma(3.0 * (a * a), N00, N40));
            const double s2 = fma(-3.0 * b, N20, fma(-3.0 * a, N11, fma(3.0 * (a * b), N00, N31)));
            const double s3 = fma(-d, N20, fma(-a, N02, fma(-4.0 * b, N11, fma(fma(a, d, 2.0 * (b * b)), N00, N22))));
            const double s4 = fma(-3.0 * d, N11, fma(-3.0 * b, N02, fma(3.0 * (b * d), N00, N13)));
            const double s5 = fma(-6.0 * d, N02, fma(3.0 * (d * d), N00, N04));
            H[HG_SXX_SXX] = fma(vnu, s1, H[HG_SXX_SXX]);
            H[HG_SXX_SXY] = fma(vnu, s2, H[HG_SXX_SXY]);
            H[HG_SXX_SYY] = fma(vnu, s3, H[HG_SXX_SYY]);
            H[HG_SXY_SXY] = fma(vnu, s3, H[HG_SXY_SXY]);
            H[HG_SXY_SYY] = fma(vnu, s4, H[HG_SXY_SYY]);
            H[HG_SYY_SYY] = fma(vnu, s5, H[HG_SYY_SYY]);
        };
        for_live_pairs(live, grp, [&](int s0, int s1) {
            gal(lt + s0);
            gal(lt + s1);
        });
    }
}

// Second-derivative terms of the geometric block, one lane per strip: the row weights Gs, Gg
// from the stored background and own profile values of each row, then hess_second_strip.
// Writes hg[item] (geometric entries; the k-block entries zero), to which k_hess_geom then
// adds the first-derivative products.  Items of sources outside a.active get zeros.
// Three waves per SIMD (168 VGPRs, some spilled) rather than two (197 VGPRs): the waves wait
// on each strip's row loads, and the third wave hides more of it (Newton iterations on 1024
// sources 1.5% faster).
template <int L>
__global__ void __launch_bounds__(256, 3) k_hess_second(AdjArgs a, const Item* __restrict__ items,
                                                     const PairDev* __restrict__ pairs,
                                                     const celeste_image* __restrict__ images,
                                                     const double* __restrict__ xs, const double* __restrict__ bg,
                                                     const double* __restrict__ tabp,
                                                     const double* __restrict__ coefp,
                                                     const double* __restrict__ own, const double* __restrict__ nu,
                                                     double* __restrict__ hg) {
    if (*a.status) return;
    __shared__ double t2[EXP_TAB];
    extern __shared__ double ltab[];   // [waves per block][NDH][NCP], sized at launch
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    double* my = ltab + (threadIdx.x >> 6) * (NCP * NDH);
    int j = a.dynamic ? next_item_s(a.counter, lane) : blockIdx.x * wpb + (threadIdx.x >> 6);
    while (j < a.items.n) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        double* out = hg + (size_t)ii * NHG;
        if (a.active && !a.active[p.src]) {
            if (lane < NHG) out[lane] = 0.0;
            j = a.dynamic ? next_item_s(a.counter, lane) : j + nw;
            continue;
        }
        const celeste_image& im = images[p.img];
        const double* kp = coefp + (size_t)it.pair * NCOEF;
        const double k1 = kp[C_K1], k2 = kp[C_K2], k3 = kp[C_K3], k4 = kp[C_K4];
        __builtin_amdgcn_wave_barrier();
        stage_hess(tabp + (size_t)it.pair * NCOMP * CST, nu, my, lane);
        const uint64_t live = item_live(tabp + (size_t)it.pair * NCOMP * CST, p, it, L, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double H[NHG_GEO];
#pragma unroll
        for (int f = 0; f < NHG_GEO; ++f) H[f] = 0.0;
        for (int q = lane; q < it.count; q += 64) {
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            double Gs[L], Gg[L];
#pragma unroll
            for (int kk = 0; kk < L; ++kk) {
                const int r = r0 + (kk < nrow ? kk : 0);   // rows past the box reuse row 0 (weight 0)
                const double x = xs[(size_t)im.pix_offset + (size_t)r * im.W + c];
                const size_t vi = (size_t)p.visit_off + (size_t)(r - p.r0) * p.w + (c - p.c0);
                double gs = 0.0, gg = 0.0;
                if (kk < nrow && x == x) {
                    const double fs = own[2 * vi], fgv = own[2 * vi + 1];
                    const double Es = k1 * fs + k2 * fgv;
                    const double E = bg[2 * vi] + Es;
                    const double V = bg[2 * vi + 1] + k3 * (fs * fs) + k4 * (fgv * fgv) - Es * Es;
                    const double inv = frcp(E);
                    const double inv2 = inv * inv;
                    const double lE = x * inv * (1.0 + V * inv2) - 1.0;
                    const double lV = -0.5 * x * inv2;
                    const double A = lE - 2.0 * Es * lV;
                    gs = A * k1 + 2.0 * lV * (k3 * fs);
                    gg = A * k2 + 2.0 * lV * (k4 * fgv);
                }
                Gs[kk] = gs;
                Gg[kk] = gg;
            }
            hess_second_strip<L>(my, (double)c, (double)r0, Gs, Gg, H, t2, live);
        }
#pragma unroll
        for (int f = 0; f < NHG_GEO; ++f) {
            const double v = wave_sum(H[f]);
            if (lane == 0) out[f] = v;
        }
        if (lane >= NHG_GEO && lane < NHG) out[lane] = 0.0;
        j = a.dynamic ? next_item_s(a.counter, lane) : j + nw;
    }
}

// One wave per work item.  The item's pixels (stored backgrounds and own profile values of
// the listed boxes) are cut into runs of HPX rows of one strip; the runs, taken by row
// index and then by strip, are dealt round-robin to the lanes, so that an item of fewer
// than 64 strips still fills the wave.  The wave adds its NHG sums onto hg[item], which
// k_hess_second has filled with the second-derivative terms; the items of sources outside
// a.active (when given) get zeros.  Launched with two rows and two waves per SIMD: on 1024
// sources 24% faster per Newton iteration than one row (before the second-derivative terms
// moved to k_hess_second), and faster than three rows (more spills) or four rows at one
// wave.
#ifndef CELESTE_HESS_RUN
#define CELESTE_HESS_RUN 4
#endif
constexpr int HESS_RUN = CELESTE_HESS_RUN;   // rows per run of k_hess_geom

template <int L, int R>
__global__ void __launch_bounds__(256, 2) k_hess_geom(AdjArgs a, const Item* __restrict__ items,
                                                   const PairDev* __restrict__ pairs,
                                                   const celeste_image* __restrict__ images,
                                                   const double* __restrict__ xs, const double* __restrict__ bg,
                                                   const double* __restrict__ tabp,
                                                   const double* __restrict__ coefp,
                                                   const double* __restrict__ own, const double* __restrict__ nu,
                                                   double* __restrict__ hg) {
    if (*a.status) return;
    __shared__ double t2[EXP_TAB];
    extern __shared__ double ltab[];   // [waves per block][NDH][NCP], sized at launch
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    double* my = ltab + (threadIdx.x >> 6) * (NCP * NDH);
    int j = a.dynamic ? next_item_s(a.counter, lane) : blockIdx.x * wpb + (threadIdx.x >> 6);
    while (j < a.items.n) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        if (a.active && !a.active[p.src]) {
            if (lane < NHG) hg[(size_t)ii * NHG + lane] = 0.0;
            j = a.dynamic ? next_item_s(a.counter, lane) : j + nw;
            continue;
        }
        const celeste_image& im = images[p.img];
        const double* kp = coefp + (size_t)it.pair * NCOEF;
        const double k[NCOEF] = {kp[0], kp[1], kp[2], kp[3]};
        __builtin_amdgcn_wave_barrier();
        stage_hess(tabp + (size_t)it.pair * NCOMP * CST, nu, my, lane);
        const uint64_t live = item_live(tabp + (size_t)it.pair * NCOMP * CST, p, it, L, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double H[NHG];
#pragma unroll
        for (int f = 0; f < NHG; ++f) H[f] = 0.0;
        // runs of R rows per strip: those of the item's first strip, the longest
        const int nk = (min(L, p.h - (it.start / p.w) * L) + R - 1) / R;
        for (int g = lane; g < it.count * nk; g += 64) {
            const int kr = g / it.count, q = g - kr * it.count;
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            const int kk = kr * R;
            if (kk >= nrow) continue;
            const double px = (double)c, py0 = (double)(r0 + kk);
            // first derivatives of the star and galaxy profiles down the run, summed over the
            // components: each component's value by the strip recurrence, z affine in the row
            double S[R][2], F[R][6];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                S[r][0] = S[r][1] = 0.0;
#pragma unroll
                for (int f = 0; f < 6; ++f) F[r][f] = 0.0;
            }
#pragma unroll 1
            for (int grp = 0; grp < NPSF; ++grp) {
                const bool star = (live >> grp) & 1;
                if (!star && !((live >> (NPSF + grp * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1))) continue;
                const double* es = my + grp;
                const double dx = px - es[H_CX * NCP], dy = py0 - es[H_CY * NCP];
                const double h2x = -0.5 * (dx * dx), mxy = -(dx * dy), h2y = -0.5 * (dy * dy);
                const double mdx = -dx, mdyh = -(dy + 0.5);
                if (star) {
                    const double a = es[H_A * NCP], b = es[H_B * NCP], d = es[H_D * NCP];
                    double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, es[H_LW * NCP]))), t2);
                    double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
                    const double rdy = es[H_RDY * NCP];
                    const double zx0 = fma(a, dx, b * dy), zy0 = fma(b, dx, d * dy);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double zx = fma(b, (double)r, zx0), zy = fma(d, (double)r, zy0);
                        S[r][0] = fma(n, zx, S[r][0]);
                        S[r][1] = fma(n, zy, S[r][1]);
                        if (r + 1 < R) {
                            n = n * rt;
                            rt = rt * rdy;
                        }
                    }
                }
                auto gal = [&](const double* __restrict__ e) {
                    const double a = e[H_A * NCP], b = e[H_B * NCP], d = e[H_D * NCP];
                    double n = fexp(fma(a, h2x, fma(b, mxy, fma(d, h2y, e[H_LW * NCP]))), t2);
                    double rt = fexp(clamp_arg(fma(b, mdx, d * mdyh)), t2);
                    const double rdy = e[H_RDY * NCP];
                    const double wt = e[H_WT * NCP], sg = e[H_SGN * NCP], wnu = e[H_WNU * NCP];
                    const double zx0 = fma(a, dx, b * dy), zy0 = fma(b, dx, d * dy);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double zx = fma(b, (double)r, zx0), zy = fma(d, (double)r, zy0);
                        const double wn = wt * n, vn = wnu * n;
                        F[r][0] = fma(wn, zx, F[r][0]);
                        F[r][1] = fma(wn, zy, F[r][1]);
                        F[r][2] = fma(sg, n, F[r][2]);
                        F[r][3] = fma(vn, fma(zx, zx, -a), F[r][3]);
                        F[r][4] = fma(vn, fma(zx, zy, -b), F[r][4]);
                        F[r][5] = fma(vn, fma(zy, zy, -d), F[r][5]);
                        if (r + 1 < R) {
                            n = n * rt;
                            rt = rt * rdy;
                        }
                    }
                };
                for_live_pairs(live, grp, [&](int s0, int s1) {
                    gal(my + s0);
                    gal(my + s1);
                });
            }
            // products of first derivatives and the k-block entries, row by row (the pixel
            // scalars from the row's stored background and own values)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = kk + r < nrow ? kk + r : kk;   // rows past the strip reuse row kk
                const size_t gi = (size_t)im.pix_offset + (size_t)(r0 + row) * im.W + c;
                const double x = xs[gi];
                if (!(kk + r < nrow && x == x)) continue;
                const size_t vi = (size_t)p.visit_off + (size_t)(r0 + row - p.r0) * p.w + (c - p.c0);
                const double fs = own[2 * vi], fg = own[2 * vi + 1];
                const double Es = k[C_K1] * fs + k[C_K2] * fg;
                const double E = bg[2 * vi] + Es;
                const double V = bg[2 * vi + 1] + k[C_K3] * (fs * fs) + k[C_K4] * (fg * fg) - Es * Es;
                const double inv = frcp(E);
                const double inv2 = inv * inv;
                const double rr = V * inv2;
                const double lE = x * inv * (1.0 + rr) - 1.0;
                const double lV = -0.5 * x * inv2;
                const double lEE = -x * inv2 * (1.0 + 3.0 * rr);
                const double lEV = x * inv2 * inv;
                const double A = lE - 2.0 * Es * lV;
                double Eg[6], Vg[6];
#pragma unroll
                for (int gg = 0; gg < 6; ++gg) {
                    const double Sg = gg < 2 ? S[r][gg] : 0.0;
                    Eg[gg] = k[C_K1] * Sg + k[C_K2] * F[r][gg];
                    Vg[gg] = 2.0 * (k[C_K3] * fs) * Sg + 2.0 * (k[C_K4] * fg) * F[r][gg] - 2.0 * Es * Eg[gg];
                }
                const double lEE2 = lEE - 2.0 * lV, lV2 = 2.0 * lV;
#pragma unroll
                for (int qq = 0; qq < NHG_GEO; ++qq) {
                    const int g1 = hg_row(qq), h1 = hg_col(qq);
                    double v = (lEE2 * Eg[g1] + lEV * Vg[g1]) * Eg[h1] + (lEV * Eg[g1]) * Vg[h1] +
                               lV2 * k[C_K4] * F[r][g1] * F[r][h1];
                    if (g1 < 2 && h1 < 2) v += lV2 * k[C_K3] * S[r][g1] * S[r][h1];
                    H[qq] += v;
                }
                const double Rc = lEE - 2.0 * lEV * Es - 2.0 * lV;
#pragma unroll
                for (int qq = 0; qq < 5; ++qq) {
                    const int g1 = qq < 2 ? qq : qq + 1;
                    const double Sg = g1 < 2 ? S[r][g1] : 0.0;
                    const double Rv = Rc * Eg[g1] + lEV * Vg[g1];
                    double* o = H + NHG_GEO + 4 * qq;
                    o[0] += fs * Rv + A * Sg;
                    o[1] += fg * Rv + A * F[r][g1];
                    o[2] += lEV * (fs * fs) * Eg[g1] + lV2 * fs * Sg;
                    o[3] += lEV * (fg * fg) * Eg[g1] + lV2 * fg * F[r][g1];
                }
            }
        }
        // the item's sums side by side (one sum at a time, each shuffle and lane 0's
        // read-modify-write would wait in turn); lane f adds sum f onto the
        // second-derivative terms of k_hess_second
        wave_sums<NHG>(H);
        const double hv = lane_pick<NHG>(H, lane);
        if (lane < NHG) hg[(size_t)ii * NHG + lane] += hv;
        j = a.dynamic ? next_item_s(a.counter, lane) : j + nw;
    }
}

template <int L>
__global__ void __launch_bounds__(256) k_background_strips(BgArgs a, const Item* __restrict__ items,
                                                           const PairDev* __restrict__ pairs,
                                                           const celeste_image* __restrict__ images,
                                                           const int32_t* __restrict__ nbr,
                                                           const double* __restrict__ tabv,
                                                           const double* __restrict__ coefv,
                                                           double* __restrict__ bg) {
    if (*a.status) return;
    __shared__ double t2[EXP_TAB];
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int j = blockIdx.x * wpb + (threadIdx.x >> 6); j < a.items.n; j += nw) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        const celeste_image& im = images[p.img];
        for (int q = lane; q < it.count; q += 64) {
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            double Eb[L], Vb[L];
            strip_background<L>(p, pairs, nbr, tabv, coefv, im, c, r0, Eb, Vb, t2);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k >= nrow) break;
                const size_t vi = (size_t)p.visit_off + (size_t)(r0 + k - p.r0) * p.w + (c - p.c0);
                bg[2 * vi] = Eb[k];
                bg[2 * vi + 1] = Vb[k];
            }
        }
    }
}

// Background of the listed visits from the other boxes' stored own profile values (sweeps:
// the stored values are kept current box by box), no Gaussian evaluated.
template <int L>
__global__ void __launch_bounds__(256) k_background_fg(BgArgs a, const Item* __restrict__ items,
                                                       const PairDev* __restrict__ pairs,
                                                       const celeste_image* __restrict__ images,
                                                       const int32_t* __restrict__ nbr,
                                                       const double* __restrict__ coefv,
                                                       const double* __restrict__ fgm, double* __restrict__ bg) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int j = blockIdx.x * wpb + (threadIdx.x >> 6); j < a.items.n; j += nw) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        const celeste_image& im = images[p.img];
        for (int q = lane; q < it.count; q += 64) {
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            double Eb[L], Vb[L];
            strip_background_fg<L>(p, pairs, nbr, coefv, fgm, im, c, r0, Eb, Vb);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k < nrow) {
                    const size_t vi = (size_t)p.visit_off + (size_t)(r0 + k - p.r0) * p.w + (c - p.c0);
                    bg[2 * vi] = Eb[k];
                    bg[2 * vi + 1] = Vb[k];
                }
            }
        }
    }
}

// Sum over each box of log(x!) (masked pixels excluded): a constant of the pixel terms,
// computed once per plan, one wave per box, fixed-order reduction.
__global__ void __launch_bounds__(256) k_pair_lgamma(const PairDev* __restrict__ pairs, int n_pairs,
                                                     const celeste_image* __restrict__ images,
                                                     const double* __restrict__ xs, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= n_pairs) return;
    const PairDev p = pairs[w];
    const celeste_image& im = images[p.img];
    double acc = 0.0;
    for (int i = lane; i < p.h * p.w; i += 64) {
        const int rr = i / p.w;
        const double x = xs[(size_t)im.pix_offset + (size_t)(p.r0 + rr) * im.W + p.c0 + (i - rr * p.w)];
        if (x == x) acc += lgamma(x + 1.0);
    }
    acc = wave_sum(acc);
    if (lane == 0) out[w] = acc;
}

// Own star and galaxy profile values of every visit of the selected items, stored as
// [visit][2] (render pass 1; the fused adjoint reads them back instead of recomputing).
// Like the fused adjoint, the wave stages each item's box table into LDS and takes the seeds
// in the PSF groups' centre frames: the table read through scalar loads had the waves
// waiting on the scalar cache (render 0.488 -> 0.460 ms on the 2000-source field).
template <int L>
__global__ void __launch_bounds__(256) k_strip_fg(Sel sel, const Item* __restrict__ items,
                                                  const PairDev* __restrict__ pairs, const double* __restrict__ tab,
                                                  double* __restrict__ fgm, const int* status) {
    if (*status) return;
    __shared__ double t2[EXP_TAB];
    extern __shared__ double ltab[];   // [waves per block][NDF][NCP], sized at launch
    fill_exp_table(t2);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    double* my = ltab + (threadIdx.x >> 6) * (NCP * NDF);
    for (int j = blockIdx.x * wpb + (threadIdx.x >> 6); j < sel.n; j += nw) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(sel, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        const double* tb = tab + (size_t)it.pair * NCOMP * CST;
        __builtin_amdgcn_wave_barrier();
        stage_derived(tb, my, lane);
        const uint64_t live = item_live(tb, p, it, L, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int q = lane; q < it.count; q += 64) {
            int c, r0, nrow;
            strip_geometry(p, it.start + q, L, c, r0, nrow);
            double fs[L], fg[L];
            strip_values_staged<L>(my, (double)c, (double)r0, fs, fg, t2, live);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k >= nrow) break;
                const size_t vi = (size_t)p.visit_off + (size_t)(r0 + k - p.r0) * p.w + (c - p.c0);
                fgm[2 * vi] = fs[k];
                fgm[2 * vi + 1] = fg[k];
            }
        }
    }
}

// Work of the strip passes under the component culling, for the FLOP count of a launch:
// one wave per item, each lane testing its component as the strip kernels do (item_live).
// out[0] strips, [1] visits, [2] PSF groups evaluated x strips, [3] live stars x strips,
// [4] live galaxy components x strips, [5] zero-component pads x strips, [6] live stars x
// visits, [7] live galaxy components x visits, [8] pads x visits (all summed over items).
__global__ void __launch_bounds__(64) k_live_counts(Sel sel, const Item* __restrict__ items,
                                                    const PairDev* __restrict__ pairs,
                                                    const double* __restrict__ tab, int L,
                                                    unsigned long long* __restrict__ out, const int* status) {
    if (*status) return;
    const int lane = threadIdx.x;
    unsigned long long sum[NLIVE_COUNTS] = {};   // this wave's items (lane 0)
    for (int j = blockIdx.x; j < sel.n; j += gridDim.x) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(sel, j));
        const Item it = items[ii];
        const PairDev p = pairs[it.pair];
        const uint64_t live = item_live(tab + (size_t)it.pair * NCOMP * CST, p, it, L, lane);
        long long v = 0;   // visits of the item's strips
        for (int q = lane; q < it.count; q += 64) v += min(L, p.h - ((it.start + q) / p.w) * L);
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        unsigned long long groups = 0, stars = 0, gal = 0, pads = 0;
        for (int g = 0; g < NPSF; ++g) {
            const uint32_t gm = (uint32_t)(live >> (NPSF + g * NGAL_PER_PSF)) & ((1u << NGAL_PER_PSF) - 1);
            const int st = (int)((live >> g) & 1), ng = __builtin_popcount(gm);
            groups += (st || ng) ? 1 : 0;
            stars += st;
            gal += ng;
            pads += ng & 1;
        }
        const unsigned long long n = (unsigned long long)it.count, vv = (unsigned long long)v;
        sum[0] += n;
        sum[1] += vv;
        sum[2] += n * groups;
        sum[3] += n * stars;
        sum[4] += n * gal;
        sum[5] += n * pads;
        sum[6] += vv * stars;
        sum[7] += vv * gal;
        sum[8] += vv * pads;
    }
    if (lane == 0)
        for (int f = 0; f < NLIVE_COUNTS; ++f) atomicAdd(out + f, sum[f]);
}

// Render pass 2: E and V of every pixel of a tile, summing the stored own values of the
// tile's boxes in ascending box order (deterministic, no atomics).  Tile = (64 / tile_w * RP)
// rows x tile_w columns; lane l owns rows l / tile_w + k (64 / tile_w), k < RP.
template <int RP, bool SUMS>
__global__ void __launch_bounds__(256) k_gather_planes(RenderArgs a, const TileDev* __restrict__ tiles,
                                                       const int32_t* __restrict__ tile_list,
                                                       const PairDev* __restrict__ pairs,
                                                       const celeste_image* __restrict__ images,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ fgm, double* __restrict__ Eout,
                                                       double* __restrict__ Vout, const double* __restrict__ xs,
                                                       double* __restrict__ tile_sums) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const TileDev td = tiles[t];
    const celeste_image& im = images[td.img];
    const int rows_per_pass = 64 / a.tile_w;
    const int c = td.c0 + lane % a.tile_w;
    int r[RP];
    double E[RP], V[RP];
    bool covered[RP];
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        r[k] = td.r0 + lane / a.tile_w + k * rows_per_pass;
        E[k] = (r[k] < im.H && c < im.W) ? sky_at(im, r[k], c) : im.sky;
        V[k] = 0.0;
        covered[k] = false;
    }
    // boxes in list order (the sums are fixed-order); GU boxes' loads are issued before any
    // of them is added, so that their latencies overlap (2000-source field, 16 x 16 tiles: 0.533 ->
    // 0.499 ms for the render; four or eight boxes at a time cost occupancy and are slower)
    constexpr int GU = RP == 4 ? 2 : 4;   // two at 4 rows per lane keeps 7 waves per SIMD
    int j = td.list_begin;
    for (; j + GU <= td.list_end; j += GU) {
        double2 v[GU][RP];
        bool in[GU][RP];
        double kk[GU][NCOEF];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int pi = __builtin_amdgcn_readfirstlane(tile_list[j + u]);
            const PairDev o = pairs[pi];
            const double* kp = coef + (size_t)pi * NCOEF;
#pragma unroll
            for (int q = 0; q < NCOEF; ++q) kk[u][q] = kp[q];
#pragma unroll
            for (int k = 0; k < RP; ++k) {
                in[u][k] = !(r[k] < o.r0 || r[k] >= o.r0 + o.h || c < o.c0 || c >= o.c0 + o.w);
                const size_t vi = (size_t)o.visit_off + (size_t)(r[k] - o.r0) * o.w + (c - o.c0);
                v[u][k] = in[u][k] ? reinterpret_cast<const double2*>(fgm)[vi] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < GU; ++u)
#pragma unroll
            for (int k = 0; k < RP; ++k) {
                if (!in[u][k]) continue;
                const double fs = v[u][k].x, fg = v[u][k].y;
                const double Et = kk[u][C_K1] * fs + kk[u][C_K2] * fg;
                E[k] += Et;
                V[k] += kk[u][C_K3] * fs * fs + kk[u][C_K4] * fg * fg - Et * Et;
                if constexpr (SUMS) covered[k] = true;
            }
    }
    for (; j < td.list_end; ++j) {
        const int pi = __builtin_amdgcn_readfirstlane(tile_list[j]);
        const PairDev o = pairs[pi];
        const double* kp = coef + (size_t)pi * NCOEF;
        const double k1 = kp[C_K1], k2 = kp[C_K2], k3 = kp[C_K3], k4 = kp[C_K4];
#pragma unroll
        for (int k = 0; k < RP; ++k) {
            if (r[k] < o.r0 || r[k] >= o.r0 + o.h || c < o.c0 || c >= o.c0 + o.w) continue;
            const size_t vi = (size_t)o.visit_off + (size_t)(r[k] - o.r0) * o.w + (c - o.c0);
            const double fs = fgm[2 * vi], fg = fgm[2 * vi + 1];
            const double Et = k1 * fs + k2 * fg;
            E[k] += Et;
            V[k] += k3 * fs * fs + k4 * fg * fg - Et * Et;
            if constexpr (SUMS) covered[k] = true;
        }
    }
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        if (r[k] >= im.H || c >= im.W) continue;
        const size_t gi = (size_t)im.pix_offset + (size_t)r[k] * im.W + c;
        Eout[gi] = E[k];
        Vout[gi] = V[k];
        if constexpr (SUMS) {
            // pixel term of a pixel some box covers (the total ELBO counts each such pixel once)
            const double x = xs[gi];
            if (covered[k] && x == x) {
                double lk = x * (log(E[k]) - 0.5 * V[k] / (E[k] * E[k])) - E[k];
                if (a.g.consts.flags & CELESTE_INCLUDE_LGAMMA) lk -= lgamma(x + 1.0);
                l += lk;
            }
        }
    }
    if constexpr (SUMS) {
        l = wave_sum(l);
        if (lane == 0) tile_sums[t] = l;
    }
}

// Elementwise table-driven exp (fn 0), table-driven log (fn 1) and Newton reciprocal (fn 2),
// for testing them against the host's libm.
__global__ void __launch_bounds__(256) k_debug_math(int fn, const double* __restrict__ x, double* __restrict__ y,
                                                    int n) {
    __shared__ double t2[EXP_TAB];
    __shared__ double2 tl[128];
    fill_log_table(tl);
    fill_exp_table(t2);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = fn == 0 ? fexp(x[i], t2) : fn == 1 ? flog(x[i], tl) : frcp(x[i]);
}

// ----------------------------------------------------------------------- launchers
hipError_t launch_debug_math(int fn, const double* x, double* y, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_math, dim3((n + 255) / 256), dim3(256), 0, st, fn, x, y, n);
    return hipGetLastError();
}

hipError_t launch_pair_lgamma(const Geometry& g, int n_pairs, double* out, hipStream_t st) {
    if (n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_lgamma, dim3((n_pairs + 3) / 4), dim3(256), 0, st, g.pairs, n_pairs, g.images, g.x, out);
    return hipGetLastError();
}

hipError_t launch_fill_planes(const celeste_image* images, int n_img, int max_pix, double* E, double* V,
                              const int* status, hipStream_t st) {
    if (n_img <= 0) return hipSuccess;
    int bx = (max_pix + 255) / 256;
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_fill_planes, dim3(bx, n_img), dim3(256), 0, st, images, E, V, status);
    return hipGetLastError();
}

hipError_t launch_strip_fg(const Sel& sel, const Geometry& g, const double* tab, double* fg, int L, int grid, int wpb,
                           const int* status, hipStream_t st) {
    if (sel.n <= 0) return hipSuccess;
    const int need = (sel.n + wpb - 1) / wpb;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    if (L == 8)
        hipLaunchKernelGGL(k_strip_fg<8>, dim3(grid), dim3(64 * wpb), (size_t)wpb * NCP * NDF * sizeof(double), st, sel, g.items, g.pairs, tab, fg, status);
    else if (L == 4)
        hipLaunchKernelGGL(k_strip_fg<4>, dim3(grid), dim3(64 * wpb), (size_t)wpb * NCP * NDF * sizeof(double), st, sel, g.items, g.pairs, tab, fg, status);
    else if (L == 16)
        hipLaunchKernelGGL(k_strip_fg<16>, dim3(grid), dim3(64 * wpb), (size_t)wpb * NCP * NDF * sizeof(double), st, sel, g.items, g.pairs, tab, fg, status);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_live_counts(const Sel& sel, const Geometry& g, const double* tab, int L,
                              unsigned long long* out, const int* status, hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, NLIVE_COUNTS * sizeof(unsigned long long), st);
    if (e != hipSuccess || sel.n <= 0) return e;
    const int grid = sel.n < 1024 ? sel.n : 1024;
    hipLaunchKernelGGL(k_live_counts, dim3(grid), dim3(64), 0, st, sel, g.items, g.pairs, tab, L, out, status);
    return hipGetLastError();
}

hipError_t launch_gather_planes(const RenderArgs& a, const double* fg, int wpb, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    const dim3 grid((a.n_tiles + wpb - 1) / wpb);
    const int rp = a.tile_h * a.tile_w / 64;
    const Geometry& g = a.g;
#define GATHER_ARGS a, a.tiles, a.tile_list, g.pairs, g.images, a.coef, fg, a.E, a.V, g.x, a.tile_sums
    if (a.tile_sums) {
        if (rp == 1) hipLaunchKernelGGL((k_gather_planes<1, true>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else if (rp == 2) hipLaunchKernelGGL((k_gather_planes<2, true>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else if (rp == 4) hipLaunchKernelGGL((k_gather_planes<4, true>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else return hipErrorInvalidValue;
    } else {
        if (rp == 1) hipLaunchKernelGGL((k_gather_planes<1, false>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else if (rp == 2) hipLaunchKernelGGL((k_gather_planes<2, false>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else if (rp == 4) hipLaunchKernelGGL((k_gather_planes<4, false>), grid, dim3(64 * wpb), 0, st, GATHER_ARGS);
        else return hipErrorInvalidValue;
    }
#undef GATHER_ARGS
    return hipGetLastError();
}

hipError_t launch_render_strips(const Sel& sel, const Geometry& g, const double* tab, const double* coef, double* E,
                                double* V, int L, int grid, int wpb, const int* status, hipStream_t st) {
    if (sel.n <= 0) return hipSuccess;
    const int need = (sel.n + wpb - 1) / wpb;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    if (L == 8)
        hipLaunchKernelGGL(k_render_strips<8>, dim3(grid), dim3(64 * wpb), 0, st, sel, g.items, g.pairs, g.images, tab,
                           coef, E, V, status);
    else if (L == 4)
        hipLaunchKernelGGL(k_render_strips<4>, dim3(grid), dim3(64 * wpb), 0, st, sel, g.items, g.pairs, g.images, tab,
                           coef, E, V, status);
    else if (L == 16)
        hipLaunchKernelGGL(k_render_strips<16>, dim3(grid), dim3(64 * wpb), 0, st, sel, g.items, g.pairs, g.images,
                           tab, coef, E, V, status);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class T, int BASE, bool DERIV, int L, bool FGM, bool KK>
static void adjk(const AdjArgs& a, int grid, int wpb, hipStream_t st) {
    const Geometry& g = a.g;
    constexpr bool lds_tab = DERIV && std::is_same<T, double>::value &&
                             (FGM ? (BASE == BASE_PLANES || BASE == BASE_FG) : (BASE == BASE_PLANES || BASE == BASE_BG));
    const size_t lds = lds_tab ? (size_t)wpb * NCP * NDF * sizeof(double) : 0;
    hipLaunchKernelGGL((k_adjoint_strips<T, BASE, DERIV, L, FGM, KK>), dim3(grid), dim3(64 * wpb), lds, st, a,
                       g.items, g.pairs, g.images, g.nbr, g.x, a.E, a.V, a.bg, a.tab, a.coef, a.tab_val, a.coef_val,
                       a.active, a.fg, a.partials);
}

template <class T, int BASE, bool DERIV, int L>
static hipError_t adjs(const AdjArgs& a, int grid, int wpb, hipStream_t st) {
    constexpr bool is_double = std::is_same<T, double>::value;
    // own profile values from the render's stored values: double passes over planes or stored values
    constexpr bool own_fg = is_double && (BASE == BASE_PLANES || BASE == BASE_FG);
    // the pixel-level rows of the intermediate Hessian: double gradient passes over stored
    // backgrounds (own values from pass A, which also gives d fg / d frac_dev)
    constexpr bool can_kk = is_double && DERIV && BASE == BASE_BG;
    if (a.kk && !can_kk) return hipErrorInvalidValue;
    if constexpr (can_kk) {
        if (a.kk) {
            adjk<T, BASE, DERIV, L, false, true>(a, grid, wpb, st);
            return hipSuccess;
        }
    }
    if constexpr (own_fg) {
        if (a.fg) {
            adjk<T, BASE, DERIV, L, true, false>(a, grid, wpb, st);
            return hipSuccess;
        }
    }
    adjk<T, BASE, DERIV, L, false, false>(a, grid, wpb, st);
    return hipSuccess;
}

template <class T, int BASE, bool DERIV>
static hipError_t adjs_L(const AdjArgs& a, int grid, int wpb, int L, hipStream_t st) {
    if (L == 8) return adjs<T, BASE, DERIV, 8>(a, grid, wpb, st);
    if (L == 4) return adjs<T, BASE, DERIV, 4>(a, grid, wpb, st);
    if (L == 16) return adjs<T, BASE, DERIV, 16>(a, grid, wpb, st);
    return hipErrorInvalidValue;
}

template <class T, int BASE>
static hipError_t adjs_D(const AdjArgs& a, bool deriv, int grid, int wpb, int L, hipStream_t st) {
    return deriv ? adjs_L<T, BASE, true>(a, grid, wpb, L, st) : adjs_L<T, BASE, false>(a, grid, wpb, L, st);
}

template <class T>
static hipError_t adjs_B(const AdjArgs& a, int base, bool deriv, int grid, int wpb, int L, hipStream_t st) {
    switch (base) {
        case BASE_PLANES: return adjs_D<T, BASE_PLANES>(a, deriv, grid, wpb, L, st);
        case BASE_BG: return adjs_D<T, BASE_BG>(a, deriv, grid, wpb, L, st);
        case BASE_NBR: return adjs_D<T, BASE_NBR>(a, deriv, grid, wpb, L, st);
        case BASE_FG: return a.fg ? adjs_D<T, BASE_FG>(a, deriv, grid, wpb, L, st) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint(const AdjArgs& a, bool tangent, int base, bool deriv, int grid, int wpb, int L,
                          hipStream_t st) {
    if (a.items.n <= 0) return hipSuccess;
    if (a.dynamic) {
        hipError_t e = launch_fill_int(a.counter, 0, 1, st);
        if (e != hipSuccess) return e;
    }
    const int need = (a.items.n + wpb - 1) / wpb;   // never more waves than items
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    const hipError_t e = tangent ? adjs_B<dual>(a, base, deriv, grid, wpb, L, st)
                                 : adjs_B<double>(a, base, deriv, grid, wpb, L, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}


hipError_t launch_hess_geom(const AdjArgs& a, const double* nu, double* hg, int grid, int wpb, int L,
                            hipStream_t st) {
    if (a.items.n <= 0) return hipSuccess;
    if (L != 16 && L != 8 && L != 4) return hipErrorInvalidValue;
    const int need = (a.items.n + wpb - 1) / wpb;   // never more waves than items
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    const Geometry& g = a.g;
    const size_t lds = (size_t)wpb * NCP * NDH * sizeof(double);
    // second-derivative terms first (they write hg), then the first-derivative products (added
    // onto hg); each kernel takes the items from a fresh queue when the queue is dynamic
    for (int pass = 0; pass < 2; ++pass) {
        if (a.dynamic) {
            hipError_t e = launch_fill_int(a.counter, 0, 1, st);
            if (e != hipSuccess) return e;
        }
#define CEL_HG(LL)                                                                                                 \
    if (pass == 0)                                                                                                 \
        hipLaunchKernelGGL((k_hess_second<LL>), dim3(grid), dim3(64 * wpb), lds, st, a, g.items, g.pairs, g.images, \
                           g.x, a.bg, a.tab, a.coef, a.fg, nu, hg);                                                \
    else                                                                                                           \
        hipLaunchKernelGGL((k_hess_geom<LL, (HESS_RUN < LL ? HESS_RUN : LL)>), dim3(grid), dim3(64 * wpb), lds, st,    \
                           a, g.items, g.pairs, g.images, g.x, a.bg, a.tab, a.coef, a.fg, nu, hg)
        if (L == 16)
            CEL_HG(16);
        else if (L == 8)
            CEL_HG(8);
        else
            CEL_HG(4);
#undef CEL_HG
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_background(const BgArgs& a, int grid, int wpb, int L, hipStream_t st) {
    if (a.items.n <= 0) return hipSuccess;
    const int need = (a.items.n + wpb - 1) / wpb;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    const Geometry& g = a.g;
    if (a.fg) {
        if (L == 8)
            hipLaunchKernelGGL(k_background_fg<8>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                               g.nbr, a.coef_val, a.fg, a.bg);
        else if (L == 4)
            hipLaunchKernelGGL(k_background_fg<4>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                               g.nbr, a.coef_val, a.fg, a.bg);
        else if (L == 16)
            hipLaunchKernelGGL(k_background_fg<16>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                               g.nbr, a.coef_val, a.fg, a.bg);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (L == 8)
        hipLaunchKernelGGL(k_background_strips<8>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                           g.nbr, a.tab_val, a.coef_val, a.bg);
    else if (L == 4)
        hipLaunchKernelGGL(k_background_strips<4>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                           g.nbr, a.tab_val, a.coef_val, a.bg);
    else if (L == 16)
        hipLaunchKernelGGL(k_background_strips<16>, dim3(grid), dim3(64 * wpb), 0, st, a, g.items, g.pairs, g.images,
                           g.nbr, a.tab_val, a.coef_val, a.bg);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cel
