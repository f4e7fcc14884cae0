// Device-side model arithmetic, templated on the scalar type T (double for values and
// gradients, dual for Hessian-vector products).  Regier et al. 2018, Section III and
// Eq. (1); the pixel-level details follow the model the paper cites and are listed with
// the library's header.
#pragma once
#include "internal.h"

namespace cel {

// log flux_b = log r + sum_k BSIGN[b][k] c_k with c_k = log(flux_{k+1} / flux_k),
// reference band r = 2.
__device__ __constant__ static const signed char BSIGN[5][4] = {
    {-1, -1, 0, 0}, {0, -1, 0, 0}, {0, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 1, 1}};

// Sky level of pixel (r, c) (inside the image) of an image: its map when it has one.
__device__ __forceinline__ double sky_at(const celeste_image& im, int r, int c) {
    return im.sky_map ? im.sky_map[(size_t)r * im.W + c] : im.sky;
}

constexpr double LOG_2PI = 1.8378770664093454836;

// Table-driven exponential (P. T. P. Tang, "Table-driven implementation of the exponential
// function in IEEE floating-point arithmetic", ACM TOMS 15(2), 1989), with 256 table
// entries: x = (256 k + j) ln2/256 + r, |r| <= ln2/512, so e^x = 2^k 2^(j/256) e^r and e^r is
// the degree-4 Taylor polynomial (truncation r^5/120 < 3.8e-17 relative).  The reduction
// x - n ln2/256 takes ln2/256 in two parts through fused multiply-adds.  The table
// t2[j] = 2^(j/256) lives in LDS (fill_exp_table).  Accuracy within a few ulps of the
// correctly rounded result for arguments down to the underflow threshold; arguments must
// be <= 709 (callers clamp) and not NaN.
constexpr int EXP_TAB = 256;
constexpr double INV_LN2_256 = 369.32993046757463228;      // 256 / ln 2
constexpr double LN2_256_HI = 2.7076061740622862743e-03;    // ln 2 / 256 rounded
constexpr double LN2_256_LO = 9.0587766165871076501e-20;    // ln 2 / 256 - LN2_256_HI

__device__ __forceinline__ void fill_exp_table(double* t2) {
    for (int j = threadIdx.x; j < EXP_TAB; j += blockDim.x) t2[j] = exp2((double)j * (1.0 / EXP_TAB));
    __syncthreads();
}

__device__ __forceinline__ double fexp(double x, const double* __restrict__ t2) {
    const double n = rint(x * INV_LN2_256);
    const double r = fma(-n, LN2_256_LO, fma(-n, LN2_256_HI, x));
    const int ni = (int)n;
    double p = fma(r, 1.0 / 24.0, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(t2[ni & (EXP_TAB - 1)] * p, ni >> 8);
}

__device__ __forceinline__ dual fexp(dual x, const double* __restrict__ t2) {
    const double e = fexp(x.v, t2);
    return mkd(e, e * x.t);
}

// Table-driven natural logarithm (after P. T. P. Tang, "Table-driven implementation of the
// logarithm function in IEEE floating-point arithmetic", ACM TOMS 16(4), 1990), for finite
// x > 0: x = 2^m y with y in [1/2, 1); F_j = 1/2 + (j + 1/2)/256 is the nearest of 128
// breakpoints (j = the top 7 fraction bits of y), f = y - F_j is exact, and
// log x = m ln2 + log F_j + log1p(f / F_j) with |f / F_j| <= 1/256, log1p by its degree-6
// Taylor polynomial (truncation < 2.1e-18).  tl[j] = (1 / F_j, log F_j) lives in LDS
// (fill_log_table).  Relative error a few ulps away from x = 1; near x = 1 the error is a
// few 1e-16 absolute (the m ln2 and log F_j terms cancel there).
constexpr double LN2_HI = 6.93147180369123816490e-01;       // ln 2, leading 32 bits
constexpr double LN2_LO = 1.90821492927058770002e-10;       // ln 2 - LN2_HI

__device__ __forceinline__ void fill_log_table(double2* tl) {
    for (int j = threadIdx.x; j < 128; j += blockDim.x) {
        const double F = 0.5 + (j + 0.5) * (1.0 / 256.0);
        tl[j] = make_double2(1.0 / F, log(F));
    }
}

__device__ __forceinline__ double flog(double x, const double2* __restrict__ tl) {
    const double y = __builtin_amdgcn_frexp_mant(x);
    const int m = __builtin_amdgcn_frexp_exp(x);
    const int j = (int)((unsigned)__double2hiint(y) >> 13) & 127;
    const double F = fma((double)j, 1.0 / 256.0, 0.5 + 1.0 / 512.0);
    const double2 t = tl[j];
    const double r = (y - F) * t.x;
    double p = fma(r, -1.0 / 6.0, 1.0 / 5.0);
    p = fma(p, r, -0.25);
    p = fma(p, r, 1.0 / 3.0);
    p = fma(p, r, -0.5);
    p = fma(p * r, r, r);
    const double md = (double)m;
    return fma(md, LN2_HI, t.y) + fma(md, LN2_LO, p);
}

// 1 / x for finite x whose reciprocal is a normal number: the hardware estimate refined by
// two Newton steps (each doubles the correct bits), within an ulp or so of the quotient.
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ dual flog(dual x, const double2* __restrict__ tl) {
    return mkd(flog(x.v, tl), x.t * frcp(x.v));
}

__device__ __forceinline__ dual frcp(dual x) {
    const double r = frcp(x.v);
    return mkd(r, -x.t * (r * r));
}

template <class T>
__device__ inline T seed(const double* theta, const double* dir, int dir_mode, int dir_unit,
                         int s, int i) {
    double t = 0.0;
    if (dir_mode == DIR_VEC) t = dir[(size_t)s * ROW + i];
    else if (dir_mode == DIR_UNIT) t = (i == dir_unit) ? 1.0 : 0.0;
    return scalar_traits<T>::make(theta[(size_t)s * ROW + i], t);
}

// Log-normal band-flux moments of both types: a = E[flux_b], b = E[flux_b^2].
template <class T>
__device__ inline void flux_moments(const T* p, int band, T* a, T* b) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int base = 7 + 10 * t;
        T m = p[base];
        T v = p[base + 1];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int sg = BSIGN[band][k];
            if (sg != 0) {
                m = m + (double)sg * p[base + 2 + k];
                v = v + p[base + 6 + k];
            }
        }
        a[t] = exp(m + 0.5 * v);
        b[t] = exp(2.0 * m + 2.0 * v);
    }
}

// Galaxy shape covariance radius^2 R(angle) diag(1, ratio^2) R(angle)^T.
template <class T>
__device__ inline void shape_cov(const T* p, T& sxx, T& sxy, T& syy) {
    const T c = cos(p[4]), s = sin(p[4]);
    const T r2 = p[5] * p[5], q2 = p[3] * p[3];
    sxx = r2 * (c * c + q2 * s * s);
    sxy = r2 * (c * s) * (1.0 - q2);
    syy = r2 * (s * s + q2 * c * c);
}

template <class T>
__device__ inline void write_comp(T* e, T cx, T cy, T sxx, T sxy, T syy, double logw0, T wt, T wnu,
                                  double sgn) {
    const T det = sxx * syy - sxy * sxy;
    const T inv = 1.0 / det;
    e[F_CX] = cx;
    e[F_CY] = cy;
    e[F_PXX] = syy * inv;
    e[F_PXY] = -(sxy * inv);
    e[F_PYY] = sxx * inv;
    e[F_LOGW] = logw0 - LOG_2PI - 0.5 * log(det);
    e[F_WT] = wt;
    e[F_WNU] = wnu;
    e[F_SGN] = scalar_traits<T>::make(sgn, 0.0);
    e[F_RDY] = exp(-(sxx * inv));
}


template <class T>
__device__ inline void pair_w(const T* p, const celeste_image& im, T* w) {
    T a[2], b[2];
    flux_moments(p, im.band, a, b);
    const T q = p[6];
    const double io = im.iota;
    w[W_K1] = io * (q * a[0]);
    w[W_K2] = io * ((1.0 - q) * a[1]);
    w[W_K3] = (io * io) * (q * b[0]);
    w[W_K4] = (io * io) * ((1.0 - q) * b[1]);
    // position and galaxy shape in the image frame: wcs (u - origin), wcs S wcs^T
    const double a00 = im.wcs[0][0], a01 = im.wcs[0][1], a10 = im.wcs[1][0], a11 = im.wcs[1][1];
    const T wx = p[0] - im.origin_x, wy = p[1] - im.origin_y;
    w[W_UX] = a00 * wx + a01 * wy;
    w[W_UY] = a10 * wx + a11 * wy;
    w[W_FDEV] = p[2];
    T sxx, sxy, syy;
    shape_cov(p, sxx, sxy, syy);
    w[W_SXX] = (a00 * a00) * sxx + (2.0 * a00 * a01) * sxy + (a01 * a01) * syy;
    w[W_SXY] = (a00 * a10) * sxx + (a00 * a11 + a01 * a10) * sxy + (a01 * a11) * syy;
    w[W_SYY] = (a10 * a10) * sxx + (2.0 * a10 * a11) * sxy + (a11 * a11) * syy;
}

// Table entry c (0 <= c < NCOMP) of one box from its intermediates w.  Layout: the NPSF
// star components, then per PSF component its NDEV de Vaucouleurs and NEXP exponential
// components.  One lane per entry builds a box's table.
template <class T>
__device__ inline void build_comp_from_w(const T* w, const celeste_image& im, const Consts& K, int c, T* e) {
    const T sxx = w[W_SXX], sxy = w[W_SXY], syy = w[W_SYY];
    const T ux = w[W_UX], uy = w[W_UY];
    const T fdev = w[W_FDEV];
    const int k = c < NPSF ? c : (c - NPSF) / NGAL_PER_PSF;
    const double* ps = im.psf[k];
    const T cx = ux + ps[1], cy = uy + ps[2];
    if (c < NPSF) {
        write_comp(e, cx, cy, scalar_traits<T>::make(ps[3], 0.0), scalar_traits<T>::make(ps[4], 0.0),
                   scalar_traits<T>::make(ps[5], 0.0), log(ps[0]), scalar_traits<T>::make(1.0, 0.0),
                   scalar_traits<T>::make(0.0, 0.0), 0.0);
        return;
    }
    const int j = (c - NPSF) % NGAL_PER_PSF;
    const bool dev = j < NDEV;
    const double nu = dev ? K.dev_nu[j] : K.exp_nu[j - NDEV];
    const double alpha = dev ? K.dev_alpha[j] : K.exp_alpha[j - NDEV];
    const T wt = dev ? fdev : 1.0 - fdev;
    write_comp(e, cx, cy, nu * sxx + ps[3], nu * sxy + ps[4], nu * syy + ps[5], log(ps[0] * alpha), wt, nu * wt,
               dev ? 1.0 : -1.0);
}

// Value-only profile sums of NPIX pixels from a double table.
template <int NPIX>
__device__ __forceinline__ void eval_value(const double* __restrict__ tab, const double* px, const double* py,
                                           double* fs, double* fg) {
#pragma unroll
    for (int k = 0; k < NPIX; ++k) {
        fs[k] = 0.0;
        fg[k] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < NPSF; ++c) {
        const double* e = tab + c * CST;
        const double cx = e[F_CX], cy = e[F_CY], a = e[F_PXX], b = e[F_PXY], d = e[F_PYY], lw = e[F_LOGW];
#pragma unroll
        for (int k = 0; k < NPIX; ++k) {
            const double dx = px[k] - cx, dy = py[k] - cy;
            const double pdx = a * dx + b * dy;
            const double pdy = b * dx + d * dy;
            fs[k] += exp(lw - 0.5 * (dx * pdx + dy * pdy));
        }
    }
#pragma unroll CELESTE_GAL_UNROLL
    for (int c = NPSF; c < NCOMP; ++c) {
        const double* e = tab + c * CST;
        const double cx = e[F_CX], cy = e[F_CY], a = e[F_PXX], b = e[F_PXY], d = e[F_PYY], lw = e[F_LOGW];
        const double wt = e[F_WT];
#pragma unroll
        for (int k = 0; k < NPIX; ++k) {
            const double dx = px[k] - cx, dy = py[k] - cy;
            const double pdx = a * dx + b * dy;
            const double pdy = b * dx + d * dy;
            fg[k] += exp(lw - 0.5 * (dx * pdx + dy * pdy)) * wt;
        }
    }
}

// Chain rule from one box's accumulated sums z[NACC] to d/d theta (27 entries).
template <class T>
__device__ inline void chain_pair(const T* p, const celeste_image& im, const T* z, T* g) {
    T a[2], b[2];
    flux_moments(p, im.band, a, b);
    const double io = im.iota, io2 = io * io;
    const T q = p[6];
    const T k1 = io * (q * a[0]), k2 = io * ((1.0 - q) * a[1]);
    const T k3 = io2 * (q * b[0]), k4 = io2 * ((1.0 - q) * b[1]);
    g[6] += z[A_K1] * (io * a[0]) - z[A_K2] * (io * a[1]) + z[A_K3] * (io2 * b[0]) -
            z[A_K4] * (io2 * b[1]);
    // d k / d m = k (first moment) or 2k (second); d k / d v = k/2 or 2k
    const T dm[2] = {z[A_K1] * k1 + 2.0 * (z[A_K3] * k3), z[A_K2] * k2 + 2.0 * (z[A_K4] * k4)};
    const T dv[2] = {0.5 * (z[A_K1] * k1) + 2.0 * (z[A_K3] * k3),
                     0.5 * (z[A_K2] * k2) + 2.0 * (z[A_K4] * k4)};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int base = 7 + 10 * t;
        g[base] += dm[t];
        g[base + 1] += dv[t];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int sg = BSIGN[im.band][k];
            if (sg != 0) {
                g[base + 2 + k] += (double)sg * dm[t];
                g[base + 6 + k] += dv[t];
            }
        }
    }
    // position: d/du = wcs^T d/d(image-frame position)
    const double a00 = im.wcs[0][0], a01 = im.wcs[0][1], a10 = im.wcs[1][0], a11 = im.wcs[1][1];
    g[0] += a00 * z[A_UX] + a10 * z[A_UY];
    g[1] += a01 * z[A_UX] + a11 * z[A_UY];
    g[2] += z[A_FDEV];
    // shape: with the symmetric gradient G of the image-frame covariance (off-diagonal
    // entries half of d/dSxy), the world-frame one is wcs^T G wcs
    const T Pxx = 0.5 * z[A_SXX], Pxy = 0.5 * z[A_SXY], Pyy = 0.5 * z[A_SYY];
    const T Mxx = Pxx * a00 + Pxy * a10, Mxy = Pxx * a01 + Pxy * a11;
    const T Myx = Pxy * a00 + Pyy * a10, Myy = Pxy * a01 + Pyy * a11;
    const T Gxx = a00 * Mxx + a10 * Myx, Gyy = a01 * Mxy + a11 * Myy;
    const T Gxy = 2.0 * (a00 * Mxy + a10 * Myy);
    const T c = cos(p[4]), s = sin(p[4]);
    const T re = p[5], r2 = re * re, rho = p[3], q2 = rho * rho;
    const T cs = c * s, c2 = c * c, s2 = s * s, om = 1.0 - q2;
    // d Sigma / d axis ratio
    g[3] += (2.0 * r2 * rho) * (Gxx * s2 - Gxy * cs + Gyy * c2);
    // d Sigma / d angle
    g[4] += r2 * om * (2.0 * cs * (Gyy - Gxx) + Gxy * (c2 - s2));
    // d Sigma / d radius
    g[5] += (2.0 * re) * (Gxx * (c2 + q2 * s2) + Gxy * (cs * om) + Gyy * (s2 + q2 * c2));
}

template <class T>
__device__ inline T kl_normal(T m, T v, double m0, double v0) {
    const T d = m - m0;
    return 0.5 * (log(v0) - log(v) + (v + d * d) / v0 - 1.0);
}

// KL(q || prior) of one source; subtracts its gradient from g.  p and g hold NPK entries
// (the mixture responsibilities at NP..NPK-1 are read only with the colour-prior mixture).
// With the mixture (K.mix set), a type's colour term is KL(Cat(kappa) || Cat(w)) +
// sum_d kappa_d KL(N(c_mu, diag c_var) || N(mu_d, S_d)), where the Gaussian KL is
// (sum_k P_kk v_k + delta^T P delta - 4 + log det S - sum_k log v_k) / 2, delta = c_mu - mu_d,
// P = S_d^-1; its derivatives: in kappa_d, log(kappa_d / w_d) + 1 + KL_d; in c_mu,
// sum_d kappa_d P_d delta_d; in c_var_k, sum_d kappa_d (P_d,kk - 1 / v_k) / 2.
template <class T>
__device__ inline T kl_source(const T* p, const Consts& K, T* g) {
    const T q = p[6];
    const double phi = K.prior_phi;
    const T lq = log(q / phi), lnq = log((1.0 - q) / (1.0 - phi));
    T kl = q * lq + (1.0 - q) * lnq;
    T dq = lq - lnq;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int base = 7 + 10 * t;
        const T w = (t == 0) ? q : 1.0 - q;
        const double m0 = K.prior_r[t][0], v0 = K.prior_r[t][1];
        T kt = kl_normal(p[base], p[base + 1], m0, v0);
        g[base] -= w * ((p[base] - m0) / v0);
        g[base + 1] -= w * (0.5 * (1.0 / v0 - 1.0 / p[base + 1]));
        if (K.mix) {
            const T zero = scalar_traits<T>::make(0.0, 0.0);
            T gm[4] = {zero, zero, zero, zero}, gv[4] = {zero, zero, zero, zero}, ksum = zero;
            T logv = zero;
#pragma unroll
            for (int k = 0; k < 4; ++k) logv += log(p[base + 6 + k]);
            for (int d = 0; d < NMIX; ++d) {
                const double* m = K.mix + (size_t)(t * NMIX + d) * MIXF;
                const T kd = p[NP + NMIX * t + d];
                T dl[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) dl[k] = p[base + 2 + k] - m[MX_MEAN + k];
                T quad = zero, tr = zero;
                T Pd[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    T r = zero;
#pragma unroll
                    for (int l = 0; l < 4; ++l) r += m[MX_P + 4 * k + l] * dl[l];
                    Pd[k] = r;
                    quad += dl[k] * r;
                    tr += m[MX_P + 5 * k] * p[base + 6 + k];
                }
                const T kln = 0.5 * (tr + quad + (m[MX_LOGDET] - 4.0) - logv);
                const T lk = log(kd) - m[MX_LOGW];
                kt += kd * (lk + kln);
                g[NP + NMIX * t + d] -= w * (lk + 1.0 + kln);
                ksum += kd;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    gm[k] += kd * Pd[k];
                    gv[k] += kd * m[MX_P + 5 * k];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                g[base + 2 + k] -= w * gm[k];
                g[base + 6 + k] -= w * (0.5 * (gv[k] - ksum / p[base + 6 + k]));
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double cm = K.prior_c[t][0][k], cv = K.prior_c[t][1][k];
                kt += kl_normal(p[base + 2 + k], p[base + 6 + k], cm, cv);
                g[base + 2 + k] -= w * ((p[base + 2 + k] - cm) / cv);
                g[base + 6 + k] -= w * (0.5 * (1.0 / cv - 1.0 / p[base + 6 + k]));
            }
        }
        kl += w * kt;
        dq += (t == 0) ? kt : -kt;
    }
    g[6] -= dq;
    return kl;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline dual wave_sum(dual v) { return mkd(wave_sum(v.v), wave_sum(v.t)); }

// Wave sums of N values at once, each by the butterfly of wave_sum (so bitwise the same
// sums): the N shuffles of a step are issued together and their latencies overlap, where
// N calls of wave_sum would wait on each in turn.
template <int N>
__device__ inline void wave_sums(double* v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double t[N];
#pragma unroll
        for (int f = 0; f < N; ++f) t[f] = __shfl_xor(v[f], o, 64);
#pragma unroll
        for (int f = 0; f < N; ++f) v[f] += t[f];
    }
}
// v[lane] in lanes below N (zero above): N wave-uniform values spread over the lanes, so
// that one coalesced store by lanes 0..N-1 writes them all
template <int N>
__device__ inline double lane_pick(const double* v, int lane) {
    double m = 0.0;
#pragma unroll
    for (int f = 0; f < N; ++f) m = lane == f ? v[f] : m;
    return m;
}

}  // namespace cel
