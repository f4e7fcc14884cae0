// Batched Newton trust-region step (Section IV-D of Regier et al. 2018: Newton's method
// with exact Hessians and a trust region; the paper solves the trust-region subproblem
// through an eigendecomposition, Section VI-B).  One wave per source:
//  1. map gradient and Hessian to unconstrained coordinates (logit of q, frac_dev and
//     axis ratio; log of radius and of every variance; identity otherwise; with the
//     colour-prior mixture, each type's 8 responsibilities through a softmax whose last
//     logit is fixed at 0, so 27 + 2 x 7 = 41 coordinates: B = J^T (-H) J - sum_i g_i
//     d2 theta_i / d eta^2 with the Jacobian J of theta(eta));
//  2. Householder reduction of the model Hessian (27 x 27, or 41 x 41) to tridiagonal
//     form T = Q^T B Q in LDS, the lanes owning the rows of the reflections; Q is kept as
//     its reflectors (Q^T g and Q p are applied reflector by reflector), never formed;
//  3. exact subproblem  min g'p + p'Bp/2, |p| <= radius  on T (More and Sorensen's
//     method; Nocedal & Wright, Alg. 4.3): positive pivots of T's factorisation at mu = 0
//     make T positive definite and allow the interior Newton step; otherwise the smallest
//     eigenvalue of T by Sturm-sequence multisection brackets the secular equation
//     |p(mu)| = radius, solved by safeguarded Newton with two O(n) solves per step;
//  4. near the hard case (gradient nearly orthogonal to the lowest eigenvector), the full
//     eigendecomposition instead: implicit QL with Wilkinson's shift on T (Golub and Van
//     Loan, Matrix Computations, Sec. 8.3; Bowdler, Martin, Reinsch and Wilkinson, Numer.
//     Math. 11, 1968) and the subproblem in the eigenbasis, the hard case along the
//     eigenvector of the smallest eigenvalue;
//  5. trial point and predicted increase.
// k_tr_update compares the actual and predicted increase and updates point and radius;
// k_tr_adopt then takes over the trial point's gradient and Hessian where it was accepted.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "model.h"

namespace cel {

constexpr int NEM = NP + 2 * (NMIX - 1);   // unconstrained coordinates with the mixture: 41
constexpr int QL_MAX_ITER = 60;   // QL iterations per eigenvalue before giving up
constexpr double EPS_D = 2.220446049250313e-16;   // 2^-52

// Value of v in lane i (i wave-uniform).
__device__ inline double lane_get(double v, int i) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide minimum and maximum (every lane receives the result).
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline int param_kind(int i) {
    // 1: logit, 2: log, 0: identity
    if (i == 2 || i == 3 || i == 6) return 1;
    if (i == 5) return 2;
    if (i >= 7) {
        const int o = (i - 7) % 10;
        if (o == 1 || o >= 6) return 2;
    }
    return 0;
}

// theta -> eta and the first two derivatives of theta(eta).
__device__ inline void to_unconstrained(int i, double th, double& eta, double& d1, double& d2) {
    const int k = param_kind(i);
    if (k == 1) {
        eta = log(th) - log1p(-th);
        d1 = th * (1.0 - th);
        d2 = d1 * (1.0 - 2.0 * th);
    } else if (k == 2) {
        eta = log(th);
        d1 = th;
        d2 = th;
    } else {
        eta = th;
        d1 = 1.0;
        d2 = 0.0;
    }
}

__device__ inline double from_unconstrained(int i, double eta) {
    const int k = param_kind(i);
    if (k == 1) return 1.0 / (1.0 + exp(-eta));
    if (k == 2) return exp(eta);
    return eta;
}

// Trial row theta(eta + p) from the unconstrained coordinates and the step (LDS), one lane per
// entry of the row: the 27 model parameters through their own maps; with the mixture, each
// type's responsibilities through the softmax of its 7 coordinates and a fixed 0 (shifted by
// their maximum so that no exponential overflows); zero padding.
template <int M>
__device__ inline void write_trial(int t, const double* eta, const double* p, double* trial) {
    if (t < NP) {
        trial[t] = from_unconstrained(t, eta[t] + p[t]);
    } else if (M != NP && t < NPK) {
        const int ty = (t - NP) / NMIX, d = (t - NP) % NMIX;
        const int c0 = NP + (NMIX - 1) * ty;
        double mx = 0.0;
        for (int e = 0; e < NMIX - 1; ++e) mx = fmax(mx, eta[c0 + e] + p[c0 + e]);
        double z = exp(-mx);
        for (int e = 0; e < NMIX - 1; ++e) z += exp(eta[c0 + e] + p[c0 + e] - mx);
        const double num = d < NMIX - 1 ? exp(eta[c0 + d] + p[c0 + d] - mx) : exp(-mx);
        trial[t] = num / z;
    } else if (t < ROW) {
        trial[t] = 0.0;
    }
}

// M = NP (27 parameters) or NEM (43 parameters with the colour-prior mixture, 41
// unconstrained coordinates); NT parameters in theta, gradient and Hessian.
template <int M>
__global__ void __launch_bounds__(64) k_tr_solve(TrArgs a) {
    constexpr int NT = M == NP ? NP : NPK;
    constexpr int NJ = M == NP ? 28 : 44;   // rows of the LDS matrices (M, padded)
    constexpr int LD = M == NP ? 28 : 45;   // padded LDS row
    if (*a.status) return;
    const int j = blockIdx.x;
    const int s = sel_at(a.srcs, j);
    const int t = threadIdx.x;
    __shared__ double B[NJ][LD];   // the model Hessian; later the eigenvectors Z of T (QL path)
    __shared__ double Q[NJ][LD];   // row k: the k-th Householder reflector v_k
    __shared__ double vs[NJ], ws[NJ], dd[NJ], ee[NJ], bh[NJ];
    __shared__ double gm[NJ], eta[NJ], d1[NJ], lam[NJ], ph[NJ], pv[NJ];
    __shared__ double sh_red[64];
    __shared__ int sh_done;
    const double* th = a.theta + (size_t)s * ROW;
    const double* gr = a.grad + (size_t)s * ROW;
    const double* H = a.hess + (size_t)j * NT * NT;
    if (t < NP) {
        double e, p1, p2;
        to_unconstrained(t, th[t], e, p1, p2);
        eta[t] = e;
        d1[t] = p1;
        // minimise f = -ELBO
        gm[t] = -p1 * gr[t];
        lam[t] = p2 * gr[t];   // diagonal curvature term of the ELBO
    }
    if constexpr (M == NP) {
        __syncthreads();
        for (int idx = t; idx < NJ * NJ; idx += 64) {
            const int r = idx / NJ, c = idx - r * NJ;
            double b = 0.0;
            if (r < NP && c < NP) {
                const double hs = 0.5 * (H[r * NP + c] + H[c * NP + r]);
                b = -d1[r] * hs * d1[c];
                if (c == r) b -= lam[r];
            }
            B[r][c] = b;
        }
    } else {
        // softmax coordinates of the responsibilities: kappa_d = e^{eta_d} / (1 + sum_e e^{eta_e})
        // (d < 7), kappa_7 = 1 / (1 + ...); J_de = kappa_d (delta_de - kappa_e);
        // sum_d g_d d2 kappa_d / d eta_e d eta_f = delta_ef (gk_e - S kappa_e) - gk_e kappa_f
        // - kappa_e gk_f + 2 S kappa_e kappa_f with gk_e = g_e kappa_e, S = sum_d g_d kappa_d
        __shared__ double kap[2][NMIX], sk[2];
        __shared__ double G[NPK][LD];   // symmetric H times J
        if (t < 2 * NMIX) kap[t / NMIX][t % NMIX] = th[NP + t];
        __syncthreads();
        if (t < 2) {
            double S = 0.0;
            for (int d = 0; d < NMIX; ++d) S += gr[NP + NMIX * t + d] * kap[t][d];
            sk[t] = S;
        }
        if (t >= NP && t < M) {
            const int ty = (t - NP) / (NMIX - 1), e = (t - NP) % (NMIX - 1);
            eta[t] = log(kap[ty][e]) - log(kap[ty][NMIX - 1]);
        }
        auto jac = [&](int k, int c) -> double {   // d theta_k / d eta_c
            if (c < NP) return k == c ? d1[c] : 0.0;
            if (k < NP) return 0.0;
            const int ty = (c - NP) / (NMIX - 1), e = (c - NP) % (NMIX - 1);
            const int tk = (k - NP) / NMIX, dk = (k - NP) % NMIX;
            if (tk != ty) return 0.0;
            return kap[ty][dk] * ((dk == e ? 1.0 : 0.0) - kap[ty][e]);
        };
        __syncthreads();
        if (t >= NP && t < M) {
            const int ty = (t - NP) / (NMIX - 1), e = (t - NP) % (NMIX - 1);
            gm[t] = -kap[ty][e] * (gr[NP + NMIX * ty + e] - sk[ty]);
        }
        // G = Hs J, lane k owning row k
        if (t < NT) {
            for (int c = 0; c < M; ++c) {
                double v = 0.0;
                if (c < NP) {
                    v = 0.5 * (H[t * NT + c] + H[c * NT + t]) * d1[c];
                } else {
                    const int ty = (c - NP) / (NMIX - 1);
                    for (int d = 0; d < NMIX; ++d) {
                        const int k2 = NP + NMIX * ty + d;
                        v += 0.5 * (H[t * NT + k2] + H[k2 * NT + t]) * jac(k2, c);
                    }
                }
                G[t][c] = v;
            }
        }
        __syncthreads();
        // B = -J^T G - curvature, lane r owning row r
        for (int c = 0; c < NJ; ++c) {
            double b = 0.0;
            if (t < M && c < M) {
                if (t < NP) {
                    b = -d1[t] * G[t][c];
                    if (c == t) b -= lam[t];
                } else {
                    const int ty = (t - NP) / (NMIX - 1), e = (t - NP) % (NMIX - 1);
                    for (int d = 0; d < NMIX; ++d) b -= jac(NP + NMIX * ty + d, t) * G[NP + NMIX * ty + d][c];
                    if (c >= NP && (c - NP) / (NMIX - 1) == ty) {
                        const int f = (c - NP) % (NMIX - 1);
                        const double ke = kap[ty][e], kf = kap[ty][f], S = sk[ty];
                        const double ge = gr[NP + NMIX * ty + e] * ke, gf = gr[NP + NMIX * ty + f] * kf;
                        double curv = -ge * kf - ke * gf + 2.0 * S * ke * kf;
                        if (e == f) curv += ge - S * ke;
                        b -= curv;
                    }
                }
            }
            if (t < NJ) B[t][c] = b;
        }
        __syncthreads();
        // symmetrise (the two halves differ by rounding only)
        for (int idx = t; idx < M * M; idx += 64) {
            const int r = idx / M, c = idx - r * M;
            if (c > r) {
                const double v = 0.5 * (B[r][c] + B[c][r]);
                B[r][c] = v;
                B[c][r] = v;
            }
        }
    }
    // stop test on the unconstrained gradient
    double gmax = (t < M) ? fabs(gm[t]) : 0.0;
    sh_red[t] = gmax;
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int i = 0; i < M; ++i) m = fmax(m, sh_red[i]);
        sh_done = (a.done[s] || !(m >= a.gtol)) ? 1 : 0;
        if (!(m == m)) sh_done = 1;
        a.live[s] = sh_done ? 0 : 1;
    }
    __syncthreads();
    double* trial = a.theta_trial + (size_t)s * ROW;
    if (sh_done) {
        if (t < ROW) trial[t] = (t < NT) ? th[t] : 0.0;
        if (t == 0) {
            a.pred[2 * s] = 0.0;
            a.pred[2 * s + 1] = 0.0;
            a.done[s] = 1;
        }
        return;
    }
    // ---- Householder reduction B = Q T Q^T, T tridiagonal: diagonal dd, ee[i] couples
    // rows i and i + 1, Q = H_0 H_1 ... with H_k = I - bh[k] v_k v_k^T.  Lane i owns row i;
    // the reflector v (zero outside k+1..26) and w = p - (v.p) beta/2 v with p = beta B v go
    // through LDS; v_k is kept in row k of Q.
    for (int k = 0; k + 2 < M; ++k) {
        const double x0 = B[k + 1][k];
        const double ci = (t >= k + 2 && t < M) ? B[t][k] : 0.0;
        const double sigma = wave_sum(ci * ci);
        const double dk = B[k][k];
        if (sigma == 0.0) {   // already tridiagonal in this column (uniform branch)
            dd[k] = dk;
            ee[k] = x0;
            bh[k] = 0.0;   // H_k = I
            if (t < NJ) Q[k][t] = 0.0;
            __syncthreads();
            continue;
        }
        const double mu = sqrt(x0 * x0 + sigma);
        const double alpha = x0 > 0.0 ? -mu : mu;
        const double v0 = x0 - alpha;
        const double beta = 2.0 / (v0 * v0 + sigma);
        const double vi = (t == k + 1) ? v0 : ci;
        if (t < NJ) {
            vs[t] = vi;
            Q[k][t] = vi;
        }
        dd[k] = dk;
        ee[k] = alpha;
        bh[k] = beta;
        __syncthreads();
        // full-length loops (v and w vanish outside k+1..26), unrolled so that the LDS
        // reads of a loop are all in flight together
        double pi = 0.0;
        if (t > k && t < M) {
#pragma unroll
            for (int c = 0; c < M; ++c) pi += B[t][c] * vs[c];
            pi *= beta;
        }
        const double K = 0.5 * beta * wave_sum(vi * pi);
        const double wi = pi - K * vi;
        if (t < NJ) ws[t] = wi;
        __syncthreads();
        if (t > k && t < M) {
#pragma unroll
            for (int c = 0; c < M; ++c) B[t][c] -= vi * ws[c] + wi * vs[c];
        }
        __syncthreads();
    }
    dd[M - 2] = B[M - 2][M - 2];
    dd[M - 1] = B[M - 1][M - 1];
    ee[M - 2] = B[M - 1][M - 2];
    ee[M - 1] = 0.0;
    __syncthreads();
    // ---- subproblem on the tridiagonal matrix T = Q^T B Q (Moré and Sorensen's method,
    // Nocedal & Wright, Alg. 4.3, with T's factorisations instead of B's): lane i keeps
    // d_i, e_i (e_i couples i and i + 1) and the i-th entries of the vectors; scalar
    // recurrences run in every lane alike on values read with a wave-uniform index.
    double dv = (t < M) ? dd[t] : 0.0, ev = (t < M) ? ee[t] : 0.0;
    const double R = a.radius[s];
    // x <- Q^T x (transpose) or Q x for the vector whose entry i lane i holds: the
    // reflectors one by one (every lane takes part in the wave sums)
    auto apply_q = [&](double x, bool transpose) {
        for (int j = 0; j + 2 < M; ++j) {
            const int k = transpose ? j : M - 3 - j;
            const double vk = (t < M) ? Q[k][t] : 0.0;
            x -= bh[k] * wave_sum(vk * x) * vk;
        }
        return x;
    };
    const double gtv = apply_q((t < M) ? gm[t] : 0.0, true);   // Q^T g
    const double gn = sqrt(wave_sum(gtv * gtv));
    // smallest eigenvalue of T (needed when T is indefinite): Sturm counts at 64 points of
    // the bracket per round
    auto smallest_eigenvalue = [&]() {
        double lo_e, hi_e;
        {
            const double em1 = __shfl(ev, t > 0 ? t - 1 : 0, 64);
            const double rad = (t < M) ? fabs(t > 0 ? em1 : 0.0) + fabs(t < M - 1 ? ev : 0.0) : 0.0;
            lo_e = wave_min((t < M) ? dv - rad : INFINITY);
            hi_e = wave_max((t < M) ? dv + rad : -INFINITY);
        }
        for (int round = 0; round < 40; ++round) {
            const double w = hi_e - lo_e;
            if (!(w > 4.0 * EPS_D * fmax(fabs(lo_e), fabs(hi_e)) + 1e-300)) break;
            const double x = lo_e + w * ((double)(t + 1) / 65.0);
            int cnt = 0;
            double q = lane_get(dv, 0) - x;
            if (q == 0.0) q = -1e-300;
            cnt += q < 0.0;
            for (int i = 1; i < M; ++i) {
                const double e1 = lane_get(ev, i - 1);
                q = lane_get(dv, i) - x - e1 * e1 / q;
                if (q == 0.0) q = -1e-300;
                cnt += q < 0.0;
            }
            const unsigned long long hit = __ballot(cnt >= 1);
            const int k = hit ? __ffsll((long long)hit) - 1 : 64;
            const double nlo = k == 0 ? lo_e : lane_get(x, k - 1);
            const double nhi = k < 64 ? lane_get(x, k) : hi_e;
            if (nlo == lo_e && nhi == hi_e) break;
            lo_e = nlo;
            hi_e = nhi;
        }
        return 0.5 * (lo_e + hi_e);
    };
    // factorisation of T + mu I (no pivoting: positive definite whenever it is used) and
    // the two triangular sweeps
    double cpv = 0.0, idv = 0.0;
    auto factor = [&](double mu) {   // returns whether every pivot is positive
        double cprev = 0.0;
        bool pos = true;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const double em1 = i > 0 ? lane_get(ev, i - 1) : 0.0;
            const double den = lane_get(dv, i) + mu - em1 * cprev;
            pos = pos && den > 0.0;
            const double inv = 1.0 / den;
            cprev = i < M - 1 ? lane_get(ev, i) * inv : 0.0;
            cpv = t == i ? cprev : cpv;
            idv = t == i ? inv : idv;
        }
        return pos;
    };
    auto subst = [&](double rhs) {
        double rprev = 0.0, rpv = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const double em1 = i > 0 ? lane_get(ev, i - 1) : 0.0;
            rprev = (lane_get(rhs, i) - em1 * rprev) * lane_get(idv, i);
            rpv = t == i ? rprev : rpv;
        }
        double ynext = rprev, yv = t == M - 1 ? rprev : 0.0;
#pragma unroll
        for (int i = M - 2; i >= 0; --i) {
            ynext = lane_get(rpv, i) - lane_get(cpv, i) * ynext;
            yv = t == i ? ynext : yv;
        }
        return yv;
    };
    bool fast = false;
    double yv = 0.0;
    // positive pivots at mu = 0: T is positive definite (the smallest eigenvalue is
    // positive), so try the interior Newton step and bracket the secular equation from 0
    const bool pd = factor(0.0);
    // a start for the secular equation left of its root, where |p(mu)| > R and Newton's
    // iteration on 1 / |p(mu)| (concave) rises to the root without overshooting it:
    // mu = 0 or the point just above the pole probed below, whichever applies with a finite
    // norm (else the iteration starts from the bracket's upper end)
    double mu_left = -1.0;
    if (pd) {
        yv = subst(-gtv);
        const double n2 = wave_sum(yv * yv);
        fast = n2 <= R * R;
        if (n2 < INFINITY) mu_left = 0.0;
    }
    if (!fast) {
        const double lmin_t = pd ? 0.0 : smallest_eigenvalue();
        const double lo0 = fmax(0.0, -lmin_t);
        bool hard = false;
        if (lo0 > 0.0) {
            // nearly the hard case (g almost orthogonal to the lowest eigenvector) goes to
            // the eigenbasis below
            const double scale = fmax(fabs(lmin_t), wave_max((t < M) ? fabs(dv) + 2.0 * fabs(ev) : 0.0));
            factor(lo0 + 1e-12 * scale);
            const double yp = subst(-gtv);
            const double n2 = wave_sum(yp * yp);
            hard = n2 < R * R;   // (an overflowing norm is the opposite of the hard case)
            if (!hard && n2 < INFINITY) mu_left = lo0 + 1e-12 * scale;
        }
        if (!hard) {
            double lo = lo0, hi = lo0 + gn / R + 1e-300;
            double mu = (mu_left >= lo0 && mu_left < hi) ? mu_left : hi;
            for (int itn = 0; itn < 200; ++itn) {
                factor(mu);
                yv = subst(-gtv);
                const double wv = subst(yv);
                const double n2 = wave_sum(yv * yv), d3 = wave_sum(yv * wv);
                const double nrm = sqrt(n2);
                if (fabs(nrm - R) <= 1e-13 * R) break;
                if (nrm > R) lo = mu;
                else hi = mu;
                double nmu = mu + (nrm - R) / R * (n2 / d3);
                if (!(nmu > lo && nmu < hi)) nmu = 0.5 * (lo + hi);
                if (nmu == mu) break;
                mu = nmu;
            }
            factor(mu);
            yv = subst(-gtv);
            fast = true;
        }
    }
    if (fast) {
        // predicted increase -(g.p + p.B.p/2) with p = Q y: g.p = gt.y, p.B.p = y.T.y
        const double ynext = __shfl(yv, t < M - 1 ? t + 1 : t, 64);
        const double tyy = (t < M) ? dv * yv * yv + (t < M - 1 ? 2.0 * ev * yv * ynext : 0.0) : 0.0;
        const double pr = -(wave_sum(gtv * yv) + 0.5 * wave_sum(tyy));
        const double pn = sqrt(wave_sum(yv * yv));
        if (t == 0) {
            a.pred[2 * s] = pr;
            a.pred[2 * s + 1] = pn;
        }
        const double pq = apply_q(yv, false);   // p = Q y
        if (t < M) pv[t] = pq;
        __syncthreads();
        write_trial<M>(t, eta, pv, trial);
        return;
    }
    // ---- otherwise the full eigendecomposition: implicit QL on T.  Lane i keeps d_i and e_i in registers;
    // the scalar recurrence runs in every lane alike on values read across lanes with a
    // wave-uniform index, and lane i applies the rotations to row i of the eigenvector
    // matrix Z of T (in LDS, where B was; the eigenvectors of the model Hessian are Q Z).
    for (int idx = t; idx < NJ * NJ; idx += 64) {
        const int r = idx / NJ, c = idx - r * NJ;
        B[r][c] = (c == r) ? 1.0 : 0.0;
    }
    if (t < NJ) vs[t] = gtv;
    __syncthreads();
    bool converged = true;
    for (int l = 0; l < M && converged; ++l) {
        for (int iter = 0;; ++iter) {
            // m: the first index from l on whose e_m is negligible against its neighbours
            // (M - 1 if none), every lane testing its own e at once
            const double dn = __shfl(dv, t < 63 ? t + 1 : t, 64);
            const bool small = t < M - 1 && fabs(ev) <= EPS_D * (fabs(dv) + fabs(dn));
            const unsigned long long sm = __ballot(small) & (~0ull << l);
            const int m = sm ? __ffsll((long long)sm) - 1 : M - 1;
            if (m == l) break;
            if (iter == QL_MAX_ITER) {
                converged = false;
                break;
            }
            const double el = lane_get(ev, l), dl = lane_get(dv, l);
            double g = (lane_get(dv, l + 1) - dl) / (2.0 * el);
            double r = hypot(g, 1.0);
            g = lane_get(dv, m) - dl + el / (g + copysign(r, g));
            double sn = 1.0, cs = 1.0, p = 0.0;
            bool deflated = false;
            // row t of Z: entry zpos, rotated but not yet stored, is carried in zc
            int zpos = m;
            double zc = (t < M) ? B[t][m] : 0.0;
            for (int i = m - 1; i >= l; --i) {
                const double ei = lane_get(ev, i);
                const double f = sn * ei, b = cs * ei;
                // r = hypot(f, g) and 1 / r: the reciprocal square root of f^2 + g^2 (hardware
                // estimate, two Newton steps) where the squares stay far from overflow and
                // underflow; hypot and a division elsewhere
                const double q2 = fma(f, f, g * g);
                double rinv = 0.0;
                if (q2 > 0x1p-1000 && q2 < 0x1p+1000) {
                    double y = __builtin_amdgcn_rsq(q2);
                    y = fma(y, 0.5 * fma(-q2 * y, y, 1.0), y);
                    y = fma(y, 0.5 * fma(-q2 * y, y, 1.0), y);
                    rinv = y;
                    r = q2 * y;
                } else {
                    r = hypot(f, g);
                    if (r != 0.0) rinv = 1.0 / r;
                }
                ev = t == i + 1 ? r : ev;
                if (r == 0.0) {   // underflow: the matrix splits here
                    dv = t == i + 1 ? dv - p : dv;
                    ev = t == m ? 0.0 : ev;
                    deflated = true;
                    break;
                }
                sn = f * rinv;
                cs = g * rinv;
                g = lane_get(dv, i + 1) - p;
                r = (lane_get(dv, i) - g) * sn + 2.0 * cs * b;
                p = sn * r;
                dv = t == i + 1 ? g + p : dv;
                g = cs * r - b;
                if (t < M) {
                    const double zi = B[t][i];
                    B[t][i + 1] = sn * zi + cs * zc;
                    zc = cs * zi - sn * zc;
                }
                zpos = i;
            }
            if (t < M) B[t][zpos] = zc;
            if (deflated) continue;
            dv = t == l ? dv - p : dv;
            ev = t == l ? g : (t == m ? 0.0 : ev);
        }
    }
    if (t < NJ) dd[t] = dv;
    __syncthreads();
    if (!converged) {   // no step this iteration: the source stops (not met in practice)
        if (t < ROW) trial[t] = (t < NT) ? th[t] : 0.0;
        if (t == 0) {
            a.pred[2 * s] = 0.0;
            a.pred[2 * s + 1] = 0.0;
            a.done[s] = 1;
            a.live[s] = 0;
        }
        return;
    }
    // ---- subproblem in the eigenbasis: lane i holds lambda_i and entry i of (Q Z)^T g; the
    // sums over the eigenvalues are wave sums (equal in every lane, so every lane takes the
    // same branches)
    const double lamv = (t < M) ? dv : 0.0;
    double ghv = 0.0;   // (Q Z)^T g = Z^T (Q^T g)
    if (t < M)
        for (int k = 0; k < M; ++k) ghv += B[k][t] * vs[k];
    const double lmin = wave_min((t < M) ? lamv : INFINITY);
    const double lmax = wave_max((t < M) ? fabs(lamv) : 0.0);
    const int imin = __ffsll((long long)__ballot(t < M && lamv == lmin)) - 1;   // its first lane
    const double gn2 = wave_sum(ghv * ghv);
    double phv = 0.0;
    bool solved = false;
    if (lmin > 0.0) {
        const double q = (t < M) ? ghv / lamv : 0.0;
        if (wave_sum(q * q) <= R * R) {
            phv = -q;
            solved = true;
        }
    }
    if (!solved) {
        const double lo0 = fmax(0.0, -lmin);
        const double tol = 1e-12 * fmax(lmax, 1e-300);
        // hard case: gradient (numerically) orthogonal to the lowest eigenspace
        const bool low = t < M && lamv <= lmin + tol;
        const double vr = (t < M && !low) ? ghv / (lamv + lo0) : 0.0;
        const double gmin2 = wave_sum(low ? ghv * ghv : 0.0), prest2 = wave_sum(vr * vr);
        if (lo0 > 0.0 && gmin2 <= 1e-28 * fmax(gn2, 1e-300) && prest2 <= R * R) {
            phv = (t == imin) ? sqrt(fmax(R * R - prest2, 0.0)) : -vr;
        } else {
            double lo = lo0, hi = lo0 + sqrt(gn2) / R + 1e-300;
            double mu = hi;
            for (int itn = 0; itn < 200; ++itn) {
                const double den = lamv + mu;
                const double v = (t < M) ? ghv / den : 0.0;
                const double n2 = wave_sum(v * v), d3 = wave_sum((t < M) ? v * v / den : 0.0);
                const double nrm = sqrt(n2);
                if (fabs(nrm - R) <= 1e-13 * R) break;
                if (nrm > R) lo = mu;
                else hi = mu;
                // Newton step on 1/R - 1/|p(mu)|
                double nmu = mu + (nrm - R) / R * (n2 / d3);
                if (!(nmu > lo && nmu < hi)) nmu = 0.5 * (lo + hi);
                if (nmu == mu) break;
                mu = nmu;
            }
            phv = (t < M) ? -ghv / (lamv + mu) : 0.0;
        }
    }
    {
        const double pr = -wave_sum(ghv * phv + 0.5 * lamv * phv * phv);
        const double pn = wave_sum(phv * phv);
        if (t == 0) {
            a.pred[2 * s] = pr;
            a.pred[2 * s + 1] = sqrt(pn);
        }
    }
    if (t < M) ph[t] = phv;
    __syncthreads();
    double zp = 0.0;   // Z ph, then p = Q (Z ph)
    if (t < M)
        for (int i = 0; i < M; ++i) zp += B[t][i] * ph[i];
    const double pq = apply_q(zp, false);
    if (t < M) pv[t] = pq;
    __syncthreads();
    write_trial<M>(t, eta, pv, trial);
}

__global__ void __launch_bounds__(128) k_tr_update(TrArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.srcs.n) return;
    const int s = sel_at(a.srcs, j);
    a.accepted[s] = 0;
    if (a.done[s]) return;
    const double f0 = a.elbo_cur[s], f1 = a.elbo_trial[s];
    const double pr = a.pred[2 * s], pn = a.pred[2 * s + 1];
    double R = a.radius[s];
    double rho = -1.0;
    const bool finite = (f1 == f1) && fabs(f1) < INFINITY;
    if (finite && pr > 0.0) rho = (f1 - f0) / pr;
    if (!finite || rho < 0.25) R = 0.25 * R;
    else if (rho > 0.75 && pn >= 0.99 * a.radius[s]) R = fmin(2.0 * R, a.radius_max);
    if (finite && rho > a.eta_accept) {
        double* th = a.theta + (size_t)s * ROW;
        const double* tr = a.theta_trial + (size_t)s * ROW;
        for (int i = 0; i < a.npar; ++i) th[i] = tr[i];
        a.elbo_cur[s] = f1;
        a.accepted[s] = 1;
    }
    // no further progress possible at working precision
    if (!(pr > 1e-15 * fabs(f0)) || R < 1e-12) a.done[s] = 1;
    a.radius[s] = R;
}

hipError_t launch_tr_solve(const TrArgs& a, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    if (a.npar == NPK)
        hipLaunchKernelGGL(k_tr_solve<NEM>, dim3(a.srcs.n), dim3(64), 0, st, a);
    else if (a.npar == NP)
        hipLaunchKernelGGL(k_tr_solve<NP>, dim3(a.srcs.n), dim3(64), 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// One work-group per listed source.
__global__ void __launch_bounds__(256) k_tr_adopt(TrArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x;
    const int s = sel_at(a.srcs, j);
    if (!a.accepted[s]) return;
    const int n2 = a.npar * a.npar;
    const double* hs = a.hess_trial + (size_t)j * n2;
    double* hd = a.hess + (size_t)j * n2;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) hd[i] = hs[i];
    if (threadIdx.x < ROW) a.grad[(size_t)s * ROW + threadIdx.x] = a.grad_trial[(size_t)s * ROW + threadIdx.x];
}

hipError_t launch_tr_adopt(const TrArgs& a, hipStream_t st) {
    if (a.srcs.n <= 0 || !a.hess_trial || !a.grad_trial) return hipSuccess;
    hipLaunchKernelGGL(k_tr_adopt, dim3(a.srcs.n), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tr_update(const TrArgs& a, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tr_update, dim3((a.srcs.n + 127) / 128), dim3(128), 0, st, a);
    return hipGetLastError();
}

}  // namespace cel
