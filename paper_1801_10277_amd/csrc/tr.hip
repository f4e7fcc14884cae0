// Batched Newton trust-region step (Section IV-D of Regier et al. 2018: Newton's method
// with exact Hessians and a trust region; the trust-region subproblem is solved through
// an eigendecomposition, Section VI-B).  One work-group per source (64 lanes, or 256 for
// small batches):
//  1. map gradient and Hessian to unconstrained coordinates (logit of q, frac_dev and
//     axis ratio; log of radius and of every variance; identity otherwise);
//  2. Jacobi eigendecomposition of the 27x27 model Hessian in LDS with the round-robin
//     ordering (27 padded to 28 indices: each of the 27 steps of a sweep rotates 14
//     disjoint index pairs at once), the rotations applied by the lanes in parallel;
//  3. exact subproblem  min g'p + p'Bp/2, |p| <= radius  in the eigenbasis: interior
//     Newton step, else the secular equation |p(mu)| = radius by safeguarded Newton
//     (Nocedal & Wright, Alg. 4.3), with the hard case handled along the eigenvector of
//     the smallest eigenvalue;
//  4. trial point and predicted increase.
// k_tr_update compares the actual and predicted increase and updates point and radius.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace cel {

constexpr int LD = 28;   // padded LDS row
constexpr int NJ = 28;   // Jacobi index range: the 27 parameters and one idle index
constexpr int NPAIR = NJ / 2;
constexpr int TR_WIDE_BELOW = 512;   // batches smaller than this take 256-lane work-groups

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

template <int TRB>
__global__ void __launch_bounds__(TRB) k_tr_solve(TrArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x;
    const int s = sel_at(a.srcs, j);
    const int t = threadIdx.x;
    __shared__ double B[NJ][LD];
    __shared__ double Q[NJ][LD];
    __shared__ double rot_c[NPAIR], rot_s[NPAIR];
    __shared__ int rot_p[NPAIR], rot_q[NPAIR];
    __shared__ double gm[NP], eta[NP], d1[NP], lam[NP], gh[NP], ph[NP], pv[NP];
    __shared__ double sh_red[64];
    __shared__ int sh_done;
    const double* th = a.theta + (size_t)s * ROW;
    const double* gr = a.grad + (size_t)s * ROW;
    const double* H = a.hess + (size_t)j * NP * NP;
    if (t < NP) {
        double e, p1, p2;
        to_unconstrained(t, th[t], e, p1, p2);
        eta[t] = e;
        d1[t] = p1;
        // minimise f = -ELBO
        gm[t] = -p1 * gr[t];
        lam[t] = p2 * gr[t];   // diagonal curvature term of the ELBO
    }
    __syncthreads();
    for (int idx = t; idx < NJ * NJ; idx += TRB) {
        const int r = idx / NJ, c = idx - r * NJ;
        double b = 0.0;
        if (r < NP && c < NP) {
            const double hs = 0.5 * (H[r * NP + c] + H[c * NP + r]);
            b = -d1[r] * hs * d1[c];
            if (c == r) b -= lam[r];
        }
        B[r][c] = b;
        Q[r][c] = (c == r) ? 1.0 : 0.0;
    }
    // stop test on the unconstrained gradient
    double gmax = (t < NP) ? fabs(gm[t]) : 0.0;
    if (t < 64) sh_red[t] = gmax;
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int i = 0; i < NP; ++i) m = fmax(m, sh_red[i]);
        sh_done = (a.done[s] || !(m >= a.gtol)) ? 1 : 0;
        if (!(m == m)) sh_done = 1;
    }
    __syncthreads();
    double* trial = a.theta_trial + (size_t)s * ROW;
    if (sh_done) {
        if (t < ROW) trial[t] = (t < NP) ? th[t] : 0.0;
        if (t == 0) {
            a.pred[2 * s] = 0.0;
            a.pred[2 * s + 1] = 0.0;
            a.done[s] = 1;
        }
        return;
    }
    // ---- Jacobi sweeps (round-robin order)
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        if (t < NP)
            for (int c = 0; c < NP; ++c) {
                const double v = B[t][c] * B[t][c];
                tot += v;
                if (c != t) off += v;
            }
        if (t < 64) sh_red[t] = off;
        __syncthreads();
        double offs = 0.0;
        for (int i = 0; i < NP; ++i) offs += sh_red[i];
        __syncthreads();
        if (t < 64) sh_red[t] = tot;
        __syncthreads();
        double tots = 0.0;
        for (int i = 0; i < NP; ++i) tots += sh_red[i];
        __syncthreads();
        if (!(offs > 1e-30 * tots) || offs == 0.0) break;
        for (int r = 0; r < NJ - 1; ++r) {
            // round r of the circle schedule: index 0 fixed, the others rotated by r
            if (t < NPAIR) {
                const int i0 = t, i1 = NJ - 1 - t;
                const int a0 = i0 == 0 ? 0 : 1 + (i0 - 1 + r) % (NJ - 1);
                const int a1 = 1 + (i1 - 1 + r) % (NJ - 1);
                const int p = a0 < a1 ? a0 : a1, q = a0 < a1 ? a1 : a0;
                double c = 1.0, sn = 0.0;
                const double apq = B[p][q];
                if (q < NP && apq != 0.0) {
                    const double app = B[p][p], aqq = B[q][q];
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * c;
                }
                rot_p[t] = p;
                rot_q[t] = q;
                rot_c[t] = c;
                rot_s[t] = sn;
            }
            __syncthreads();
            // B <- B J and Q <- Q J for all pairs (disjoint column pairs)
            for (int idx = t; idx < NPAIR * NJ; idx += TRB) {
                const int k = idx / NJ, row = idx - k * NJ;
                const int p = rot_p[k], q = rot_q[k];
                const double c = rot_c[k], sn = rot_s[k];
                const double bkp = B[row][p], bkq = B[row][q];
                B[row][p] = c * bkp - sn * bkq;
                B[row][q] = sn * bkp + c * bkq;
                const double qkp = Q[row][p], qkq = Q[row][q];
                Q[row][p] = c * qkp - sn * qkq;
                Q[row][q] = sn * qkp + c * qkq;
            }
            __syncthreads();
            // B <- J^T B (disjoint row pairs)
            for (int idx = t; idx < NPAIR * NJ; idx += TRB) {
                const int k = idx / NJ, col = idx - k * NJ;
                const int p = rot_p[k], q = rot_q[k];
                const double c = rot_c[k], sn = rot_s[k];
                const double bpk = B[p][col], bqk = B[q][col];
                B[p][col] = c * bpk - sn * bqk;
                B[q][col] = sn * bpk + c * bqk;
            }
            __syncthreads();
            if (t < NPAIR && rot_s[t] != 0.0) {
                B[rot_p[t]][rot_q[t]] = 0.0;
                B[rot_q[t]][rot_p[t]] = 0.0;
            }
            __syncthreads();
        }
    }
    if (t < NP) {
        lam[t] = B[t][t];
        double g = 0.0;
        for (int k = 0; k < NP; ++k) g += Q[k][t] * gm[k];
        gh[t] = g;
    }
    __syncthreads();
    // ---- subproblem in the eigenbasis (lane 0)
    if (t == 0) {
        const double R = a.radius[s];
        double lmin = lam[0], lmax = fabs(lam[0]), gn2 = 0.0;
        int imin = 0;
        for (int i = 0; i < NP; ++i) {
            if (lam[i] < lmin) { lmin = lam[i]; imin = i; }
            lmax = fmax(lmax, fabs(lam[i]));
            gn2 += gh[i] * gh[i];
        }
        bool solved = false;
        double mu = 0.0;
        if (lmin > 0.0) {
            double n2 = 0.0;
            for (int i = 0; i < NP; ++i) n2 += (gh[i] / lam[i]) * (gh[i] / lam[i]);
            if (n2 <= R * R) {
                for (int i = 0; i < NP; ++i) ph[i] = -gh[i] / lam[i];
                solved = true;
            }
        }
        if (!solved) {
            const double lo0 = fmax(0.0, -lmin);
            const double tol = 1e-12 * fmax(lmax, 1e-300);
            // hard case: gradient (numerically) orthogonal to the lowest eigenspace
            double gmin2 = 0.0, prest2 = 0.0;
            for (int i = 0; i < NP; ++i) {
                if (lam[i] <= lmin + tol) gmin2 += gh[i] * gh[i];
                else {
                    const double v = gh[i] / (lam[i] + lo0);
                    prest2 += v * v;
                }
            }
            if (lo0 > 0.0 && gmin2 <= 1e-28 * fmax(gn2, 1e-300) && prest2 <= R * R) {
                for (int i = 0; i < NP; ++i)
                    ph[i] = (lam[i] <= lmin + tol) ? 0.0 : -gh[i] / (lam[i] + lo0);
                ph[imin] = sqrt(fmax(R * R - prest2, 0.0));
                mu = lo0;
            } else {
                double lo = lo0, hi = lo0 + sqrt(gn2) / R + 1e-300;
                mu = hi;
                for (int itn = 0; itn < 200; ++itn) {
                    double n2 = 0.0, d3 = 0.0;
                    for (int i = 0; i < NP; ++i) {
                        const double den = lam[i] + mu;
                        const double v = gh[i] / den;
                        n2 += v * v;
                        d3 += v * v / den;
                    }
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
                for (int i = 0; i < NP; ++i) ph[i] = -gh[i] / (lam[i] + mu);
            }
        }
        double pr = 0.0, pn = 0.0;
        for (int i = 0; i < NP; ++i) {
            pr -= gh[i] * ph[i] + 0.5 * lam[i] * ph[i] * ph[i];
            pn += ph[i] * ph[i];
        }
        a.pred[2 * s] = pr;
        a.pred[2 * s + 1] = sqrt(pn);
    }
    __syncthreads();
    if (t < NP) {
        double p = 0.0;
        for (int i = 0; i < NP; ++i) p += Q[t][i] * ph[i];
        pv[t] = p;
        trial[t] = from_unconstrained(t, eta[t] + p);
    } else if (t < ROW) {
        trial[t] = 0.0;
    }
}

__global__ void __launch_bounds__(128) k_tr_update(TrArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.srcs.n) return;
    const int s = sel_at(a.srcs, j);
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
        for (int i = 0; i < NP; ++i) th[i] = tr[i];
        a.elbo_cur[s] = f1;
    }
    // no further progress possible at working precision
    if (!(pr > 1e-15 * fabs(f0)) || R < 1e-12) a.done[s] = 1;
    a.radius[s] = R;
}

hipError_t launch_tr_solve(const TrArgs& a, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    // a large batch keeps every SIMD busy with one wave per source; a small one gains from
    // spreading each rotation update over four waves (Cyclades rounds on the 20000-source
    // region: 5% per epoch; 256 lanes for 1024 sources would cost 10% per Newton iteration)
    if (a.srcs.n < TR_WIDE_BELOW)
        hipLaunchKernelGGL(k_tr_solve<256>, dim3(a.srcs.n), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_tr_solve<64>, dim3(a.srcs.n), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tr_update(const TrArgs& a, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tr_update, dim3((a.srcs.n + 127) / 128), dim3(128), 0, st, a);
    return hipGetLastError();
}

}  // namespace cel
