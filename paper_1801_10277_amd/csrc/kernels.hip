// HIP kernels of the FP64 ELBO path for gfx950 (CDNA4, wave64).
//
// Work decomposition:
//  * k_prep:      one thread per (source, image) box builds the box's 45-Gaussian table
//                 and brightness factors (value, or value + tangent).
//  * k_render:    one wave per 64-pixel tile sums E[F] and Var[F] of every box that
//                 covers each pixel, in box order (deterministic, no atomics).
//  * k_adjoint:   persistent waves pop work items (a chunk of one box's pixels); each lane
//                 walks pixels of the chunk, recomputes the own source's Gaussians, forms
//                 the pixel term and its adjoint, and the wave reduces its 11 sums with
//                 cross-lane shuffles into one per-item slot.
//  * k_finalize:  one thread per source sums its items in a fixed order and applies the
//                 chain rule to the 27 parameters, plus the KL term.
// Table entries are addressed with wave-uniform indices so the compiler serves them
// through scalar loads; pixel data is read coalesced along box rows.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "model.h"

namespace cel {

// ----------------------------------------------------------------------- validation
// Domain of a source row: finite; q in (0,1); frac_dev in [0,1]; axis ratio in (0,1];
// radius > 0; variances > 0.
__device__ inline bool row_ok(const double* p) {
    for (int i = 0; i < NP; ++i)
        if (!isfinite(p[i])) return false;
    if (!(p[6] > 0.0 && p[6] < 1.0)) return false;
    if (!(p[2] >= 0.0 && p[2] <= 1.0)) return false;
    if (!(p[3] > 0.0 && p[3] <= 1.0)) return false;
    if (!(p[5] > 0.0)) return false;
    for (int t = 0; t < 2; ++t) {
        const int base = 7 + 10 * t;
        if (!(p[base + 1] > 0.0)) return false;
        for (int k = 0; k < 4; ++k)
            if (!(p[base + 6 + k] > 0.0)) return false;
    }
    return true;
}

__global__ void __launch_bounds__(256) k_validate(const double* __restrict__ theta, const uint8_t* active,
                                                  const int32_t* list, int n, int S, int* status) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int local = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int s = list ? list[j] : j;
        if (s < 0 || s >= S) { local = 1; continue; }
        if (active && !active[s]) continue;
        if (!row_ok(theta + (size_t)s * ROW)) local = 1;
    }
    if (local) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) status[0] = bad ? CELESTE_EDOMAIN : 0;
}

// ----------------------------------------------------------------------- prep
template <class T>
__global__ void __launch_bounds__(128) k_prep(PrepArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.pairs.n) return;
    const int pi = sel_at(a.pairs, j);
    const PairDev pd = a.g.pairs[pi];
    T p[NP];
    for (int i = 0; i < NP; ++i) p[i] = seed<T>(a.theta, a.dir, a.dir_mode, a.dir_unit, pd.src, i);
    const celeste_image im = a.g.images[pd.img];
    T* tab = reinterpret_cast<T*>(a.tab) + (size_t)pi * NCOMP * CST;
    T* coef = reinterpret_cast<T*>(a.coef) + (size_t)pi * NCOEF;
    build_pair<T>(p, im, a.g.consts, tab, coef);
}

// ----------------------------------------------------------------------- render
__global__ void __launch_bounds__(256) k_render(RenderArgs a) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const TileDev td = a.tiles[t];
    const celeste_image& im = a.g.images[td.img];
    const int r = td.r0 + lane / a.tile_w;
    const int c = td.c0 + lane % a.tile_w;
    const bool inside = r < im.H && c < im.W;
    double E = im.sky, V = 0.0;
    bool covered = false;
    for (int k = td.list_begin; k < td.list_end; ++k) {
        const int pi = __builtin_amdgcn_readfirstlane(a.tile_list[k]);
        const PairDev o = a.g.pairs[pi];
        if (!inside || r < o.r0 || r >= o.r0 + o.h || c < o.c0 || c >= o.c0 + o.w) continue;
        covered = true;
        double fs, fg;
        eval_value(a.tab + (size_t)pi * NCOMP * CST, 1, (double)c, (double)r, fs, fg);
        const double* k4 = a.coef + (size_t)pi * NCOEF;
        const double Et = k4[C_K1] * fs + k4[C_K2] * fg;
        E += Et;
        V += k4[C_K3] * fs * fs + k4[C_K4] * fg * fg - Et * Et;
    }
    const size_t gi = (size_t)im.pix_offset + (size_t)r * im.W + c;
    if (inside) {
        a.E[gi] = E;
        a.V[gi] = V;
    }
    if (a.tile_sums) {
        double l = 0.0;
        if (covered) {
            const double x = a.g.x[gi];
            if (x == x) {
                l = x * (log(E) - 0.5 * V / (E * E)) - E;
                if (a.g.consts.flags & CELESTE_INCLUDE_LGAMMA) l -= lgamma(x + 1.0);
            }
        }
        l = wave_sum(l);
        if (lane == 0) a.tile_sums[t] = l;
    }
}

// ----------------------------------------------------------------------- adjoint
__device__ inline void nbr_background(const Geometry& g, const PairDev& p, const double* tab_val,
                                      const double* coef_val, int stride, double sky, int r, int c,
                                      double& Eb, double& Vb) {
    Eb = sky;
    Vb = 0.0;
    for (int q = p.nbr_begin; q < p.nbr_end; ++q) {
        const int pi = __builtin_amdgcn_readfirstlane(g.nbr[q]);
        const PairDev o = g.pairs[pi];
        if (r < o.r0 || r >= o.r0 + o.h || c < o.c0 || c >= o.c0 + o.w) continue;
        double fs, fg;
        eval_value(tab_val + (size_t)pi * NCOMP * CST * stride, stride, (double)c, (double)r, fs, fg);
        const double* k = coef_val + (size_t)pi * NCOEF * stride;
        const double Et = k[C_K1 * stride] * fs + k[C_K2 * stride] * fg;
        Eb += Et;
        Vb += k[C_K3 * stride] * fs * fs + k[C_K4 * stride] * fg * fg - Et * Et;
    }
}

__device__ inline int next_item(int* counter, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(counter, 1);
    return __shfl(v, 0, 64);
}

template <class T, int BASE, bool DERIV>
__global__ void __launch_bounds__(256) k_adjoint(AdjArgs a) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const bool lgam = (a.g.consts.flags & CELESTE_INCLUDE_LGAMMA) != 0;
    int j = a.dynamic ? next_item(a.counter, lane) : blockIdx.x * wpb + (threadIdx.x >> 6);
    while (j < a.items.n) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = a.g.items[ii];
        const PairDev p = a.g.pairs[it.pair];
        if (!a.active || a.active[p.src]) {
            const celeste_image& im = a.g.images[p.img];
            const T* tab = reinterpret_cast<const T*>(a.tab) + (size_t)it.pair * NCOMP * CST;
            const T* kp = reinterpret_cast<const T*>(a.coef) + (size_t)it.pair * NCOEF;
            const T k[NCOEF] = {kp[0], kp[1], kp[2], kp[3]};
            T acc[NACC];
#pragma unroll
            for (int f = 0; f < NACC; ++f) acc[f] = scalar_traits<T>::make(0.0, 0.0);
            for (int q = lane; q < it.count; q += 64) {
                const int idx = it.start + q;
                const int rr = idx / p.w;
                const int r = p.r0 + rr;
                const int c = p.c0 + (idx - rr * p.w);
                const size_t gi = (size_t)im.pix_offset + (size_t)r * im.W + c;
                const double x = a.g.x[gi];
                if (x != x) continue;   // masked pixel
                double Eb, Vb;
                if (BASE == BASE_PLANES) {
                    Eb = a.E[gi];
                    Vb = a.V[gi];
                } else if (BASE == BASE_BG) {
                    const size_t vi = (size_t)(p.visit_off + idx);
                    Eb = a.bg[2 * vi];
                    Vb = a.bg[2 * vi + 1];
                } else {
                    nbr_background(a.g, p, a.tab_val, a.coef_val, a.tab_val_stride, im.sky, r, c, Eb, Vb);
                }
                if (BASE == BASE_PLANES && !DERIV) {
                    // value only: the planes already hold the totals
                    Own<T> o;
                    pixel_accumulate<T, false>(x, scalar_traits<T>::make(Eb, 0.0),
                                               scalar_traits<T>::make(Vb, 0.0),
                                               scalar_traits<T>::make(0.0, 0.0), o, k, acc, lgam);
                    continue;
                }
                Own<T> o;
                eval_own<T, DERIV>(tab, (double)c, (double)r, o);
                const T Es = k[C_K1] * o.fs + k[C_K2] * o.fg;
                const T Vs = k[C_K3] * (o.fs * o.fs) + k[C_K4] * (o.fg * o.fg) - Es * Es;
                T E, V;
                if (BASE == BASE_PLANES) {
                    E = value_with_tangent(Eb, Es);
                    V = value_with_tangent(Vb, Vs);
                } else {
                    E = Eb + Es;
                    V = Vb + Vs;
                }
                pixel_accumulate<T, DERIV>(x, E, V, Es, o, k, acc, lgam);
            }
            T* out = reinterpret_cast<T*>(a.partials) + (size_t)ii * NACC;
#pragma unroll
            for (int f = 0; f < NACC; ++f) {
                const T s = wave_sum(acc[f]);
                if (lane == 0) out[f] = s;
            }
        }
        j = a.dynamic ? next_item(a.counter, lane) : j + nw;
    }
}

// Per-visit background (sky + every other overlapping box) of the selected items.
__global__ void __launch_bounds__(256) k_background(BgArgs a) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int j = blockIdx.x * wpb + (threadIdx.x >> 6); j < a.items.n; j += nw) {
        const int ii = __builtin_amdgcn_readfirstlane(sel_at(a.items, j));
        const Item it = a.g.items[ii];
        const PairDev p = a.g.pairs[it.pair];
        const celeste_image& im = a.g.images[p.img];
        for (int q = lane; q < it.count; q += 64) {
            const int idx = it.start + q;
            const int rr = idx / p.w;
            const int r = p.r0 + rr;
            const int c = p.c0 + (idx - rr * p.w);
            double Eb, Vb;
            nbr_background(a.g, p, a.tab_val, a.coef_val, 1, im.sky, r, c, Eb, Vb);
            const size_t vi = (size_t)(p.visit_off + idx);
            a.bg[2 * vi] = Eb;
            a.bg[2 * vi + 1] = Vb;
        }
    }
}

// ----------------------------------------------------------------------- finalize
template <class T>
__global__ void __launch_bounds__(128) k_finalize(FinArgs a) {
    if (*a.status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.srcs.n) return;
    const int s = sel_at(a.srcs, j);
    if (a.active && !a.active[s]) return;
    T p[NP];
    for (int i = 0; i < NP; ++i) p[i] = seed<T>(a.theta, a.dir, a.dir_mode, a.dir_unit, s, i);
    const T zero = scalar_traits<T>::make(0.0, 0.0);
    T g[NP];
    for (int i = 0; i < NP; ++i) g[i] = zero;
    T val = zero;
    const T* part = reinterpret_cast<const T*>(a.partials);
    for (int pi = a.patch_ptr[s]; pi < a.patch_ptr[s + 1]; ++pi) {
        const PairDev pd = a.g.pairs[pi];
        T z[NACC];
        for (int f = 0; f < NACC; ++f) z[f] = zero;
        for (int it = pd.item_begin; it < pd.item_end; ++it) {
            const T* q = part + (size_t)it * NACC;
            if (a.deriv) {
                for (int f = 0; f < NACC; ++f) z[f] += q[f];
            } else {
                z[A_VAL] += q[A_VAL];
            }
        }
        val += z[A_VAL];
        if (a.deriv) chain_pair<T>(p, a.g.images[pd.img], z, g);
    }
    if (a.g.consts.flags & CELESTE_INCLUDE_KL) {
        T gk[NP];
        for (int i = 0; i < NP; ++i) gk[i] = zero;
        val -= kl_source<T>(p, a.g.consts, gk);
        if (a.deriv)
            for (int i = 0; i < NP; ++i) g[i] += gk[i];
    }
    if (a.elbo) a.elbo[s] = value_of(val);
    if (a.deriv && a.grad) {
        double* o = a.grad + (size_t)s * ROW;
        for (int i = 0; i < NP; ++i) o[i] = value_of(g[i]);
        for (int i = NP; i < ROW; ++i) o[i] = 0.0;
    }
    if (a.deriv && a.tangent) {
        double* o = a.tangent + (size_t)(a.tangent_by_list ? j : s) * a.tangent_stride;
        for (int i = 0; i < NP; ++i) o[i] = tangent_of(g[i]);
        if (a.tangent_pad)
            for (int i = NP; i < ROW; ++i) o[i] = 0.0;
    }
}

// Total ELBO: fixed-order sum of the per-tile pixel sums minus every source's KL.
__global__ void __launch_bounds__(256) k_tile_total(const double* tile_sums, int n_tiles,
                                                    const double* theta, Consts K, int S,
                                                    double* out, const int* status) {
    if (*status) return;
    __shared__ double red[256];
    double acc = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) acc += tile_sums[t];
    if (K.flags & CELESTE_INCLUDE_KL) {
        for (int s = threadIdx.x; s < S; s += blockDim.x) {
            double p[NP], g[NP];
            for (int i = 0; i < NP; ++i) { p[i] = theta[(size_t)s * ROW + i]; g[i] = 0.0; }
            acc -= kl_source<double>(p, K, g);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_fill_int(int* p, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u8_sel(uint8_t* p, Sel s, uint8_t v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < s.n) p[sel_at(s, j)] = v;
}

__global__ void k_fill_f64_sel(double* p, Sel s, double v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < s.n) p[sel_at(s, j)] = v;
}

// ----------------------------------------------------------------------- launchers
hipError_t launch_validate(const double* theta, const uint8_t* active, const int32_t* list, int n,
                           int S, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_validate, dim3(1), dim3(256), 0, st, theta, active, list, n, S, status);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, bool tangent, hipStream_t st) {
    if (a.pairs.n <= 0) return hipSuccess;
    const dim3 grid((a.pairs.n + 127) / 128);
    if (tangent) hipLaunchKernelGGL(k_prep<dual>, grid, dim3(128), 0, st, a);
    else hipLaunchKernelGGL(k_prep<double>, grid, dim3(128), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs& a, int wpb, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    const dim3 grid((a.n_tiles + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_render, grid, dim3(64 * wpb), 0, st, a);
    return hipGetLastError();
}

template <class T, int BASE, bool DERIV>
static void adj(const AdjArgs& a, int grid, int wpb, hipStream_t st) {
    hipLaunchKernelGGL((k_adjoint<T, BASE, DERIV>), dim3(grid), dim3(64 * wpb), 0, st, a);
}

hipError_t launch_adjoint(const AdjArgs& a, bool tangent, int base, bool deriv, int grid, int wpb,
                          hipStream_t st) {
    if (a.items.n <= 0) return hipSuccess;
    if (a.dynamic) {
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, a.counter, 0, 1);
    } else {
        const int need = (a.items.n + wpb - 1) / wpb;
        if (grid > need) grid = need;
    }
    if (grid < 1) grid = 1;
    if (tangent) {
        if (base == BASE_PLANES) deriv ? adj<dual, BASE_PLANES, true>(a, grid, wpb, st)
                                       : adj<dual, BASE_PLANES, false>(a, grid, wpb, st);
        else if (base == BASE_BG) deriv ? adj<dual, BASE_BG, true>(a, grid, wpb, st)
                                        : adj<dual, BASE_BG, false>(a, grid, wpb, st);
        else deriv ? adj<dual, BASE_NBR, true>(a, grid, wpb, st) : adj<dual, BASE_NBR, false>(a, grid, wpb, st);
    } else {
        if (base == BASE_PLANES) deriv ? adj<double, BASE_PLANES, true>(a, grid, wpb, st)
                                       : adj<double, BASE_PLANES, false>(a, grid, wpb, st);
        else if (base == BASE_BG) deriv ? adj<double, BASE_BG, true>(a, grid, wpb, st)
                                        : adj<double, BASE_BG, false>(a, grid, wpb, st);
        else deriv ? adj<double, BASE_NBR, true>(a, grid, wpb, st)
                   : adj<double, BASE_NBR, false>(a, grid, wpb, st);
    }
    return hipGetLastError();
}

hipError_t launch_background(const BgArgs& a, int grid, int wpb, hipStream_t st) {
    if (a.items.n <= 0) return hipSuccess;
    const int need = (a.items.n + wpb - 1) / wpb;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_background, dim3(grid), dim3(64 * wpb), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, bool tangent, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    const dim3 grid((a.srcs.n + 127) / 128);
    if (tangent) hipLaunchKernelGGL(k_finalize<dual>, grid, dim3(128), 0, st, a);
    else hipLaunchKernelGGL(k_finalize<double>, grid, dim3(128), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tile_total(const double* tile_sums, int n_tiles, const double* theta, const Consts& c,
                             int S, double* out, const int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_total, dim3(1), dim3(256), 0, st, tile_sums, n_tiles, theta, c, S, out, status);
    return hipGetLastError();
}

hipError_t launch_fill_u8_sel(uint8_t* p, const Sel& s, uint8_t v, hipStream_t st) {
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8_sel, dim3((s.n + 255) / 256), dim3(256), 0, st, p, s, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64_sel(double* p, const Sel& s, double v, hipStream_t st) {
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64_sel, dim3((s.n + 255) / 256), dim3(256), 0, st, p, s, v);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace cel
