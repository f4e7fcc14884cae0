// HIP kernels of the FP64 ELBO path for gfx950 (CDNA4, wave64).
//
// Work decomposition:
//  * k_prep:      one wave per (source, image) box, one lane per table entry, builds the
//                 box's 45-Gaussian table (staged in LDS, written out contiguously) and
//                 brightness factors (value, or value + tangent).
//  * k_render:    one wave per render tile sums E[F] and Var[F] of every box that
//                 covers each pixel, in box order (deterministic, no atomics), and
//                 optionally the pixel terms of covered pixels (total ELBO).
//  * the fused adjoint and the strip render live in strips.hip.
//  * k_finalize:  eight lanes per source, eight sources per wave: each lane sums one box's
//                 items in order and applies the chain rule to the 27 parameters; a fixed
//                 butterfly over the eight lanes sums the boxes, then the KL term is added.
// Table entries are addressed with wave-uniform indices so the compiler serves them
// through scalar loads; pixel data is read coalesced along box rows.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "model.h"

namespace cel {

// ----------------------------------------------------------------------- validation
// Domain of a source row: finite; q in (0,1); frac_dev in [0,1]; axis ratio in (0,1];
// radius > 0; variances > 0; with the colour-prior mixture (npar = NPK) every
// responsibility positive and each type's eight summing to 1 within 1e-9.  Branch-free so
// that the row's loads issue together.
__device__ inline bool row_ok(const double* __restrict__ p, int npar) {
    double v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) v[i] = p[i];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NP; ++i) ok &= (bool)isfinite(v[i]);
    if (npar == NPK) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            double sum = 0.0;
#pragma unroll
            for (int d = 0; d < NMIX; ++d) {
                const double k = p[NP + NMIX * t + d];
                ok &= k > 0.0 && k <= 1.0;
                sum += k;
            }
            ok &= fabs(sum - 1.0) <= 1e-9;
        }
    }
    ok &= v[6] > 0.0 && v[6] < 1.0;
    ok &= v[2] >= 0.0 && v[2] <= 1.0;
    ok &= v[3] > 0.0 && v[3] <= 1.0;
    ok &= v[5] > 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int base = 7 + 10 * t;
        ok &= v[base + 1] > 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) ok &= v[base + 6 + k] > 0.0;
    }
    return ok;
}

// One thread per listed source; the status word was cleared by the launcher's fill.
__global__ void __launch_bounds__(256) k_validate(const double* __restrict__ theta, const uint8_t* active,
                                                  const int32_t* list, int n, int S, int npar, int* status) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int s = list ? list[j] : j;
    bool bad;
    if (s < 0 || s >= S) bad = true;
    else if (active && !active[s]) bad = false;
    else bad = !row_ok(theta + (size_t)s * ROW, npar);
    if (bad) atomicOr(status, CELESTE_EDOMAIN);
}

// ----------------------------------------------------------------------- prep
// One wave per box, four boxes per block.  The boxes' intermediates (brightness factors,
// shape, PSF terms) are computed first by lanes 0..3 of the first wave, one box per lane,
// and passed through LDS (one wave pass for the block's four boxes instead of four);
// then lane c of each wave writes table entry c of its box and lane NCOMP the four
// brightness coefficients.
template <class T>
__global__ void __launch_bounds__(256) k_prep(PrepArgs a) {
    if (*a.status) return;
    // the box's table is staged in LDS and written out contiguously by the whole wave
    constexpr int TW = NCOMP * CST * scalar_traits<T>::width;   // doubles per table
    __shared__ double stage[4][TW];
    __shared__ T wsh[4][NW];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    if (threadIdx.x < wpb) {   // box of wave threadIdx.x
        const int jb = blockIdx.x * wpb + threadIdx.x;
        if (jb < a.pairs.n) {
            const PairDev pd = a.g.pairs[sel_at(a.pairs, jb)];
            const celeste_image& im = a.g.images[pd.img];
            T* w = wsh[threadIdx.x];
            if (a.dir_mode == DIR_W) {
                // tangent along one of the box's intermediates
                double p[NP], wd[NW];
                for (int i = 0; i < NP; ++i) p[i] = a.theta[(size_t)pd.src * ROW + i];
                pair_w<double>(p, im, wd);
                for (int i = 0; i < NW; ++i) w[i] = scalar_traits<T>::make(wd[i], i == a.dir_unit ? 1.0 : 0.0);
            } else {
                T p[NP];
                for (int i = 0; i < NP; ++i) p[i] = seed<T>(a.theta, a.dir, a.dir_mode, a.dir_unit, pd.src, i);
                pair_w<T>(p, im, w);
            }
        }
    }
    __syncthreads();
    const int j = blockIdx.x * wpb + wave;
    const bool valid = j < a.pairs.n;
    const int pi = valid ? sel_at(a.pairs, j) : 0;
    if (valid) {
        const PairDev pd = a.g.pairs[pi];
        const celeste_image& im = a.g.images[pd.img];
        T* coef = reinterpret_cast<T*>(a.coef) + (size_t)pi * NCOEF;
        T w[NW];
        for (int i = 0; i < NW; ++i) w[i] = wsh[wave][i];
        if (lane < NCOMP) {
            build_comp_from_w<T>(w, im, a.g.consts, lane, reinterpret_cast<T*>(stage[wave]) + lane * CST);
        } else if (lane == NCOMP) {
            coef[C_K1] = w[W_K1];
            coef[C_K2] = w[W_K2];
            coef[C_K3] = w[W_K3];
            coef[C_K4] = w[W_K4];
        }
    }
    __syncthreads();
    if (valid) {
        double* out = reinterpret_cast<double*>(a.tab) + (size_t)pi * TW;
        for (int i = lane; i < TW; i += 64) out[i] = stage[wave][i];
    }
}

// ----------------------------------------------------------------------- render
// Tile = (64 / tile_w * RP) rows x tile_w cols; lane l owns rows (l / tile_w) + k * (64 / tile_w),
// k < RP, of column l % tile_w.
template <int RP>
__global__ void __launch_bounds__(256) k_render(RenderArgs a, const TileDev* __restrict__ tiles,
                                                const int32_t* __restrict__ tile_list,
                                                const PairDev* __restrict__ pairs,
                                                const celeste_image* __restrict__ images,
                                                const double* __restrict__ tab, const double* __restrict__ coef,
                                                const double* __restrict__ xs, double* __restrict__ Eout,
                                                double* __restrict__ Vout, double* __restrict__ tile_sums) {
    if (*a.status) return;
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= a.n_tiles) return;
    const TileDev td = tiles[t];
    const celeste_image& im = images[td.img];
    const int rows_per_pass = 64 / a.tile_w;
    const int c = td.c0 + lane % a.tile_w;
    int r[RP];
    bool inside[RP], covered[RP];
    double E[RP], V[RP], px[RP], py[RP];
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        r[k] = td.r0 + lane / a.tile_w + k * rows_per_pass;
        inside[k] = r[k] < im.H && c < im.W;
        covered[k] = false;
        E[k] = inside[k] ? sky_at(im, r[k], c) : im.sky;
        V[k] = 0.0;
        px[k] = (double)c;
        py[k] = (double)r[k];
    }
    for (int j = td.list_begin; j < td.list_end; ++j) {
        const int pi = __builtin_amdgcn_readfirstlane(tile_list[j]);
        const PairDev o = pairs[pi];
        bool in[RP];
        bool any = false;
#pragma unroll
        for (int k = 0; k < RP; ++k) {
            in[k] = inside[k] && r[k] >= o.r0 && r[k] < o.r0 + o.h && c >= o.c0 && c < o.c0 + o.w;
            any |= in[k];
        }
        if (!any) continue;
        double fs[RP], fg[RP];
        eval_value<RP>(tab + (size_t)pi * NCOMP * CST, px, py, fs, fg);
        const double* k4 = coef + (size_t)pi * NCOEF;
        const double k1 = k4[C_K1], k2 = k4[C_K2], k3 = k4[C_K3], kk4 = k4[C_K4];
#pragma unroll
        for (int k = 0; k < RP; ++k) {
            if (!in[k]) continue;
            covered[k] = true;
            const double Et = k1 * fs[k] + k2 * fg[k];
            E[k] += Et;
            V[k] += k3 * fs[k] * fs[k] + kk4 * fg[k] * fg[k] - Et * Et;
        }
    }
    double l = 0.0;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        if (!inside[k]) continue;
        const size_t gi = (size_t)im.pix_offset + (size_t)r[k] * im.W + c;
        Eout[gi] = E[k];
        Vout[gi] = V[k];
        if (tile_sums && covered[k]) {
            const double x = xs[gi];
            if (x == x) {
                double lk = x * (log(E[k]) - 0.5 * V[k] / (E[k] * E[k])) - E[k];
                if (a.g.consts.flags & CELESTE_INCLUDE_LGAMMA) lk -= lgamma(x + 1.0);
                l += lk;
            }
        }
    }
    if (tile_sums) {
        l = wave_sum(l);
        if (lane == 0) tile_sums[t] = l;
    }
}

// ----------------------------------------------------------------------- finalize
// Sum over the FIN_LANES lanes of a lane group (fixed butterfly: every lane of the group
// ends with the same sum).
constexpr int FIN_LANES = 8;
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int o = FIN_LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline dual group_sum(dual v) { return mkd(group_sum(v.v), group_sum(v.t)); }

template <class T>
__global__ void __launch_bounds__(64) k_finalize(FinArgs a) {
    if (*a.status) return;
    const int lane = threadIdx.x & (FIN_LANES - 1);
    const int j = blockIdx.x * (64 / FIN_LANES) + threadIdx.x / FIN_LANES;
    // every lane takes part in the butterflies; groups past the list or inactive write nothing
    const bool listed = j < a.srcs.n;
    const int s = listed ? sel_at(a.srcs, j) : sel_at(a.srcs, 0);
    const bool act = listed && (!a.active || a.active[s]);
    T p[NPK];
    for (int i = 0; i < NPK; ++i) p[i] = seed<T>(a.theta, a.dir, a.dir_mode, a.dir_unit, s, i);
    const T zero = scalar_traits<T>::make(0.0, 0.0);
    T g[NPK];
    for (int i = 0; i < NPK; ++i) g[i] = zero;
    T val = zero;
    const T* part = reinterpret_cast<const T*>(a.partials);
    // lane l of the group takes the source's boxes l, l + FIN_LANES, ...; each box's items in order
    const int pe = act ? a.patch_ptr[s + 1] : 0;
    for (int pi = a.patch_ptr[s] + lane; pi < pe; pi += FIN_LANES) {
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
        if (a.pair_lgamma) val = val - a.pair_lgamma[pi];
        if (a.deriv) chain_pair<T>(p, a.g.images[pd.img], z, g);
    }
    val = group_sum(val);
    if (a.deriv) {
#pragma unroll
        for (int i = 0; i < NP; ++i) g[i] = group_sum(g[i]);
    }
    if (a.g.consts.flags & CELESTE_INCLUDE_KL) {
        T gk[NPK];
        for (int i = 0; i < NPK; ++i) gk[i] = zero;
        val -= kl_source<T>(p, a.g.consts, gk);
        if (a.deriv)
            for (int i = 0; i < NPK; ++i) g[i] += gk[i];
    }
    if (lane != 0 || !act) return;
    if (a.elbo) a.elbo[s] = value_of(val);
    if (a.deriv && a.grad) {
        double* o = a.grad + (size_t)s * ROW;
        for (int i = 0; i < NPK; ++i) o[i] = value_of(g[i]);
        for (int i = NPK; i < ROW; ++i) o[i] = 0.0;
    }
    if (a.deriv && a.tangent) {
        double* o = a.tangent + (size_t)(a.tangent_by_list ? j : s) * a.tangent_stride;
        for (int i = 0; i < NPK; ++i) o[i] = tangent_of(g[i]);
        if (a.tangent_pad)
            for (int i = NPK; i < ROW; ++i) o[i] = 0.0;
    }
}

// Per-box sums of the item partials (fixed order).
__global__ void __launch_bounds__(128) k_pair_reduce(Sel sel, const PairDev* __restrict__ pairs,
                                                     const double* __restrict__ partials,
                                                     const double* __restrict__ kk, int tangent, int dir,
                                                     double* __restrict__ gw, double* __restrict__ hw,
                                                     const int* status) {
    if (*status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sel.n) return;
    const int pi = sel_at(sel, j);
    const PairDev pd = pairs[pi];
    double z[NACC];
    for (int f = 0; f < NACC; ++f) z[f] = 0.0;
    for (int it = pd.item_begin; it < pd.item_end; ++it) {
        if (tangent) {
            const dual* q = reinterpret_cast<const dual*>(partials) + (size_t)it * NACC;
            for (int f = 0; f < NACC; ++f) z[f] += q[f].t;
        } else {
            const double* q = partials + (size_t)it * NACC;
            for (int f = 0; f < NACC; ++f) z[f] += q[f];
        }
    }
    if (tangent) {
        double* o = hw + ((size_t)pi * NW + dir) * NW;
        for (int f = 0; f < NW; ++f) o[f] = z[f + 1];
    } else {
        double* o = gw + (size_t)pi * NACC;
        for (int f = 0; f < NACC; ++f) o[f] = z[f];
        if (kk) {
            // pixel-level block of hw[pair] over (k1..k4, frac_dev), symmetric; (k3, k4) is 0
            double h[NKK_USED];
            for (int f = 0; f < NKK_USED; ++f) h[f] = 0.0;
            for (int it = pd.item_begin; it < pd.item_end; ++it)
                for (int f = 0; f < NKK_USED; ++f) h[f] += kk[(size_t)it * NKK + f];
            const double blk[5][5] = {{h[KK_11], h[KK_12], h[KK_13], h[KK_14], h[KK_F1]},
                                      {h[KK_12], h[KK_22], h[KK_23], h[KK_24], h[KK_F2]},
                                      {h[KK_13], h[KK_23], 0.0, 0.0, h[KK_F3]},
                                      {h[KK_14], h[KK_24], 0.0, 0.0, h[KK_F4]},
                                      {h[KK_F1], h[KK_F2], h[KK_F3], h[KK_F4], h[KK_FF]}};
            const int idx[5] = {W_K1, W_K2, W_K3, W_K4, W_FDEV};
            double* hb = hw + (size_t)pi * NW * NW;
            for (int i = 0; i < 5; ++i)
                for (int f = 0; f < 5; ++f) hb[idx[i] * NW + idx[f]] = blk[i][f];
        }
    }
}

// Position and shape rows of each listed box's intermediate Hessian from the closed-form
// item sums: hw[dir][f] = (entry between dir and f) / c_dir, the entries being in the
// accumulator scaling c_dir c_f d2L / dw_dir dw_f (c = 2 for Sxx, Syy).
__global__ void __launch_bounds__(128) k_pair_hess(Sel sel, const PairDev* __restrict__ pairs,
                                                   const double* __restrict__ hg, double* __restrict__ hw,
                                                   const int* status) {
    if (*status) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sel.n) return;
    const int pi = sel_at(sel, j);
    const PairDev pd = pairs[pi];
    double h[NHG];
    for (int f = 0; f < NHG; ++f) h[f] = 0.0;
    for (int it = pd.item_begin; it < pd.item_end; ++it)
        for (int f = 0; f < NHG; ++f) h[f] += hg[(size_t)it * NHG + f];
    // geometric index of each intermediate (-1: brightness factor)
    const int geo[NW] = {-1, -1, -1, -1, 0, 1, 2, 3, 4, 5};
    double* o = hw + (size_t)pi * NW * NW;
    for (int q = 0; q < 5; ++q) {
        const int dir = q < 2 ? W_UX + q : W_SXX + (q - 2);
        const double inv_c = (dir == W_SXX || dir == W_SYY) ? 0.5 : 1.0;
        const int gd = geo[dir];
        for (int f = 0; f < NW; ++f) {
            double v;
            if (f < 4) {
                v = h[NHG_GEO + 4 * q + f];
            } else {
                const int gf = geo[f];
                const int lo = gd < gf ? gd : gf, hi = gd < gf ? gf : gd;
                int e = 0;
                while (e < NHG_GEO && !(hg_row(e) == lo && hg_col(e) == hi)) ++e;
                v = h[e];
            }
            o[dir * NW + f] = v * inv_c;
        }
    }
}

// Hessian of ELBO_s: column d is the tangent, along parameter d, of the chain rule
// J^T z applied to the pair gradients z (value gw, tangent hw * (dw / dtheta_d)), plus the
// KL term.  One thread per (listed source, direction); npar (NP, or NPK with the colour-prior
// mixture, whose responsibilities enter the KL only) rows and columns per source.
__global__ void __launch_bounds__(128) k_assemble_hessian(Sel srcs, Geometry g, const int32_t* __restrict__ patch_ptr,
                                                          const double* __restrict__ theta,
                                                          const double* __restrict__ gw,
                                                          const double* __restrict__ hw,
                                                          double* __restrict__ hess, const int* status) {
    if (*status) return;
    const int npar = g.consts.npar;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= srcs.n * npar) return;
    const int j = t / npar, d = t - j * npar;
    const int s = sel_at(srcs, j);
    dual p[NPK], gh[NPK];
    for (int i = 0; i < NPK; ++i) {
        p[i] = mkd(theta[(size_t)s * ROW + i], i == d ? 1.0 : 0.0);
        gh[i] = mkd(0.0, 0.0);
    }
    for (int pi = patch_ptr[s]; pi < patch_ptr[s + 1]; ++pi) {
        const celeste_image& im = g.images[g.pairs[pi].img];
        dual w[NW];
        pair_w<dual>(p, im, w);
        dual z[NACC];
        const double* gz = gw + (size_t)pi * NACC;
        const double* h = hw + (size_t)pi * NW * NW;
        z[A_VAL] = mkd(gz[A_VAL], 0.0);
        for (int a = 0; a < NW; ++a) {
            double tz = 0.0;
            // hw[dir][f] = c_f d2L / dw_dir dw_f with c = 2 for the A_SXX, A_SYY accumulators
            // and 1 otherwise.  The pixel-level rows (brightness factors, frac_dev) hold only
            // their own block; the rest of such a row is c_a times the symmetric entry of the
            // tangent pass along a.
            for (int i = 0; i < NW; ++i) {
                const bool pix_i = i < 4 || i == W_FDEV, pix_a = a < 4 || a == W_FDEV;
                const double hia = (pix_i && !pix_a) ? (a == W_SXX || a == W_SYY ? 2.0 : 1.0) * h[a * NW + i]
                                                     : h[i * NW + a];
                tz += hia * w[i].t;
            }
            z[a + 1] = mkd(gz[a + 1], tz);
        }
        chain_pair<dual>(p, im, z, gh);
    }
    if (g.consts.flags & CELESTE_INCLUDE_KL) kl_source<dual>(p, g.consts, gh);
    double* o = hess + (size_t)j * npar * npar + (size_t)d * npar;
    for (int i = 0; i < npar; ++i) o[i] = gh[i].t;
}

// Total ELBO: a fixed-order two-level sum.  Block b of k_total_partial sums its contiguous
// slices of the per-tile pixel sums and of the sources' KL terms (a fixed tree per block) into
// part[b]; k_total_final sums the TT_BLOCKS partials in block order.  Deterministic, and
// spread over the chip instead of one work-group.
constexpr int TT_THREADS = 256;
constexpr int TT_BLOCKS = 1024;

__device__ inline double block_sum_256(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = TT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(TT_THREADS) k_total_partial(const double* __restrict__ tile_sums, int n_tiles,
                                                              const double* __restrict__ theta, Consts K, int S,
                                                              double* __restrict__ part, const int* status) {
    if (*status) return;
    __shared__ double red[TT_THREADS];
    const int b = blockIdx.x;
    const int t0 = (int)((int64_t)n_tiles * b / TT_BLOCKS), t1 = (int)((int64_t)n_tiles * (b + 1) / TT_BLOCKS);
    double acc = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += TT_THREADS) acc += tile_sums[t];
    if (K.flags & CELESTE_INCLUDE_KL) {
        const int s0 = (int)((int64_t)S * b / TT_BLOCKS), s1 = (int)((int64_t)S * (b + 1) / TT_BLOCKS);
        for (int s = s0 + threadIdx.x; s < s1; s += TT_THREADS) {
            double p[NPK], g[NPK];
            for (int i = 0; i < NPK; ++i) { p[i] = theta[(size_t)s * ROW + i]; g[i] = 0.0; }
            acc -= kl_source<double>(p, K, g);
        }
    }
    const double v = block_sum_256(acc, red);
    if (threadIdx.x == 0) part[b] = v;
}

__global__ void __launch_bounds__(TT_THREADS) k_total_final(const double* __restrict__ part, double* out,
                                                            const int* status) {
    if (*status) return;
    __shared__ double red[TT_THREADS];
    double acc = 0.0;
    for (int b = threadIdx.x; b < TT_BLOCKS; b += TT_THREADS) acc += part[b];
    const double v = block_sum_256(acc, red);
    if (threadIdx.x == 0) out[0] = v;
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
                           int S, int npar, int* status, hipStream_t st) {
    const hipError_t e = launch_fill_int(status, 0, 1, st);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_validate, dim3((n + 255) / 256), dim3(256), 0, st, theta, active, list, n, S, npar,
                       status);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs& a, bool tangent, hipStream_t st) {
    if (a.pairs.n <= 0) return hipSuccess;
    const dim3 grid((a.pairs.n + 3) / 4);
    if (tangent) hipLaunchKernelGGL(k_prep<dual>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_prep<double>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs& a, int wpb, hipStream_t st) {
    if (a.n_tiles <= 0) return hipSuccess;
    const dim3 grid((a.n_tiles + wpb - 1) / wpb);
    const int rp = a.tile_h * a.tile_w / 64;
    const Geometry& g = a.g;
#define RENDER_ARGS a, a.tiles, a.tile_list, g.pairs, g.images, a.tab, a.coef, g.x, a.E, a.V, a.tile_sums
    if (rp == 1) hipLaunchKernelGGL(k_render<1>, grid, dim3(64 * wpb), 0, st, RENDER_ARGS);
    else if (rp == 2) hipLaunchKernelGGL(k_render<2>, grid, dim3(64 * wpb), 0, st, RENDER_ARGS);
    else if (rp == 4) hipLaunchKernelGGL(k_render<4>, grid, dim3(64 * wpb), 0, st, RENDER_ARGS);
    else return hipErrorInvalidValue;
#undef RENDER_ARGS
    return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, bool tangent, hipStream_t st) {
    if (a.srcs.n <= 0) return hipSuccess;
    const dim3 grid((a.srcs.n + 64 / FIN_LANES - 1) / (64 / FIN_LANES));
    if (tangent) hipLaunchKernelGGL(k_finalize<dual>, grid, dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_finalize<double>, grid, dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tile_total(const double* tile_sums, int n_tiles, const double* theta, const Consts& c,
                             int S, double* part, double* out, const int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_total_partial, dim3(TT_BLOCKS), dim3(TT_THREADS), 0, st, tile_sums, n_tiles, theta, c, S,
                       part, status);
    hipLaunchKernelGGL(k_total_final, dim3(1), dim3(TT_THREADS), 0, st, part, out, status);
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

hipError_t launch_pair_reduce(const Sel& sel, const PairDev* dpairs, const double* partials, const double* kk,
                              bool tangent, int dir, double* gw, double* hw, const int* status, hipStream_t st) {
    if (sel.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_reduce, dim3((sel.n + 127) / 128), dim3(128), 0, st, sel, dpairs, partials, kk,
                       tangent ? 1 : 0, dir, gw, hw, status);
    return hipGetLastError();
}

hipError_t launch_pair_hess(const Sel& sel, const PairDev* dpairs, const double* hg, double* hw, const int* status,
                            hipStream_t st) {
    if (sel.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_hess, dim3((sel.n + 127) / 128), dim3(128), 0, st, sel, dpairs, hg, hw, status);
    return hipGetLastError();
}

hipError_t launch_assemble_hessian(const Sel& srcs, const Geometry& g, const int32_t* patch_ptr, const double* theta,
                                   const double* gw, const double* hw, double* hess, const int* status,
                                   hipStream_t st) {
    if (srcs.n <= 0) return hipSuccess;
    const int n = srcs.n * g.consts.npar;
    hipLaunchKernelGGL(k_assemble_hessian, dim3((n + 127) / 128), dim3(128), 0, st, srcs, g, patch_ptr, theta, gw,
                       hw, hess, status);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace cel
