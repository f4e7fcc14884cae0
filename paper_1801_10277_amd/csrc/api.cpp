// Host side of libceleste: plan construction (validation, box binning, work items,
// overlap lists), the C entry points, HIP graph capture of the batched evaluation, the
// launch-configuration autotuner, conflict-free batching and the sweep loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "celeste.h"
#include "internal.h"

using namespace cel;

namespace {

thread_local std::string g_hip_error;

int hip_fail(hipError_t e, const char* what) {
    g_hip_error = std::string(what) + ": " + hipGetErrorString(e);
    return CELESTE_EHIP;
}

#define HIPCHK(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hip_fail(e_, #call);       \
    } while (0)

template <class T>
int dalloc(T** p, size_t n, size_t& total) {
    *p = nullptr;
    if (n == 0) n = 1;
    const size_t bytes = n * sizeof(T);
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        *p = nullptr;
        return CELESTE_ENOMEM;
    }
    total += bytes;
    return CELESTE_OK;
}

bool finite(double v) { return std::isfinite(v); }

}  // namespace

struct celeste_plan {
    int device = 0;
    int n_img = 0, n_src = 0;
    int64_t n_pix = 0, n_visits = 0;
    std::vector<celeste_image> images;
    std::vector<int32_t> patch_ptr;
    std::vector<PairDev> pairs;
    std::vector<Item> items;
    std::vector<int32_t> nbr;
    std::vector<TileDev> tiles;
    std::vector<int32_t> tile_list;
    Consts consts{};
    const double* d_x = nullptr;
    int n_cu = 256;

    // launch configuration
    int chunk = 64, wpb = 4, grid = 0, dynamic = 0, tile_h = 16, tile_w = 16, rows = 16;
    // 0: strips per conflict-free class, 1: binned tiles, 2: stored values + tile gather,
    // 3: stored values, background gathered inside the fused adjoint (no planes)
    int render_mode = 2;
    bool use_graph = false;

    // device memory
    celeste_image* d_images = nullptr;
    PairDev* d_pairs = nullptr;
    Item* d_items = nullptr;
    size_t cap_items = 0;
    int32_t* d_nbr = nullptr;
    TileDev* d_tiles = nullptr;
    size_t cap_tiles = 0;
    int32_t* d_tile_list = nullptr;
    size_t cap_tile_list = 0;
    int32_t* d_patch_ptr = nullptr;
    double* d_tab1 = nullptr;    // double tables
    double* d_coef1 = nullptr;
    double* d_tab2 = nullptr;    // dual tables
    double* d_coef2 = nullptr;
    double* d_partials = nullptr;
    double* d_kk = nullptr;          // [cap_items][NKK] brightness-factor Hessian blocks
    double* d_hg = nullptr;          // [cap_items][NHG] closed-form position / shape Hessian blocks
    double* d_nu = nullptr;          // [NGAL] nu of each galaxy component (closed-form pass)
    int hess_mode = 0;               // 0: closed-form block pass, 1: tangent passes of the adjoint
    double* d_E = nullptr;
    double* d_V = nullptr;
    double* d_bg = nullptr;
    double* d_fg = nullptr;      // [n_visits][2] own profile values (render mode 2)
    bool fg_valid = false;       // d_fg holds the values of the last render
    double* d_tile_sums = nullptr;
    double* d_pair_lgamma = nullptr;
    int* d_status = nullptr;
    double* d_mix = nullptr;     // [2][NMIX][MIXF] colour-prior mixture table, or null
    int* d_counter = nullptr;
    unsigned long long* d_wcount = nullptr;   // [NLIVE_COUNTS] celeste_work_counts
    double* d_grad = nullptr;
    double* d_hess = nullptr;        // [S][npar][npar]
    double* d_grad_trial = nullptr;  // gradient and Hessian at the Newton trial points
    double* d_hess_trial = nullptr;
    uint8_t* d_accepted = nullptr;
    uint8_t* d_live = nullptr;
    double* d_gw = nullptr;      // [n_pairs][11] per-box gradient sums
    double* d_hw = nullptr;      // [n_pairs][10][10] per-box Hessian of the pixel part w.r.t. its intermediates
    double* d_theta_trial = nullptr;
    double* d_pred = nullptr;
    double* d_elbo_cur = nullptr;
    double* d_elbo_trial = nullptr;
    double* d_radius = nullptr;
    uint8_t* d_done = nullptr;
    int32_t* d_list_src = nullptr;   // [n_src]
    int32_t* d_list_pair = nullptr;  // [n_pairs]
    int32_t* d_list_item = nullptr;  // [cap_items]
    int32_t* d_list_npair = nullptr; // [n_pairs] boxes whose stored values a Newton call renders
    int32_t* d_list_nitem = nullptr; // [max_items] their items
    size_t cap_list_item = 0, cap_list_src = 0, cap_list_pair = 0;
    // conflict-free classes of boxes (no two boxes of a class share a pixel) and their items
    std::vector<int32_t> pair_class;
    int n_class = 0;
    std::vector<int32_t> cls_ptr, cls_items;
    int32_t* d_cls_items = nullptr;
    int max_pix = 0;
    size_t workspace = 0;

    // phase timing of the batched sequence
    bool profiling = false;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double phase_ms[4] = {0, 0, 0, 0};
    int64_t phase_calls = 0;

    // pinned host staging of the source / box / item lists, uploaded on the caller's stream;
    // stage_ev marks the end of the last upload (the staging may be rewritten after it)
    int32_t* h_stage = nullptr;
    size_t cap_stage = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    // sweep graph: one sweep over a schedule captured once per celeste_sweep call and replayed
    hipGraphExec_t sweep_exec = nullptr;
    hipEvent_t sweep_ev = nullptr;   // recorded after the last replay
    bool sweep_pending = false;
    double* d_scalar = nullptr;      // total ELBO written by a replayed sweep
    double* d_tt_part = nullptr;     // [1024] partial sums of the total ELBO

    // graph cache of the batched elbo_grad sequence
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gkey[4] = {nullptr, nullptr, nullptr, nullptr};
    int gkey_cfg = -1;

    Geometry geom() const {
        Geometry g;
        g.images = d_images;
        g.pairs = d_pairs;
        g.items = d_items;
        g.nbr = d_nbr;
        g.x = d_x;
        g.consts = consts;
        return g;
    }
    int64_t n_pairs() const { return (int64_t)pairs.size(); }
    int launch_grid() const { return grid > 0 ? grid : 64 * n_cu; }
};

namespace {

// ---------------------------------------------------------------- geometry builders

// Work items: runs of up to `chunk` strips (a strip = `rows` consecutive pixels of one
// column of a box), in box order.
int64_t strips_of(const PairDev& pd, int rows) { return (int64_t)pd.w * ((pd.h + rows - 1) / rows); }

void build_items(celeste_plan* p) {
    p->items.clear();
    for (size_t i = 0; i < p->pairs.size(); ++i) {
        PairDev& pd = p->pairs[i];
        const int n = (int)strips_of(pd, p->rows);
        pd.item_begin = (int32_t)p->items.size();
        for (int s = 0; s < n; s += p->chunk) {
            Item it;
            it.pair = (int32_t)i;
            it.start = s;
            it.count = std::min(p->chunk, n - s);
            it.pad = 0;
            p->items.push_back(it);
        }
        pd.item_end = (int32_t)p->items.size();
    }
}

// Greedy colouring of the box-overlap graph (largest boxes first): boxes of one class
// never share a pixel, so a class can add its light to the planes without atomics.
void build_pair_classes(celeste_plan* p) {
    const size_t n = p->pairs.size();
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)p->pairs[a].h * p->pairs[a].w > (int64_t)p->pairs[b].h * p->pairs[b].w;
    });
    p->pair_class.assign(n, -1);
    p->n_class = 0;
    std::vector<int32_t> mark;
    for (int32_t i : order) {
        const PairDev& pd = p->pairs[i];
        for (int k = pd.nbr_begin; k < pd.nbr_end; ++k) {
            const int c = p->pair_class[p->nbr[k]];
            if (c >= 0) {
                if ((int)mark.size() <= c) mark.resize(c + 1, -1);
                mark[c] = i;
            }
        }
        int c = 0;
        while (c < (int)mark.size() && mark[c] == i) ++c;
        p->pair_class[i] = c;
        p->n_class = std::max(p->n_class, c + 1);
    }
}

void build_class_items(celeste_plan* p) {
    p->cls_ptr.assign(p->n_class + 1, 0);
    for (size_t i = 0; i < p->pairs.size(); ++i)
        p->cls_ptr[p->pair_class[i] + 1] += p->pairs[i].item_end - p->pairs[i].item_begin;
    for (int c = 0; c < p->n_class; ++c) p->cls_ptr[c + 1] += p->cls_ptr[c];
    p->cls_items.assign(p->items.size(), 0);
    std::vector<int32_t> fill(p->cls_ptr.begin(), p->cls_ptr.end() - 1);
    for (size_t i = 0; i < p->pairs.size(); ++i)
        for (int it = p->pairs[i].item_begin; it < p->pairs[i].item_end; ++it)
            p->cls_items[fill[p->pair_class[i]]++] = it;
}

void build_tiles(celeste_plan* p) {
    const int th = p->tile_h, tw = p->tile_w;
    std::vector<std::vector<int32_t>> per_img_pairs(p->n_img);
    for (size_t i = 0; i < p->pairs.size(); ++i) per_img_pairs[p->pairs[i].img].push_back((int32_t)i);
    p->tiles.clear();
    p->tile_list.clear();
    for (int n = 0; n < p->n_img; ++n) {
        const celeste_image& im = p->images[n];
        const int ntr = (im.H + th - 1) / th, ntc = (im.W + tw - 1) / tw;
        std::vector<int32_t> cnt((size_t)ntr * ntc, 0);
        for (int32_t pi : per_img_pairs[n]) {
            const PairDev& pd = p->pairs[pi];
            for (int tr = pd.r0 / th; tr <= (pd.r0 + pd.h - 1) / th; ++tr)
                for (int tc = pd.c0 / tw; tc <= (pd.c0 + pd.w - 1) / tw; ++tc) cnt[(size_t)tr * ntc + tc]++;
        }
        std::vector<int64_t> start(cnt.size(), -1);
        const size_t base_tile = p->tiles.size();
        int64_t off = (int64_t)p->tile_list.size();
        for (size_t t = 0; t < cnt.size(); ++t) {
            if (!cnt[t]) continue;
            TileDev td;
            td.img = n;
            td.r0 = (int)(t / ntc) * th;
            td.c0 = (int)(t % ntc) * tw;
            td.list_begin = (int32_t)off;
            td.list_end = (int32_t)(off + cnt[t]);
            td.pad = 0;
            start[t] = (int64_t)(p->tiles.size() - base_tile);
            p->tiles.push_back(td);
            off += cnt[t];
        }
        p->tile_list.resize(off);
        std::vector<int32_t> fill(p->tiles.size() - base_tile, 0);
        for (int32_t pi : per_img_pairs[n]) {   // ascending pair order inside every tile
            const PairDev& pd = p->pairs[pi];
            for (int tr = pd.r0 / th; tr <= (pd.r0 + pd.h - 1) / th; ++tr)
                for (int tc = pd.c0 / tw; tc <= (pd.c0 + pd.w - 1) / tw; ++tc) {
                    const int64_t k = start[(size_t)tr * ntc + tc];
                    TileDev& td = p->tiles[base_tile + k];
                    p->tile_list[td.list_begin + fill[k]++] = pi;
                }
        }
    }
}

bool boxes_intersect(const PairDev& a, const PairDev& b) {
    return a.r0 < b.r0 + b.h && b.r0 < a.r0 + a.h && a.c0 < b.c0 + b.w && b.c0 < a.c0 + a.w;
}

void build_nbr(celeste_plan* p) {
    const int cell = 128;
    p->nbr.clear();
    std::vector<std::vector<int32_t>> per_img(p->n_img);
    for (size_t i = 0; i < p->pairs.size(); ++i) per_img[p->pairs[i].img].push_back((int32_t)i);
    std::vector<std::vector<int32_t>> lists(p->pairs.size());
    for (int n = 0; n < p->n_img; ++n) {
        const celeste_image& im = p->images[n];
        const int nr = (im.H + cell - 1) / cell, nc = (im.W + cell - 1) / cell;
        std::vector<std::vector<int32_t>> cells((size_t)nr * nc);
        for (int32_t pi : per_img[n]) {
            const PairDev& pd = p->pairs[pi];
            for (int r = pd.r0 / cell; r <= (pd.r0 + pd.h - 1) / cell; ++r)
                for (int c = pd.c0 / cell; c <= (pd.c0 + pd.w - 1) / cell; ++c)
                    cells[(size_t)r * nc + c].push_back(pi);
        }
        for (int32_t pi : per_img[n]) {
            const PairDev& pd = p->pairs[pi];
            std::vector<int32_t>& L = lists[pi];
            for (int r = pd.r0 / cell; r <= (pd.r0 + pd.h - 1) / cell; ++r)
                for (int c = pd.c0 / cell; c <= (pd.c0 + pd.w - 1) / cell; ++c)
                    for (int32_t qi : cells[(size_t)r * nc + c])
                        if (qi != pi && boxes_intersect(pd, p->pairs[qi])) L.push_back(qi);
            std::sort(L.begin(), L.end());
            L.erase(std::unique(L.begin(), L.end()), L.end());
        }
    }
    for (size_t i = 0; i < p->pairs.size(); ++i) {
        p->pairs[i].nbr_begin = (int32_t)p->nbr.size();
        p->nbr.insert(p->nbr.end(), lists[i].begin(), lists[i].end());
        p->pairs[i].nbr_end = (int32_t)p->nbr.size();
    }
}

int upload_geometry(celeste_plan* p) {
    HIPCHK(hipMemcpy(p->d_pairs, p->pairs.data(), p->pairs.size() * sizeof(PairDev), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_items, p->items.data(), p->items.size() * sizeof(Item), hipMemcpyHostToDevice));
    if (!p->cls_items.empty())
        HIPCHK(hipMemcpy(p->d_cls_items, p->cls_items.data(), p->cls_items.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_tiles, p->tiles.data(), p->tiles.size() * sizeof(TileDev), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_tile_list, p->tile_list.data(), p->tile_list.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    return CELESTE_OK;
}

void drop_graph(celeste_plan* p) {
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    p->gkey_cfg = -1;
}

// ---------------------------------------------------------------- validation
// Every sky-map entry finite and > 0 (a synchronous copy of each map; plan creation only).
int validate_sky_maps(const celeste_problem_desc* d) {
    std::vector<double> buf;
    for (int n = 0; n < d->n_img; ++n) {
        const celeste_image& im = d->images[n];
        if (!im.sky_map) continue;
        buf.resize((size_t)im.H * im.W);
        HIPCHK(hipMemcpy(buf.data(), im.sky_map, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (double v : buf)
            if (!(v > 0.0) || !finite(v)) return CELESTE_EINVAL;
    }
    return CELESTE_OK;
}

// Colour-prior mixture table [2][NMIX][MIXF] (weight, log weight, mean, precision, log det)
// from the problem description: every weight positive and each type's summing to 1 within
// 1e-9, finite means, covariances symmetric and positive definite (a Cholesky factor with
// positive pivots, whose columns give the precision).  CELESTE_EINVAL otherwise.
int mixture_table(const celeste_problem_desc* d, double* tab) {
    for (int t = 0; t < 2; ++t) {
        double wsum = 0.0;
        for (int c = 0; c < NMIX; ++c) {
            const double w = d->color_mix_w[t][c];
            if (!(w > 0.0) || !finite(w)) return CELESTE_EINVAL;
            wsum += w;
            double* e = tab + (t * NMIX + c) * MIXF;
            for (int f = 0; f < MIXF; ++f) e[f] = 0.0;
            e[MX_W] = w;
            e[MX_LOGW] = std::log(w);
            const double(&S)[4][4] = d->color_mix_cov[t][c];
            for (int k = 0; k < 4; ++k) {
                if (!finite(d->color_mix_mean[t][c][k])) return CELESTE_EINVAL;
                e[MX_MEAN + k] = d->color_mix_mean[t][c][k];
                for (int l = 0; l < 4; ++l) {
                    if (!finite(S[k][l])) return CELESTE_EINVAL;
                    if (std::fabs(S[k][l] - S[l][k]) > 1e-12 * (std::fabs(S[k][l]) + std::fabs(S[l][k])))
                        return CELESTE_EINVAL;
                }
            }
            double L[4][4] = {};
            double logdet = 0.0;
            for (int j = 0; j < 4; ++j) {
                double v = S[j][j];
                for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
                if (!(v > 0.0)) return CELESTE_EINVAL;
                L[j][j] = std::sqrt(v);
                logdet += 2.0 * std::log(L[j][j]);
                for (int i = j + 1; i < 4; ++i) {
                    double u = S[i][j];
                    for (int k = 0; k < j; ++k) u -= L[i][k] * L[j][k];
                    L[i][j] = u / L[j][j];
                }
            }
            for (int col = 0; col < 4; ++col) {   // S^-1 e_col = L^-T L^-1 e_col
                double y[4], x[4];
                for (int i = 0; i < 4; ++i) {
                    double u = i == col ? 1.0 : 0.0;
                    for (int k = 0; k < i; ++k) u -= L[i][k] * y[k];
                    y[i] = u / L[i][i];
                }
                for (int i = 3; i >= 0; --i) {
                    double u = y[i];
                    for (int k = i + 1; k < 4; ++k) u -= L[k][i] * x[k];
                    x[i] = u / L[i][i];
                }
                for (int i = 0; i < 4; ++i) e[MX_P + 4 * i + col] = x[i];
            }
            e[MX_LOGDET] = logdet;
        }
        if (!(std::fabs(wsum - 1.0) <= 1e-9)) return CELESTE_EINVAL;
    }
    return CELESTE_OK;
}

int validate_desc(const celeste_problem_desc* d) {
    if (!d || d->n_img <= 0 || d->n_src <= 0 || !d->images || !d->x || !d->patch_ptr || d->n_pix <= 0)
        return CELESTE_EINVAL;
    if (d->flags & ~(uint32_t)(CELESTE_INCLUDE_KL | CELESTE_INCLUDE_LGAMMA | CELESTE_COLOR_MIXTURE))
        return CELESTE_EINVAL;
    for (int n = 0; n < d->n_img; ++n) {
        const celeste_image& im = d->images[n];
        if (im.band < 0 || im.band > 4 || im.H <= 0 || im.W <= 0 || im.pix_offset < 0) return CELESTE_EINVAL;
        if ((int64_t)im.H * im.W >= ((int64_t)1 << 29)) return CELESTE_EINVAL;   // 32-bit byte offsets
        if (im.pix_offset + (int64_t)im.H * im.W > d->n_pix) return CELESTE_EINVAL;
        if (!(im.sky > 0.0) || !finite(im.sky) || !(im.iota > 0.0) || !finite(im.iota)) return CELESTE_EINVAL;
        if (!finite(im.origin_x) || !finite(im.origin_y)) return CELESTE_EINVAL;
        {
            const double a = im.wcs[0][0], b = im.wcs[0][1], c = im.wcs[1][0], e = im.wcs[1][1];
            if (!finite(a) || !finite(b) || !finite(c) || !finite(e)) return CELESTE_EINVAL;
            const double mx = std::max(std::max(std::fabs(a), std::fabs(b)), std::max(std::fabs(c), std::fabs(e)));
            if (!(std::fabs(a * e - b * c) >= 1e-6 * mx * mx)) return CELESTE_EINVAL;   // invertible
        }
        for (int k = 0; k < NPSF; ++k) {
            const double* ps = im.psf[k];
            for (int f = 0; f < 6; ++f)
                if (!finite(ps[f])) return CELESTE_EINVAL;
            if (!(ps[0] > 0.0) || !(ps[3] > 0.0) || !(ps[5] > 0.0) || !(ps[3] * ps[5] - ps[4] * ps[4] > 0.0))
                return CELESTE_EINVAL;
            // smallest eigenvalue of the PSF covariance >= 0.01 px^2 (sigma >= 0.1 px)
            const double tr = ps[3] + ps[5], df = ps[3] - ps[5];
            if (!(0.5 * (tr - std::sqrt(df * df + 4.0 * ps[4] * ps[4])) >= 0.01)) return CELESTE_EINVAL;
        }
    }
    if (d->patch_ptr[0] != 0) return CELESTE_EINVAL;
    for (int s = 0; s < d->n_src; ++s)
        if (d->patch_ptr[s + 1] < d->patch_ptr[s]) return CELESTE_EINVAL;
    const int nb = d->patch_ptr[d->n_src];
    if (nb > 0 && !d->boxes) return CELESTE_EINVAL;
    for (int s = 0; s < d->n_src; ++s) {
        for (int b = d->patch_ptr[s]; b < d->patch_ptr[s + 1]; ++b) {
            const celeste_box& bx = d->boxes[b];
            if (bx.img < 0 || bx.img >= d->n_img) return CELESTE_EINVAL;
            const celeste_image& im = d->images[bx.img];
            if (bx.h <= 0 || bx.w <= 0 || bx.r0 < 0 || bx.c0 < 0 || bx.r0 + bx.h > im.H || bx.c0 + bx.w > im.W)
                return CELESTE_EINVAL;
            if ((int64_t)bx.h * bx.w >= ((int64_t)1 << 28)) return CELESTE_EINVAL;   // 32-bit byte offsets
            for (int b2 = d->patch_ptr[s]; b2 < b; ++b2)
                if (d->boxes[b2].img == bx.img) return CELESTE_EINVAL;
        }
    }
    for (int j = 0; j < NEXP; ++j)
        if (!(d->exp_alpha[j] > 0.0) || !(d->exp_nu[j] > 0.0) || !finite(d->exp_nu[j])) return CELESTE_EINVAL;
    for (int j = 0; j < NDEV; ++j)
        if (!(d->dev_alpha[j] > 0.0) || !(d->dev_nu[j] > 0.0) || !finite(d->dev_nu[j])) return CELESTE_EINVAL;
    if (d->flags & CELESTE_COLOR_MIXTURE) {
        double tab[2 * NMIX * MIXF];
        if (mixture_table(d, tab) != CELESTE_OK) return CELESTE_EINVAL;
    }
    if (!(d->prior_phi > 0.0 && d->prior_phi < 1.0)) return CELESTE_EINVAL;
    for (int t = 0; t < 2; ++t) {
        if (!finite(d->prior_r[t][0]) || !(d->prior_r[t][1] > 0.0)) return CELESTE_EINVAL;
        for (int k = 0; k < 4; ++k)
            if (!finite(d->prior_c[t][0][k]) || !(d->prior_c[t][1][k] > 0.0)) return CELESTE_EINVAL;
    }
    return CELESTE_OK;
}

// ---------------------------------------------------------------- launch helpers
struct Scope {
    Sel src, pair, item;
};

Scope scope_all(const celeste_plan* p) {
    Scope s;
    s.src = Sel{nullptr, 0, p->n_src};
    s.pair = Sel{nullptr, 0, (int32_t)p->pairs.size()};
    s.item = Sel{nullptr, 0, (int32_t)p->items.size()};
    return s;
}

Scope scope_source(const celeste_plan* p, int s) {
    Scope sc;
    const int pb = p->patch_ptr[s], pe = p->patch_ptr[s + 1];
    sc.src = Sel{nullptr, s, 1};
    sc.pair = Sel{nullptr, pb, pe - pb};
    const int ib = pb < pe ? p->pairs[pb].item_begin : 0;
    const int ie = pb < pe ? p->pairs[pe - 1].item_end : 0;
    sc.item = Sel{nullptr, ib, ie - ib};
    return sc;
}

int prep(celeste_plan* p, const double* theta, const Sel& pairs, bool tangent, int dir_mode,
         const double* dir, int dir_unit, hipStream_t st) {
    PrepArgs a{};
    a.g = p->geom();
    a.theta = theta;
    a.dir = dir;
    a.dir_mode = dir_mode;
    a.dir_unit = dir_unit;
    a.pairs = pairs;
    a.tab = tangent ? p->d_tab2 : p->d_tab1;
    a.coef = tangent ? p->d_coef2 : p->d_coef1;
    a.status = p->d_status;
    HIPCHK(launch_prep(a, tangent, st));
    return CELESTE_OK;
}

int render_tiles(celeste_plan* p, bool sums, hipStream_t st) {
    RenderArgs a{};
    a.g = p->geom();
    a.tiles = p->d_tiles;
    a.tile_list = p->d_tile_list;
    a.n_tiles = (int32_t)p->tiles.size();
    a.tile_h = p->tile_h;
    a.tile_w = p->tile_w;
    a.tab = p->d_tab1;
    a.coef = p->d_coef1;
    a.E = p->d_E;
    a.V = p->d_V;
    a.tile_sums = sums ? p->d_tile_sums : nullptr;
    a.status = p->d_status;
    HIPCHK(launch_render(a, 4, st));
    return CELESTE_OK;
}

// Planes (and with `sums` the per-tile ELBO sums) gathered from every box's stored own
// profile values and brightness coefficients, which must be current.
int gather(celeste_plan* p, bool sums, hipStream_t st) {
    RenderArgs a{};
    a.g = p->geom();
    a.tiles = p->d_tiles;
    a.tile_list = p->d_tile_list;
    a.n_tiles = (int32_t)p->tiles.size();
    a.tile_h = p->tile_h;
    a.tile_w = p->tile_w;
    a.coef = p->d_coef1;
    a.E = p->d_E;
    a.V = p->d_V;
    a.tile_sums = sums ? p->d_tile_sums : nullptr;
    a.status = p->d_status;
    HIPCHK(launch_gather_planes(a, p->d_fg, 4, st));
    p->fg_valid = true;
    return CELESTE_OK;
}

// E and V planes of all sources.  Mode 2: every box's own profile values (one parallel
// strip pass), then a tile gather; mode 1: tiles evaluate the Gaussians; mode 0: sky fill,
// then one strip launch per conflict-free class.  sums: also the per-tile sums of the
// pixel terms of covered pixels into d_tile_sums (modes 0 and 1 then use the tiles).
int render(celeste_plan* p, hipStream_t st, bool sums = false) {
    p->fg_valid = false;
    if (p->render_mode == 1 || (sums && p->render_mode == 0)) return render_tiles(p, sums, st);
    if (p->render_mode == 2 || p->render_mode == 3) {
        const Sel all{nullptr, 0, (int32_t)p->items.size()};
        HIPCHK(launch_strip_fg(all, p->geom(), p->d_tab1, p->d_fg, p->rows, p->launch_grid(), p->wpb,
                               p->d_status, st));
        p->fg_valid = true;
        // mode 3: no planes (the adjoint gathers from stored values) unless sums are asked for
        if (p->render_mode == 3 && !sums) return CELESTE_OK;
        return gather(p, sums, st);
    }
    HIPCHK(launch_fill_planes(p->d_images, p->n_img, p->max_pix, p->d_E, p->d_V, p->d_status, st));
    const Geometry g = p->geom();
    for (int c = 0; c < p->n_class; ++c) {
        const Sel sel{p->d_cls_items + p->cls_ptr[c], 0, p->cls_ptr[c + 1] - p->cls_ptr[c]};
        HIPCHK(launch_render_strips(sel, g, p->d_tab1, p->d_coef1, p->d_E, p->d_V, p->rows, p->launch_grid(),
                                    p->wpb, p->d_status, st));
    }
    return CELESTE_OK;
}

// kk: also the pixel-level rows (brightness factors, frac_dev) of every box's intermediate
// Hessian (double gradient passes on stored backgrounds before hessian_from_intermediates).
int adjoint(celeste_plan* p, const Sel& items, const uint8_t* active, bool tangent, int base, bool deriv,
            hipStream_t st, int grid_override = 0, bool kk = false) {
    AdjArgs a{};
    a.g = p->geom();
    a.items = items;
    a.active = active;
    a.tab = tangent ? p->d_tab2 : p->d_tab1;
    a.coef = tangent ? p->d_coef2 : p->d_coef1;
    a.tab_val = p->d_tab1;
    a.coef_val = p->d_coef1;
    a.dynamic = p->dynamic;
    a.counter = p->d_counter;
    a.E = p->d_E;
    a.V = p->d_V;
    a.bg = p->d_bg;
    if (base == BASE_PLANES && p->render_mode == 3) base = BASE_FG;
    a.fg = ((base == BASE_PLANES || base == BASE_FG) && p->fg_valid) ? p->d_fg : nullptr;
    a.partials = p->d_partials;
    a.kk = kk ? p->d_kk : nullptr;
    if (kk) {
        // the pass also leaves the listed boxes' own profile values in d_fg for the
        // closed-form Hessian pass, so d_fg no longer holds a render's values
        a.fg_out = p->d_fg;
        p->fg_valid = false;
    }
    a.status = p->d_status;
    const int grid = grid_override > 0 ? grid_override : p->launch_grid();
    HIPCHK(launch_adjoint(a, tangent, base, deriv, grid, p->wpb, p->rows, st));
    return CELESTE_OK;
}

int finalize(celeste_plan* p, const double* theta, const Sel& srcs, const uint8_t* active, bool tangent,
             int dir_mode, const double* dir, int dir_unit, bool deriv, double* elbo, double* grad,
             double* tan_out, int64_t tan_stride, bool tan_by_list, hipStream_t st) {
    const bool pad = tan_out && tan_stride == ROW;
    FinArgs a{};
    a.g = p->geom();
    a.srcs = srcs;
    a.active = active;
    a.theta = theta;
    a.dir = dir;
    a.dir_mode = dir_mode;
    a.dir_unit = dir_unit;
    a.patch_ptr = p->d_patch_ptr;
    a.pair_lgamma = (p->consts.flags & CELESTE_INCLUDE_LGAMMA) ? p->d_pair_lgamma : nullptr;
    a.partials = p->d_partials;
    a.deriv = deriv ? 1 : 0;
    a.elbo = elbo;
    a.grad = grad;
    a.tangent = tan_out;
    a.tangent_stride = tan_stride;
    a.tangent_by_list = tan_by_list ? 1 : 0;
    a.tangent_pad = pad ? 1 : 0;
    a.status = p->d_status;
    HIPCHK(launch_finalize(a, tangent, st));
    return CELESTE_OK;
}

// Background of the listed visits: the other boxes' Gaussians evaluated from the current
// tables, or (stored = true) their stored own values, which must be current.
int background(celeste_plan* p, const Sel& items, hipStream_t st, bool stored = false) {
    BgArgs a{};
    a.g = p->geom();
    a.items = items;
    a.tab_val = p->d_tab1;
    a.coef_val = p->d_coef1;
    a.fg = stored ? p->d_fg : nullptr;
    a.bg = p->d_bg;
    a.status = p->d_status;
    HIPCHK(launch_background(a, p->launch_grid(), p->wpb, p->rows, st));
    return CELESTE_OK;
}

// Dense Hessians of the listed sources (d_hess by list position).  Expects the item
// partials and pixel-level Hessian rows (kk: brightness factors and frac_dev) of a double
// gradient pass over `item` on stored backgrounds (and, for the closed-form pass, the
// own profile values that pass stores).  With the position and shape rows (closed-form
// pass, or five tangent passes along those intermediates) they give each box's 10x10
// Hessian of its pixel terms; the chain rule and its tangent assemble the 27x27 blocks.
// With `active`, the closed-form pass covers only the boxes of the sources it marks (the
// other sources' blocks are left undefined).
int hessian_from_intermediates(celeste_plan* p, const double* theta, const Sel& src, const Sel& pair, const Sel& item,
                               int base, double* hess, hipStream_t st, const uint8_t* active = nullptr);

#define CHK(x)                              \
    do {                                    \
        int r_ = (x);                       \
        if (r_ != CELESTE_OK) return r_;    \
    } while (0)

int validate_theta(celeste_plan* p, const double* theta, const uint8_t* active, const int32_t* d_list, int n,
                   hipStream_t st) {
    HIPCHK(launch_validate(theta, active, d_list, n, p->n_src, p->consts.npar, p->d_status, st));
    return CELESTE_OK;
}

// Batched evaluation: validate, tables, render, fused adjoint, finalize.
int batched_sequence(celeste_plan* p, const double* theta, const uint8_t* active, bool deriv, double* elbo,
                     double* grad, hipStream_t st, bool capturing = false) {
    const Scope sc = scope_all(p);
    const bool prof = p->profiling && !capturing;
    if (prof) HIPCHK(hipEventRecord(p->ev[0], st));
    CHK(validate_theta(p, theta, active, nullptr, p->n_src, st));
    CHK(prep(p, theta, sc.pair, false, DIR_NONE, nullptr, 0, st));
    if (prof) HIPCHK(hipEventRecord(p->ev[1], st));
    CHK(render(p, st));
    if (prof) HIPCHK(hipEventRecord(p->ev[2], st));
    CHK(adjoint(p, sc.item, active, false, BASE_PLANES, deriv, st));
    if (prof) HIPCHK(hipEventRecord(p->ev[3], st));
    CHK(finalize(p, theta, sc.src, active, false, DIR_NONE, nullptr, 0, deriv, elbo, grad, nullptr, 0, false, st));
    if (prof) {
        HIPCHK(hipEventRecord(p->ev[4], st));
        HIPCHK(hipEventSynchronize(p->ev[4]));
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, p->ev[k], p->ev[k + 1]));
            p->phase_ms[k] += ms;
        }
        p->phase_calls++;
    }
    return CELESTE_OK;
}

int plain_sequence(celeste_plan* p, const double* theta, const uint8_t* active, bool deriv, double* elbo,
                   double* grad, hipStream_t st) {
    const Scope all = scope_all(p);
    CHK(validate_theta(p, theta, active, nullptr, p->n_src, st));
    CHK(prep(p, theta, all.pair, false, DIR_NONE, nullptr, 0, st));
    for (int s = 0; s < p->n_src; ++s) {
        const Scope sc = scope_source(p, s);
        CHK(adjoint(p, sc.item, active, false, BASE_NBR, deriv, st));
        CHK(finalize(p, theta, sc.src, active, false, DIR_NONE, nullptr, 0, deriv, elbo, grad, nullptr, 0, false,
                     st));
    }
    return CELESTE_OK;
}

int config_code(const celeste_plan* p) {
    return ((((p->chunk * 8 + p->wpb) * 2 + p->dynamic) * 32 + p->rows) * 2 + p->render_mode) * 1000003 +
           p->launch_grid() * 131 + p->tile_h * 7 + p->tile_w;
}

// Lists of boxes and items of a set of sources (host), uploaded into the plan's list buffers
// at the given offsets.
struct HostScope {
    std::vector<int32_t> src, pair, item;
};

void scope_lists(const celeste_plan* p, const int32_t* src, int n, HostScope& hs) {
    const size_t i0 = hs.item.size();
    for (int j = 0; j < n; ++j) {
        const int s = src[j];
        hs.src.push_back(s);
        for (int pi = p->patch_ptr[s]; pi < p->patch_ptr[s + 1]; ++pi) {
            hs.pair.push_back(pi);
            for (int it = p->pairs[pi].item_begin; it < p->pairs[pi].item_end; ++it) hs.item.push_back(it);
        }
    }
    // items of more strips first, so that a launch over the list ends on short items and its
    // last waves finish close together (every item writes its own outputs and the box sums
    // run in item order: the list order changes no result); a stable counting sort on the
    // strip count
    const size_t n_it = hs.item.size() - i0;
    if (n_it < 2) return;
    int mx = 0;
    for (size_t i = i0; i < hs.item.size(); ++i) mx = std::max(mx, (int)p->items[hs.item[i]].count);
    std::vector<size_t> pos(mx + 2, 0);
    for (size_t i = i0; i < hs.item.size(); ++i) pos[mx - p->items[hs.item[i]].count + 1]++;
    for (int k = 1; k <= mx + 1; ++k) pos[k] += pos[k - 1];
    std::vector<int32_t> out(n_it);
    for (size_t i = i0; i < hs.item.size(); ++i) out[pos[mx - p->items[hs.item[i]].count]++] = hs.item[i];
    std::copy(out.begin(), out.end(), hs.item.begin() + i0);
}

int fill_u8(uint8_t* d, const Sel& srcs, uint8_t v, hipStream_t st) {
    HIPCHK(launch_fill_u8_sel(d, srcs, v, st));
    return CELESTE_OK;
}

int fill_f64(double* d, const Sel& srcs, double v, hipStream_t st) {
    HIPCHK(launch_fill_f64_sel(d, srcs, v, st));
    return CELESTE_OK;
}

// Host lists into device buffers on `st`, through the plan's pinned staging: no host
// synchronisation except, when the staging is still being read by the previous upload, a
// wait for that copy.  Growing the staging allocates pinned host memory.
int upload(celeste_plan* p, std::initializer_list<std::pair<const std::vector<int32_t>*, int32_t*>> lists,
           hipStream_t st) {
    size_t n = 0;
    for (const auto& l : lists) n += l.first->size();
    if (p->stage_pending) {
        HIPCHK(hipEventSynchronize(p->stage_ev));
        p->stage_pending = false;
    }
    if (n > p->cap_stage) {
        if (p->h_stage) HIPCHK(hipHostFree(p->h_stage));
        p->h_stage = nullptr;
        p->cap_stage = 0;
        HIPCHK(hipHostMalloc((void**)&p->h_stage, std::max<size_t>(n, 1024) * sizeof(int32_t), hipHostMallocDefault));
        p->cap_stage = std::max<size_t>(n, 1024);
    }
    size_t off = 0;
    for (const auto& l : lists) {
        const std::vector<int32_t>& v = *l.first;
        if (v.empty()) continue;
        std::copy(v.begin(), v.end(), p->h_stage + off);
        HIPCHK(hipMemcpyAsync(l.second, p->h_stage + off, v.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        off += v.size();
    }
    HIPCHK(hipEventRecord(p->stage_ev, st));
    p->stage_pending = true;
    return CELESTE_OK;
}

int upload_lists(celeste_plan* p, const HostScope& hs, hipStream_t st) {
    return upload(p, {{&hs.src, p->d_list_src}, {&hs.pair, p->d_list_pair}, {&hs.item, p->d_list_item}}, st);
}

// The boxes whose tables, coefficients and stored own profile values a call on the listed
// boxes reads: the listed boxes and every box of the same image meeting one (whose stored
// values the listed boxes' backgrounds sum), with their items.
void neighbour_lists(const celeste_plan* p, const HostScope& hs, std::vector<int32_t>& npair,
                     std::vector<int32_t>& nitem) {
    std::vector<char> mark(p->pairs.size(), 0);
    for (int32_t pi : hs.pair) {
        mark[pi] = 1;
        for (int q = p->pairs[pi].nbr_begin; q < p->pairs[pi].nbr_end; ++q) mark[p->nbr[q]] = 1;
    }
    npair.clear();
    nitem.clear();
    for (size_t q = 0; q < mark.size(); ++q)
        if (mark[q]) {
            npair.push_back((int32_t)q);
            for (int it = p->pairs[q].item_begin; it < p->pairs[q].item_end; ++it) nitem.push_back(it);
        }
}

// Lists of hs and, when the stored-value render is used (`stored`), the boxes whose stored
// own profile values and brightness coefficients the listed boxes' backgrounds read: every
// box when those are most of the field, else the neighbour boxes only (uploaded with the
// lists).  *render receives the boxes and items to render.
int upload_scope(celeste_plan* p, const HostScope& hs, bool stored, Scope* render, hipStream_t st) {
    std::vector<int32_t> npair, nitem;
    if (stored) neighbour_lists(p, hs, npair, nitem);
    const bool restrict_render = stored && 2 * nitem.size() < p->items.size();
    if (restrict_render)
        CHK(upload(p, {{&hs.src, p->d_list_src}, {&hs.pair, p->d_list_pair}, {&hs.item, p->d_list_item},
                       {&npair, p->d_list_npair}, {&nitem, p->d_list_nitem}},
                   st));
    else
        CHK(upload_lists(p, hs, st));
    *render = scope_all(p);
    if (restrict_render) {
        render->pair = Sel{p->d_list_npair, 0, (int32_t)npair.size()};
        render->item = Sel{p->d_list_nitem, 0, (int32_t)nitem.size()};
    }
    return CELESTE_OK;
}

// Stored own profile values and coefficients of the boxes of `render` (d_fg then no longer
// holds a full render's values).
int render_stored(celeste_plan* p, const double* theta, const Scope& render, hipStream_t st) {
    CHK(prep(p, theta, render.pair, false, DIR_NONE, nullptr, 0, st));
    HIPCHK(launch_strip_fg(render.item, p->geom(), p->d_tab1, p->d_fg, p->rows, p->launch_grid(), p->wpb,
                           p->d_status, st));
    p->fg_valid = false;
    return CELESTE_OK;
}

int hessian_from_intermediates(celeste_plan* p, const double* theta, const Sel& src, const Sel& pair, const Sel& item,
                               int base, double* hess, hipStream_t st, const uint8_t* active) {
    HIPCHK(launch_pair_reduce(pair, p->d_pairs, p->d_partials, p->d_kk, false, 0, p->d_gw, p->d_hw, p->d_status,
                              st));
    // the brightness-factor and frac_dev rows came with the gradient pass; the five position
    // and shape rows (by symmetry, the other rows' remaining entries too) come from the
    // closed-form pass over the stored backgrounds, or from tangent passes of the adjoint
    if (p->hess_mode == 0 && base == BASE_BG) {
        AdjArgs a{};
        a.g = p->geom();
        a.items = item;
        a.active = active;
        a.tab = p->d_tab1;
        a.coef = p->d_coef1;
        a.bg = p->d_bg;
        a.fg = p->d_fg;
        a.dynamic = p->dynamic;
        a.counter = p->d_counter;
        a.status = p->d_status;
        HIPCHK(launch_hess_geom(a, p->d_nu, p->d_hg, p->launch_grid(), p->wpb, p->rows, st));
        HIPCHK(launch_pair_hess(pair, p->d_pairs, p->d_hg, p->d_hw, p->d_status, st));
        HIPCHK(launch_assemble_hessian(src, p->geom(), p->d_patch_ptr, theta, p->d_gw, p->d_hw, hess, p->d_status,
                                       st));
        return CELESTE_OK;
    }
    for (int i = W_UX; i < NW; ++i) {
        if (i == W_FDEV) continue;
        CHK(prep(p, theta, pair, true, DIR_W, nullptr, i, st));
        CHK(adjoint(p, item, nullptr, true, base, true, st));
        HIPCHK(launch_pair_reduce(pair, p->d_pairs, p->d_partials, nullptr, true, i, p->d_gw, p->d_hw, p->d_status,
                                  st));
    }
    HIPCHK(launch_assemble_hessian(src, p->geom(), p->d_patch_ptr, theta, p->d_gw, p->d_hw, hess, p->d_status, st));
    return CELESTE_OK;
}

// Newton trust-region iterations for one source set; lists already on the device.
// stored_bg: every box's stored own values and coefficients are current (sweeps keep them
// so), and the background is summed from them instead of evaluated.
int newton_run(celeste_plan* p, double* theta, const Sel& src, const Sel& pair, const Sel& item, int n_steps,
               const celeste_tr_params* prm, double* radius, hipStream_t st, bool stored_bg = false) {
    // background of every listed visit with all sources at their entry values
    if (stored_bg) {
        CHK(background(p, item, st, true));
    } else {
        const Scope all = scope_all(p);
        CHK(prep(p, theta, all.pair, false, DIR_NONE, nullptr, 0, st));
        CHK(background(p, item, st));
    }
    TrArgs tr{};
    tr.srcs = src;
    tr.theta = theta;
    tr.grad = p->d_grad;
    tr.hess = p->d_hess;
    tr.grad_trial = p->d_grad_trial;
    tr.hess_trial = p->d_hess_trial;
    tr.accepted = p->d_accepted;
    tr.live = p->d_live;
    tr.radius = radius;
    tr.theta_trial = p->d_theta_trial;
    tr.pred = p->d_pred;
    tr.elbo_cur = p->d_elbo_cur;
    tr.elbo_trial = p->d_elbo_trial;
    tr.done = p->d_done;
    tr.eta_accept = prm->eta_accept;
    tr.radius_max = prm->radius_max;
    tr.gtol = prm->gtol;
    tr.npar = p->consts.npar;
    tr.status = p->d_status;
    if (n_steps <= 0) return CELESTE_OK;
    // value, gradient and Hessian at the entry point
    CHK(prep(p, theta, pair, false, DIR_NONE, nullptr, 0, st));
    CHK(adjoint(p, item, nullptr, false, BASE_BG, true, st, 0, true));
    CHK(finalize(p, theta, src, nullptr, false, DIR_NONE, nullptr, 0, true, p->d_elbo_cur, p->d_grad, nullptr, 0,
                 false, st));
    CHK(hessian_from_intermediates(p, theta, src, pair, item, BASE_BG, p->d_hess, st));
    for (int it = 0; it < n_steps; ++it) {
        HIPCHK(launch_tr_solve(tr, st));
        // the trial point of every source still stepping (d_live): its value and, except
        // after the last step, its gradient; then, for the sources whose step was accepted,
        // its Hessian, and gradient and Hessian become the current ones (a rejected step
        // keeps the point and with it the current gradient and Hessian)
        const bool more = it + 1 < n_steps;
        CHK(prep(p, p->d_theta_trial, pair, false, DIR_NONE, nullptr, 0, st));
        CHK(adjoint(p, item, p->d_live, false, BASE_BG, more, st, 0, more));
        CHK(finalize(p, p->d_theta_trial, src, p->d_live, false, DIR_NONE, nullptr, 0, more, p->d_elbo_trial,
                     more ? p->d_grad_trial : nullptr, nullptr, 0, false, st));
        HIPCHK(launch_tr_update(tr, st));
        if (more) {
            CHK(hessian_from_intermediates(p, p->d_theta_trial, src, pair, item, BASE_BG, p->d_hess_trial, st,
                                           p->d_accepted));
            HIPCHK(launch_tr_adopt(tr, st));
        }
    }
    return CELESTE_OK;
}

}  // namespace

namespace cel {

int batched_elbo_grad_scratch(celeste_plan* p, const double* theta, const uint8_t* active, double* elbo,
                              double* grad, double* partials, int* counter, hipStream_t st) {
    // the plan's own partials and counter are set aside for this call only (calls on one
    // plan never overlap)
    double* const own_partials = p->d_partials;
    int* const own_counter = p->d_counter;
    p->d_partials = partials;
    p->d_counter = counter;
    const int rc = batched_sequence(p, theta, active, true, elbo, grad, st);
    p->d_partials = own_partials;
    p->d_counter = own_counter;
    return rc;
}

int64_t plan_item_count(const celeste_plan* p) { return (int64_t)p->items.size(); }

int plan_device(const celeste_plan* p) { return p->device; }

}  // namespace cel

// ================================================================ C entry points
extern "C" {

int celeste_version(void) { return CELESTE_ABI_VERSION; }

int celeste_debug_math(int fn, const double* x, double* y, int n, hipStream_t st) {
    if (!x || !y || n < 0 || fn < CELESTE_FN_EXP || fn > CELESTE_FN_RCP) return CELESTE_EINVAL;
    HIPCHK(launch_debug_math(fn, x, y, n, st));
    return CELESTE_OK;
}

const char* celeste_last_hip_error(void) { return g_hip_error.c_str(); }

const char* celeste_status_string(int s) {
    switch (s) {
        case CELESTE_OK: return "ok";
        case CELESTE_EINVAL: return "invalid argument, size or geometry";
        case CELESTE_ECONFLICT: return "batch members share pixels";
        case CELESTE_EHIP: return "HIP runtime error";
        case CELESTE_ENOMEM: return "device allocation failed";
        case CELESTE_EDOMAIN: return "parameters outside their domain";
        case CELESTE_ESCRATCH: return "problem larger than the static scratch buffer";
        default: return "unknown status";
    }
}

void celeste_plan_destroy(celeste_plan* p) {
    if (!p) return;
    drop_graph(p);
    if (p->sweep_pending && p->sweep_ev) (void)hipEventSynchronize(p->sweep_ev);
    if (p->sweep_exec) (void)hipGraphExecDestroy(p->sweep_exec);
    if (p->stage_pending && p->stage_ev) (void)hipEventSynchronize(p->stage_ev);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->stage_ev) (void)hipEventDestroy(p->stage_ev);
    if (p->sweep_ev) (void)hipEventDestroy(p->sweep_ev);
    void* bufs[] = {p->d_images, p->d_pairs, p->d_items, p->d_nbr, p->d_tiles, p->d_tile_list, p->d_patch_ptr,
                    p->d_tab1, p->d_coef1, p->d_tab2, p->d_coef2, p->d_partials, p->d_E, p->d_V, p->d_bg,
                    p->d_tile_sums, p->d_status, p->d_counter, p->d_grad, p->d_hess, p->d_theta_trial,
                    p->d_pred, p->d_elbo_cur, p->d_elbo_trial, p->d_radius, p->d_done, p->d_list_src,
                    p->d_list_pair, p->d_list_item, p->d_cls_items, p->d_pair_lgamma, p->d_fg, p->d_gw,
                    p->d_hw, p->d_kk, p->d_hg, p->d_nu, p->d_grad_trial, p->d_hess_trial, p->d_accepted, p->d_live,
                    p->d_mix, p->d_scalar, p->d_tt_part, p->d_list_npair, p->d_list_nitem, p->d_wcount};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (hipEvent_t& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

int celeste_plan_create(const celeste_problem_desc* d, celeste_plan** out) {
    if (!out) return CELESTE_EINVAL;
    *out = nullptr;
    int v = validate_desc(d);
    if (v == CELESTE_OK) v = validate_sky_maps(d);
    if (v != CELESTE_OK) return v;
    celeste_plan* p = new celeste_plan();
    HIPCHK(hipGetDevice(&p->device));
    {
        // set-up of the entry point without allocation on this device
        const int rs = noalloc_attach(p->device);
        if (rs != CELESTE_OK) {
            delete p;
            return rs;
        }
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess && prop.multiProcessorCount > 0)
        p->n_cu = prop.multiProcessorCount;
    p->n_img = d->n_img;
    p->n_src = d->n_src;
    p->n_pix = d->n_pix;
    p->d_x = d->x;
    p->images.assign(d->images, d->images + d->n_img);
    p->patch_ptr.assign(d->patch_ptr, d->patch_ptr + d->n_src + 1);
    std::memcpy(p->consts.exp_alpha, d->exp_alpha, sizeof(d->exp_alpha));
    std::memcpy(p->consts.exp_nu, d->exp_nu, sizeof(d->exp_nu));
    std::memcpy(p->consts.dev_alpha, d->dev_alpha, sizeof(d->dev_alpha));
    std::memcpy(p->consts.dev_nu, d->dev_nu, sizeof(d->dev_nu));
    p->consts.prior_phi = d->prior_phi;
    std::memcpy(p->consts.prior_r, d->prior_r, sizeof(d->prior_r));
    std::memcpy(p->consts.prior_c, d->prior_c, sizeof(d->prior_c));
    p->consts.flags = d->flags;
    p->consts.npar = (d->flags & CELESTE_COLOR_MIXTURE) ? NPK : NP;
    p->consts.mix = nullptr;
    const int nb = d->patch_ptr[d->n_src];
    p->pairs.resize(nb);
    int64_t voff = 0;
    for (int s = 0; s < d->n_src; ++s)
        for (int b = d->patch_ptr[s]; b < d->patch_ptr[s + 1]; ++b) {
            const celeste_box& bx = d->boxes[b];
            PairDev& pd = p->pairs[b];
            pd.src = s;
            pd.img = bx.img;
            pd.r0 = bx.r0;
            pd.c0 = bx.c0;
            pd.h = bx.h;
            pd.w = bx.w;
            pd.visit_off = voff;
            voff += (int64_t)bx.h * bx.w;
        }
    p->n_visits = voff;
    for (const celeste_image& im : p->images) p->max_pix = std::max<int64_t>(p->max_pix, (int64_t)im.H * im.W);
    build_items(p);
    build_nbr(p);
    build_pair_classes(p);
    build_class_items(p);
    build_tiles(p);
    // capacity of per-item buffers: the shortest strips (4 rows) and smallest chunk (64)
    size_t max_items = 0;
    for (const PairDev& pd : p->pairs) max_items += (size_t)((strips_of(pd, 4) + 63) / 64);
    const size_t np = std::max<size_t>(p->pairs.size(), 1);
    size_t& W = p->workspace;
    int r = CELESTE_OK;
    auto A = [&](int rc) { if (rc != CELESTE_OK && r == CELESTE_OK) r = rc; };
    A(dalloc(&p->d_images, p->n_img, W));
    A(dalloc(&p->d_pairs, np, W));
    A(dalloc(&p->d_items, max_items, W));
    p->cap_items = max_items;
    A(dalloc(&p->d_nbr, std::max<size_t>(p->nbr.size(), 1), W));
    A(dalloc(&p->d_tiles, p->tiles.size(), W));
    p->cap_tiles = p->tiles.size();
    A(dalloc(&p->d_tile_list, p->tile_list.size(), W));
    p->cap_tile_list = p->tile_list.size();
    A(dalloc(&p->d_patch_ptr, (size_t)p->n_src + 1, W));
    A(dalloc(&p->d_tab1, np * NCOMP * CST, W));
    A(dalloc(&p->d_coef1, np * NCOEF, W));
    A(dalloc(&p->d_tab2, np * NCOMP * CST * 2, W));
    A(dalloc(&p->d_coef2, np * NCOEF * 2, W));
    A(dalloc(&p->d_partials, max_items * NACC * 2, W));
    A(dalloc(&p->d_kk, max_items * NKK, W));
    A(dalloc(&p->d_hg, max_items * NHG, W));
    A(dalloc(&p->d_nu, NGAL, W));
    A(dalloc(&p->d_E, (size_t)p->n_pix, W));
    A(dalloc(&p->d_V, (size_t)p->n_pix, W));
    A(dalloc(&p->d_bg, (size_t)p->n_visits * 2, W));
    A(dalloc(&p->d_fg, (size_t)p->n_visits * 2, W));
    A(dalloc(&p->d_tile_sums, std::max<size_t>(p->tiles.size(), 1), W));
    A(dalloc(&p->d_pair_lgamma, np, W));
    A(dalloc(&p->d_status, 1, W));
    A(dalloc(&p->d_counter, 1, W));
    A(dalloc(&p->d_wcount, NLIVE_COUNTS, W));
    const size_t S = (size_t)p->n_src;
    A(dalloc(&p->d_grad, S * ROW, W));
    A(dalloc(&p->d_hess, S * NPK * NPK, W));
    A(dalloc(&p->d_grad_trial, S * ROW, W));
    A(dalloc(&p->d_hess_trial, S * NPK * NPK, W));
    A(dalloc(&p->d_accepted, S, W));
    A(dalloc(&p->d_live, S, W));
    A(dalloc(&p->d_gw, np * NACC, W));
    A(dalloc(&p->d_hw, np * 100, W));
    A(dalloc(&p->d_theta_trial, S * ROW, W));
    A(dalloc(&p->d_pred, S * 2, W));
    A(dalloc(&p->d_elbo_cur, S, W));
    A(dalloc(&p->d_elbo_trial, S, W));
    A(dalloc(&p->d_radius, S, W));
    A(dalloc(&p->d_done, S, W));
    A(dalloc(&p->d_list_src, S, W));
    A(dalloc(&p->d_list_pair, np, W));
    A(dalloc(&p->d_list_item, max_items, W));
    A(dalloc(&p->d_list_npair, np, W));
    A(dalloc(&p->d_list_nitem, max_items, W));
    A(dalloc(&p->d_cls_items, max_items, W));
    A(dalloc(&p->d_scalar, 1, W));
    A(dalloc(&p->d_tt_part, 1024, W));
    if (d->flags & CELESTE_COLOR_MIXTURE) A(dalloc(&p->d_mix, 2 * NMIX * MIXF, W));
    p->cap_list_item = max_items;
    p->cap_list_src = S;
    p->cap_list_pair = np;
    if (r != CELESTE_OK) {
        celeste_plan_destroy(p);
        return r;
    }
    int rc = upload_geometry(p);
    if (rc == CELESTE_OK) {
        double nu[NGAL];
        for (int g = 0; g < NGAL; ++g) {
            const int jj = g % NGAL_PER_PSF;
            nu[g] = jj < NDEV ? p->consts.dev_nu[jj] : p->consts.exp_nu[jj - NDEV];
        }
        if (hipMemcpy(p->d_nu, nu, sizeof(nu), hipMemcpyHostToDevice) != hipSuccess)
            rc = hip_fail(hipGetLastError(), "component table upload");
    }
    if (rc == CELESTE_OK && p->d_mix) {
        double tab[2 * NMIX * MIXF];
        mixture_table(d, tab);
        if (hipMemcpy(p->d_mix, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
            rc = hip_fail(hipGetLastError(), "mixture table upload");
        p->consts.mix = p->d_mix;
    }
    if (rc == CELESTE_OK) {
        if (hipMemcpy(p->d_images, p->images.data(), p->images.size() * sizeof(celeste_image),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_nbr, p->nbr.data(), p->nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(p->d_patch_ptr, p->patch_ptr.data(), p->patch_ptr.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(p->d_status, 0, sizeof(int)) != hipSuccess ||
            hipMemset(p->d_counter, 0, sizeof(int)) != hipSuccess ||
            hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->stage_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->sweep_ev, hipEventDisableTiming) != hipSuccess)
            rc = hip_fail(hipGetLastError(), "plan upload");
    }
    if (rc == CELESTE_OK && (p->consts.flags & CELESTE_INCLUDE_LGAMMA)) {
        const hipError_t e = launch_pair_lgamma(p->geom(), (int)p->pairs.size(), p->d_pair_lgamma, nullptr);
        if (e != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = hip_fail(hipGetLastError(), "log(x!) sums");
    }
    if (rc != CELESTE_OK) {
        celeste_plan_destroy(p);
        return rc;
    }
    *out = p;
    return CELESTE_OK;
}

int celeste_plan_get_info(const celeste_plan* p, celeste_plan_info* info) {
    if (!p || !info) return CELESTE_EINVAL;
    info->n_visits = p->n_visits;
    info->n_pairs = (int64_t)p->pairs.size();
    info->n_items = (int64_t)p->items.size();
    info->n_tiles = (int64_t)p->tiles.size();
    info->n_nbr = (int64_t)p->nbr.size();
    info->chunk = p->chunk;
    info->waves_per_block = p->wpb;
    info->grid_blocks = p->launch_grid();
    info->tile_h = p->tile_h;
    info->tile_w = p->tile_w;
    info->dynamic_queue = p->dynamic;
    info->strip_rows = p->rows;
    info->render_mode = p->render_mode;
    info->n_classes = p->n_class;
    info->n_params = p->consts.npar;
    info->workspace_bytes = (int64_t)p->workspace;
    return CELESTE_OK;
}

int celeste_plan_set_launch(celeste_plan* p, int chunk, int wpb, int grid, int dynamic, int tile_h, int tile_w,
                            int strip_rows, int render_mode) {
    if (!p || chunk < 64 || chunk > 1024 || chunk % 64 || (wpb != 1 && wpb != 2 && wpb != 4) || grid < 0 ||
        (dynamic != 0 && dynamic != 1) || tile_w < 1 || tile_w > 64 || 64 % tile_w || tile_h < 1 ||
        (tile_h * tile_w != 64 && tile_h * tile_w != 128 && tile_h * tile_w != 256) ||
        (strip_rows != 4 && strip_rows != 8 && strip_rows != 16) || render_mode < 0 || render_mode > 3)
        return CELESTE_EINVAL;
    HIPCHK(hipDeviceSynchronize());
    drop_graph(p);
    if (tile_h != p->tile_h || tile_w != p->tile_w) {
        const int old_h = p->tile_h, old_w = p->tile_w;
        p->tile_h = tile_h;
        p->tile_w = tile_w;
        build_tiles(p);
        // grow the tile buffers: new ones first, so that a failed allocation leaves the plan
        // working with its previous tiles
        TileDev* nt = nullptr;
        double* ns = nullptr;
        int32_t* nl = nullptr;
        bool ok = true;
        if (p->tiles.size() > p->cap_tiles)
            ok = hipMalloc((void**)&nt, p->tiles.size() * sizeof(TileDev)) == hipSuccess &&
                 hipMalloc((void**)&ns, p->tiles.size() * sizeof(double)) == hipSuccess;
        if (ok && p->tile_list.size() > p->cap_tile_list)
            ok = hipMalloc((void**)&nl, p->tile_list.size() * sizeof(int32_t)) == hipSuccess;
        if (!ok) {
            (void)hipFree(nt);
            (void)hipFree(ns);
            (void)hipFree(nl);
            (void)hipGetLastError();
            p->tile_h = old_h;
            p->tile_w = old_w;
            build_tiles(p);
            return CELESTE_ENOMEM;
        }
        if (nt) {
            (void)hipFree(p->d_tiles);
            (void)hipFree(p->d_tile_sums);
            p->d_tiles = nt;
            p->d_tile_sums = ns;
            p->cap_tiles = p->tiles.size();
        }
        if (nl) {
            (void)hipFree(p->d_tile_list);
            p->d_tile_list = nl;
            p->cap_tile_list = p->tile_list.size();
        }
    }
    p->rows = strip_rows;
    p->render_mode = render_mode;
    p->chunk = chunk;
    p->wpb = wpb;
    p->grid = grid;
    p->dynamic = dynamic;
    build_items(p);
    build_class_items(p);
    return upload_geometry(p);
}

int celeste_plan_profile(celeste_plan* p, int enable, double* ms, int64_t* calls, int reset) {
    if (!p) return CELESTE_EINVAL;
    if (enable && !p->ev[0])
        for (hipEvent_t& e : p->ev) HIPCHK(hipEventCreate(&e));
    p->profiling = enable != 0;
    if (ms)
        for (int k = 0; k < 4; ++k) ms[k] = p->phase_ms[k];
    if (calls) *calls = p->phase_calls;
    if (reset) {
        for (double& v : p->phase_ms) v = 0.0;
        p->phase_calls = 0;
    }
    return CELESTE_OK;
}

int celeste_plan_use_graph(celeste_plan* p, int enable) {
    if (!p) return CELESTE_EINVAL;
    p->use_graph = enable != 0;
    if (!p->use_graph) drop_graph(p);
    return CELESTE_OK;
}

int celeste_plan_status(celeste_plan* p, hipStream_t st) {
    if (!p) return CELESTE_EINVAL;
    HIPCHK(hipStreamSynchronize(st));
    int s = 0;
    HIPCHK(hipMemcpy(&s, p->d_status, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemset(p->d_status, 0, sizeof(int)));
    return s;
}

int celeste_elbo(celeste_plan* p, const double* theta, const uint8_t* active, int mode, double* elbo,
                 hipStream_t st) {
    if (!p || !theta || !elbo || (mode != CELESTE_PLAIN && mode != CELESTE_BATCHED)) return CELESTE_EINVAL;
    if (mode == CELESTE_BATCHED) return batched_sequence(p, theta, active, false, elbo, nullptr, st);
    return plain_sequence(p, theta, active, false, elbo, nullptr, st);
}

int celeste_elbo_grad(celeste_plan* p, const double* theta, const uint8_t* active, int mode, double* elbo,
                      double* grad, hipStream_t st) {
    if (!p || !theta || !elbo || !grad || (mode != CELESTE_PLAIN && mode != CELESTE_BATCHED))
        return CELESTE_EINVAL;
    if (mode == CELESTE_PLAIN) return plain_sequence(p, theta, active, true, elbo, grad, st);
    if (!p->use_graph) return batched_sequence(p, theta, active, true, elbo, grad, st);
    const void* key[4] = {theta, active, elbo, grad};
    const int cfg = config_code(p);
    if (!p->gexec || std::memcmp(key, p->gkey, sizeof(key)) != 0 || cfg != p->gkey_cfg) {
        drop_graph(p);
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        const int rc = batched_sequence(p, theta, active, true, elbo, grad, p->cap_stream, true);
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (rc != CELESTE_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        const hipError_t e2 = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            p->gexec = nullptr;
            return hip_fail(e2, "hipGraphInstantiate");
        }
        std::memcpy(p->gkey, key, sizeof(key));
        p->gkey_cfg = cfg;
    }
    HIPCHK(hipGraphLaunch(p->gexec, st));
    return CELESTE_OK;
}

int celeste_hvp(celeste_plan* p, const double* theta, const double* v, double* hv, double* grad, hipStream_t st) {
    if (!p || !theta || !v || !hv) return CELESTE_EINVAL;
    const Scope sc = scope_all(p);
    CHK(validate_theta(p, theta, nullptr, nullptr, p->n_src, st));
    CHK(prep(p, theta, sc.pair, false, DIR_NONE, nullptr, 0, st));
    CHK(render(p, st));
    CHK(prep(p, theta, sc.pair, true, DIR_VEC, v, 0, st));
    CHK(adjoint(p, sc.item, nullptr, true, BASE_PLANES, true, st));
    CHK(finalize(p, theta, sc.src, nullptr, true, DIR_VEC, v, 0, true, nullptr, grad, hv, ROW, false, st));
    return CELESTE_OK;
}

int celeste_hessian(celeste_plan* p, const double* theta, const int32_t* src, int n, double* hess,
                    hipStream_t st) {
    if (!p || !theta || !src || n <= 0 || n > p->n_src || !hess) return CELESTE_EINVAL;
    std::vector<char> seen(p->n_src, 0);
    for (int j = 0; j < n; ++j) {
        if (src[j] < 0 || src[j] >= p->n_src || seen[src[j]]) return CELESTE_EINVAL;
        seen[src[j]] = 1;
    }
    HostScope hs;
    scope_lists(p, src, n, hs);
    const bool stored = p->render_mode == 2 || p->render_mode == 3;
    Scope rs;
    CHK(upload_scope(p, hs, stored, &rs, st));
    const Sel ss{p->d_list_src, 0, (int32_t)hs.src.size()};
    const Sel sp{p->d_list_pair, 0, (int32_t)hs.pair.size()};
    const Sel si{p->d_list_item, 0, (int32_t)hs.item.size()};
    CHK(validate_theta(p, theta, nullptr, nullptr, p->n_src, st));
    // stored per-visit backgrounds, as in a Newton iteration (with the strip render, summed
    // from the neighbour boxes' stored own values)
    if (stored) {
        CHK(render_stored(p, theta, rs, st));
        CHK(background(p, si, st, true));
    } else {
        const Scope all = scope_all(p);
        CHK(prep(p, theta, all.pair, false, DIR_NONE, nullptr, 0, st));
        CHK(background(p, si, st));
    }
    CHK(adjoint(p, si, nullptr, false, BASE_BG, true, st, 0, true));
    CHK(hessian_from_intermediates(p, theta, ss, sp, si, BASE_BG, p->d_hess, st));
    const size_t np2 = (size_t)p->consts.npar * p->consts.npar;
    HIPCHK(hipMemcpyAsync(hess, p->d_hess, (size_t)n * np2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    return CELESTE_OK;
}

int celeste_work_counts(celeste_plan* p, const double* theta, int64_t* counts, hipStream_t st) {
    if (!p || !theta || !counts) return CELESTE_EINVAL;
    const Scope sc = scope_all(p);
    CHK(validate_theta(p, theta, nullptr, nullptr, p->n_src, st));
    CHK(prep(p, theta, sc.pair, false, DIR_NONE, nullptr, 0, st));
    HIPCHK(launch_live_counts(sc.item, p->geom(), p->d_tab1, p->rows, p->d_wcount, p->d_status, st));
    unsigned long long h[NLIVE_COUNTS];
    HIPCHK(hipMemcpyAsync(h, p->d_wcount, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int status = 0;
    HIPCHK(hipMemcpy(&status, p->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (status) {
        HIPCHK(hipMemset(p->d_status, 0, sizeof(int)));
        return status;
    }
    for (int i = 0; i < NLIVE_COUNTS; ++i) counts[i] = (int64_t)h[i];
    return CELESTE_OK;
}

int celeste_total_elbo(celeste_plan* p, const double* theta, double* out, hipStream_t st) {
    if (!p || !theta || !out) return CELESTE_EINVAL;
    const Scope sc = scope_all(p);
    CHK(validate_theta(p, theta, nullptr, nullptr, p->n_src, st));
    CHK(prep(p, theta, sc.pair, false, DIR_NONE, nullptr, 0, st));
    CHK(render(p, st, true));
    HIPCHK(launch_tile_total(p->d_tile_sums, (int)p->tiles.size(), theta, p->consts, p->n_src, p->d_tt_part, out,
                             p->d_status, st));
    return CELESTE_OK;
}

int celeste_newton(celeste_plan* p, double* theta, const int32_t* src, int n, int n_steps,
                   const celeste_tr_params* prm, double* radius, double* elbo_out, hipStream_t st) {
    if (!p || !theta || !src || n <= 0 || n > p->n_src || n_steps < 0 || !prm || !radius) return CELESTE_EINVAL;
    if (!(prm->radius0 > 0.0) || !(prm->radius_max >= prm->radius0) || !(prm->eta_accept >= 0.0) ||
        !(prm->eta_accept < 0.25) || !(prm->gtol >= 0.0))
        return CELESTE_EINVAL;
    std::vector<char> seen(p->n_src, 0);
    for (int j = 0; j < n; ++j) {
        if (src[j] < 0 || src[j] >= p->n_src || seen[src[j]]) return CELESTE_EINVAL;
        seen[src[j]] = 1;
    }
    HostScope hs;
    scope_lists(p, src, n, hs);
    // with the strip render, the own profile values of the boxes the listed visits' backgrounds
    // read are stored once and the backgrounds are summed from them (cheaper than evaluating
    // the neighbours' Gaussians per visit)
    const bool stored = p->render_mode == 2 || p->render_mode == 3;
    Scope rs;
    CHK(upload_scope(p, hs, stored && n_steps > 0, &rs, st));
    const Sel ss{p->d_list_src, 0, (int32_t)hs.src.size()};
    const Sel sp{p->d_list_pair, 0, (int32_t)hs.pair.size()};
    const Sel si{p->d_list_item, 0, (int32_t)hs.item.size()};
    CHK(validate_theta(p, theta, nullptr, p->d_list_src, n, st));
    CHK(fill_u8(p->d_done, ss, 0, st));
    if (stored && n_steps > 0) CHK(render_stored(p, theta, rs, st));
    CHK(newton_run(p, theta, ss, sp, si, n_steps, prm, radius, st, stored && n_steps > 0));
    if (elbo_out) {
        // final ELBO_s at the returned point
        CHK(prep(p, theta, sp, false, DIR_NONE, nullptr, 0, st));
        CHK(adjoint(p, si, nullptr, false, BASE_BG, false, st));
        CHK(finalize(p, theta, ss, nullptr, false, DIR_NONE, nullptr, 0, false, elbo_out, nullptr, nullptr, 0, false,
                     st));
    }
    return CELESTE_OK;
}

int celeste_color_batches(const celeste_plan* p, uint64_t seed, int32_t* batch_ptr, int32_t* batch_src,
                          int32_t* n_batches) {
    if (!p || !batch_ptr || !batch_src || !n_batches) return CELESTE_EINVAL;
    const int S = p->n_src;
    std::vector<std::vector<int32_t>> adj(S);
    for (const PairDev& pd : p->pairs)
        for (int k = pd.nbr_begin; k < pd.nbr_end; ++k) {
            const int t = p->pairs[p->nbr[k]].src;
            if (t != pd.src) adj[pd.src].push_back(t);
        }
    std::vector<int32_t> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::mt19937_64 rng(seed);
    for (int i = S - 1; i > 0; --i) {   // Fisher-Yates with the engine's raw output
        const int j = (int)(rng() % (uint64_t)(i + 1));
        std::swap(order[i], order[j]);
    }
    std::vector<int32_t> color(S, -1);
    int n_col = 0;
    std::vector<int32_t> mark;
    for (int s : order) {
        for (int t : adj[s])
            if (color[t] >= 0) {
                if ((int)mark.size() <= color[t]) mark.resize(color[t] + 1, -1);
                mark[color[t]] = s;
            }
        int c = 0;
        while (c < (int)mark.size() && mark[c] == s) ++c;
        color[s] = c;
        n_col = std::max(n_col, c + 1);
    }
    std::vector<int32_t> cnt(n_col + 1, 0);
    for (int s = 0; s < S; ++s) cnt[color[s] + 1]++;
    for (int c = 0; c < n_col; ++c) cnt[c + 1] += cnt[c];
    for (int c = 0; c <= n_col; ++c) batch_ptr[c] = cnt[c];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int s = 0; s < S; ++s) batch_src[fill[color[s]]++] = s;
    *n_batches = n_col;
    return CELESTE_OK;
}

int celeste_plan_set_hessian_mode(celeste_plan* p, int mode) {
    if (!p || mode < 0 || mode > 1) return CELESTE_EINVAL;
    p->hess_mode = mode;
    return CELESTE_OK;
}

int celeste_conflict_graph(const celeste_plan* p, int32_t* adj_ptr, int32_t* adj, int64_t cap, int64_t* n_adj) {
    if (!p || !adj_ptr || !n_adj || cap < 0 || (cap > 0 && !adj)) return CELESTE_EINVAL;
    const int S = p->n_src;
    std::vector<std::vector<int32_t>> rows(S);
    for (const PairDev& pd : p->pairs)
        for (int k = pd.nbr_begin; k < pd.nbr_end; ++k) {
            const int t = p->pairs[p->nbr[k]].src;
            if (t != pd.src) rows[pd.src].push_back(t);
        }
    int64_t total = 0;
    for (auto& r : rows) {
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        total += (int64_t)r.size();
    }
    *n_adj = total;
    if (total > cap || total > INT32_MAX) return CELESTE_EINVAL;
    int64_t k = 0;
    for (int s = 0; s < S; ++s) {
        adj_ptr[s] = (int32_t)k;
        for (int32_t t : rows[s]) adj[k++] = t;
    }
    adj_ptr[S] = (int32_t)k;
    return CELESTE_OK;
}

int celeste_cyclades_batches(int32_t n, const int32_t* adj_ptr, const int32_t* adj, const int32_t* order,
                             int32_t sample_size, int32_t* batch_ptr, int32_t* batch_src, int32_t* n_batches,
                             int32_t* n_components) {
    if (n < 0 || sample_size < 1 || !adj_ptr || !batch_ptr || !n_batches || (n > 0 && (!order || !batch_src)))
        return CELESTE_EINVAL;
    if (adj_ptr[0] != 0) return CELESTE_EINVAL;
    for (int s = 0; s < n; ++s)
        if (adj_ptr[s + 1] < adj_ptr[s]) return CELESTE_EINVAL;
    if (adj_ptr[n] > 0 && !adj) return CELESTE_EINVAL;
    for (int32_t k = 0; k < adj_ptr[n]; ++k)
        if (adj[k] < 0 || adj[k] >= n) return CELESTE_EINVAL;
    std::vector<int32_t> pos(n, -1);   // position inside the current sample, -1 outside it
    for (int i = 0; i < n; ++i) {
        if (order[i] < 0 || order[i] >= n || pos[order[i]] != -1) return CELESTE_EINVAL;
        pos[order[i]] = 0;
    }
    std::fill(pos.begin(), pos.end(), -1);
    // disjoint-set forest over sample positions; the root of a set is its earliest member
    std::vector<int32_t> parent, comp_rank, member_round, round_cnt;
    auto find = [&](int32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    int32_t nb = 0, out = 0, comps = 0;
    batch_ptr[0] = 0;
    for (int32_t b0 = 0; b0 < n; b0 += sample_size) {
        const int32_t m = std::min(sample_size, n - b0);
        const int32_t* smp = order + b0;
        for (int32_t i = 0; i < m; ++i) pos[smp[i]] = i;
        parent.resize(m);
        std::iota(parent.begin(), parent.end(), 0);
        for (int32_t i = 0; i < m; ++i)
            for (int32_t k = adj_ptr[smp[i]]; k < adj_ptr[smp[i] + 1]; ++k) {
                const int32_t j = pos[adj[k]];
                if (j < 0) continue;
                const int32_t a = find(i), c = find(j);
                if (a != c) parent[std::max(a, c)] = std::min(a, c);
            }
        // round of a member = how many earlier members its component already has
        comp_rank.assign(m, 0);
        member_round.resize(m);
        int32_t rounds = 0;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t r = find(i);
            if (r == i) ++comps;
            member_round[i] = comp_rank[r]++;
            rounds = std::max(rounds, member_round[i] + 1);
        }
        // counting sort by round, stable in sample order
        round_cnt.assign(rounds + 1, 0);
        for (int32_t i = 0; i < m; ++i) round_cnt[member_round[i] + 1]++;
        for (int32_t r = 0; r < rounds; ++r) {
            round_cnt[r + 1] += round_cnt[r];
            batch_ptr[nb + r + 1] = out + round_cnt[r + 1];
        }
        for (int32_t i = 0; i < m; ++i) batch_src[out + round_cnt[member_round[i]]++] = smp[i];
        nb += rounds;
        out += m;
        for (int32_t i = 0; i < m; ++i) pos[smp[i]] = -1;
    }
    *n_batches = nb;
    if (n_components) *n_components = comps;
    return CELESTE_OK;
}

int celeste_sweep(celeste_plan* p, double* theta, const int32_t* batch_ptr, const int32_t* batch_src, int n_batches,
                  int n_sweeps, const celeste_tr_params* prm, double* elbo_trace, hipStream_t st) {
    if (!p || !theta || !batch_ptr || !batch_src || n_batches <= 0 || n_sweeps < 0 || !prm || !elbo_trace)
        return CELESTE_EINVAL;
    if (!(prm->radius0 > 0.0) || !(prm->radius_max >= prm->radius0) || !(prm->eta_accept >= 0.0) ||
        !(prm->eta_accept < 0.25) || !(prm->gtol >= 0.0) || prm->newton_steps < 0)
        return CELESTE_EINVAL;
    if (batch_ptr[0] != 0) return CELESTE_EINVAL;
    for (int b = 0; b < n_batches; ++b)
        if (batch_ptr[b + 1] < batch_ptr[b]) return CELESTE_EINVAL;
    const int total = batch_ptr[n_batches];
    for (int k = 0; k < total; ++k)
        if (batch_src[k] < 0 || batch_src[k] >= p->n_src) return CELESTE_EINVAL;
    // conflict check: no two members of a batch share a pixel; no source twice in a batch
    std::vector<int32_t> in_batch(p->n_src, -1);
    for (int b = 0; b < n_batches; ++b) {
        for (int k = batch_ptr[b]; k < batch_ptr[b + 1]; ++k) {
            if (in_batch[batch_src[k]] == b) return CELESTE_EINVAL;
            in_batch[batch_src[k]] = b;
        }
        for (int k = batch_ptr[b]; k < batch_ptr[b + 1]; ++k) {
            const int s = batch_src[k];
            for (int pi = p->patch_ptr[s]; pi < p->patch_ptr[s + 1]; ++pi)
                for (int q = p->pairs[pi].nbr_begin; q < p->pairs[pi].nbr_end; ++q) {
                    const int t = p->pairs[p->nbr[q]].src;
                    if (t != s && in_batch[t] == b) return CELESTE_ECONFLICT;
                }
        }
    }
    // all batches' lists, concatenated
    HostScope hs;
    std::vector<int32_t> off_src(n_batches + 1), off_pair(n_batches + 1), off_item(n_batches + 1);
    for (int b = 0; b < n_batches; ++b) {
        off_src[b] = (int32_t)hs.src.size();
        off_pair[b] = (int32_t)hs.pair.size();
        off_item[b] = (int32_t)hs.item.size();
        scope_lists(p, batch_src + batch_ptr[b], batch_ptr[b + 1] - batch_ptr[b], hs);
    }
    off_src[n_batches] = (int32_t)hs.src.size();
    off_pair[n_batches] = (int32_t)hs.pair.size();
    off_item[n_batches] = (int32_t)hs.item.size();
    // list buffers sized for one appearance of each source; grown (plan-owned) if a schedule
    // repeats sources, after the stream has finished with the old ones
    if (hs.src.size() > p->cap_list_src || hs.pair.size() > p->cap_list_pair || hs.item.size() > p->cap_list_item) {
        HIPCHK(hipStreamSynchronize(st));
        int32_t *ns = nullptr, *np_ = nullptr, *ni = nullptr;
        const size_t cs = std::max(hs.src.size(), p->cap_list_src), cp = std::max(hs.pair.size(), p->cap_list_pair),
                     ci = std::max(hs.item.size(), p->cap_list_item);
        if (hipMalloc((void**)&ns, cs * 4) != hipSuccess || hipMalloc((void**)&np_, cp * 4) != hipSuccess ||
            hipMalloc((void**)&ni, ci * 4) != hipSuccess) {
            (void)hipFree(ns);
            (void)hipFree(np_);
            (void)hipFree(ni);
            (void)hipGetLastError();
            return CELESTE_ENOMEM;
        }
        (void)hipFree(p->d_list_src);
        (void)hipFree(p->d_list_pair);
        (void)hipFree(p->d_list_item);
        p->d_list_src = ns;
        p->d_list_pair = np_;
        p->d_list_item = ni;
        p->cap_list_src = cs;
        p->cap_list_pair = cp;
        p->cap_list_item = ci;
    }
    CHK(upload_lists(p, hs, st));
    int32_t *dl_src = p->d_list_src, *dl_pair = p->d_list_pair, *dl_item = p->d_list_item;
    // With the strip render, the total ELBO leaves every box's own profile values and
    // coefficients current; each batch then takes its background from them, and its boxes
    // are rendered again at their new parameters before the next batch.
    const bool stored = p->render_mode == 2 || p->render_mode == 3;
    // one sweep over the schedule, then the total ELBO into `total`
    auto one_sweep = [&](double* total, hipStream_t s) -> int {
        for (int b = 0; b < n_batches; ++b) {
            const Sel ss{dl_src + off_src[b], 0, off_src[b + 1] - off_src[b]};
            const Sel sp{dl_pair + off_pair[b], 0, off_pair[b + 1] - off_pair[b]};
            const Sel si{dl_item + off_item[b], 0, off_item[b + 1] - off_item[b]};
            if (ss.n == 0) continue;
            CHK(fill_u8(p->d_done, ss, 0, s));
            // fresh trust region for every visit of a batch
            CHK(fill_f64(p->d_radius, ss, prm->radius0, s));
            CHK(newton_run(p, theta, ss, sp, si, prm->newton_steps, prm, p->d_radius, s, stored));
            if (!stored) continue;
            CHK(prep(p, theta, sp, false, DIR_NONE, nullptr, 0, s));
            HIPCHK(launch_strip_fg(si, p->geom(), p->d_tab1, p->d_fg, p->rows, p->launch_grid(), p->wpb,
                                   p->d_status, s));
        }
        if (!stored) return celeste_total_elbo(p, theta, total, s);
        // every box's stored own values and coefficients are current: the total needs the
        // gather only, not the strip pass
        CHK(gather(p, true, s));
        HIPCHK(launch_tile_total(p->d_tile_sums, (int)p->tiles.size(), theta, p->consts, p->n_src, p->d_tt_part, total,
                                 p->d_status, s));
        return CELESTE_OK;
    };
    CHK(celeste_total_elbo(p, theta, elbo_trace, st));
    if (!p->use_graph || n_sweeps == 0) {
        for (int sw = 0; sw < n_sweeps; ++sw) CHK(one_sweep(elbo_trace + sw + 1, st));
        return CELESTE_OK;
    }
    // graph mode: the sweep is captured once (its total into the plan's scalar) and replayed
    // n_sweeps times on `st`, each replay's total copied into the trace
    if (p->sweep_exec) {
        if (p->sweep_pending) HIPCHK(hipEventSynchronize(p->sweep_ev));
        p->sweep_pending = false;
        (void)hipGraphExecDestroy(p->sweep_exec);
        p->sweep_exec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = one_sweep(p->d_scalar, p->cap_stream);
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc != CELESTE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "sweep capture");
    const hipError_t e2 = hipGraphInstantiate(&p->sweep_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        p->sweep_exec = nullptr;
        return hip_fail(e2, "sweep graph instantiation");
    }
    for (int sw = 0; sw < n_sweeps; ++sw) {
        HIPCHK(hipGraphLaunch(p->sweep_exec, st));
        HIPCHK(hipMemcpyAsync(elbo_trace + sw + 1, p->d_scalar, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipEventRecord(p->sweep_ev, st));
    p->sweep_pending = true;
    return CELESTE_OK;
}

int celeste_autotune(celeste_plan* p, const double* theta, int reps, double* best_ms, hipStream_t st) {
    if (!p || !theta || reps < 1) return CELESTE_EINVAL;
    double* d_elbo = nullptr;
    double* d_grad = nullptr;
    if (hipMalloc((void**)&d_elbo, (size_t)p->n_src * 8) != hipSuccess) return CELESTE_ENOMEM;
    if (hipMalloc((void**)&d_grad, (size_t)p->n_src * ROW * 8) != hipSuccess) {
        (void)hipFree(d_elbo);
        return CELESTE_ENOMEM;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const bool graph = p->use_graph;
    p->use_graph = false;
    auto time_cfg = [&](double& ms) -> int {
        std::vector<double> t;
        for (int r = 0; r < reps + 1; ++r) {
            HIPCHK(hipEventRecord(e0, st));
            CHK(batched_sequence(p, theta, nullptr, true, d_elbo, d_grad, st));
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float f = 0.f;
            HIPCHK(hipEventElapsedTime(&f, e0, e1));
            if (r > 0) t.push_back(f);
        }
        std::sort(t.begin(), t.end());
        ms = t[t.size() / 2];
        return CELESTE_OK;
    };
    struct Cfg { int chunk, wpb, grid, dyn, th, tw, rows, rmode; };
    Cfg best{p->chunk, p->wpb, p->launch_grid(), p->dynamic, p->tile_h, p->tile_w, p->rows, p->render_mode};
    double best_t = 1e300;
    int rc = celeste_plan_set_launch(p, best.chunk, best.wpb, best.grid, best.dyn, best.th, best.tw, best.rows,
                                     best.rmode);
    if (rc == CELESTE_OK) rc = time_cfg(best_t);
    auto trial = [&](Cfg c) {
        if (rc != CELESTE_OK) return;
        rc = celeste_plan_set_launch(p, c.chunk, c.wpb, c.grid, c.dyn, c.th, c.tw, c.rows, c.rmode);
        if (rc != CELESTE_OK) return;
        double t = 0;
        rc = time_cfg(t);
        // a candidate must beat the current choice by 1%, about the spread of the medians of
        // one configuration, so that timing noise does not move the choice
        if (rc == CELESTE_OK && t < 0.99 * best_t) {
            best_t = t;
            best = c;
        }
    };
    // render mode and strip height interact (the register footprint of the fused adjoint
    // depends on both), so they are searched jointly first; then one coordinate pass over the
    // remaining knobs, and a second joint pass at the chosen launch shape
    auto mode_rows = [&]() {
        const Cfg start = best;
        for (int m : {0, 1, 2, 3})
            for (int r : {4, 8, 16}) {
                Cfg c = start;
                c.rmode = m;
                c.rows = r;
                if (c.rmode != start.rmode || c.rows != start.rows) trial(c);
            }
    };
    mode_rows();
    Cfg c = best;
    for (int ch : {64, 128, 256, 512, 1024}) { c = best; c.chunk = ch; trial(c); }
    // waves per block and grid jointly: the cost of a work item varies with the Gaussians
    // it culls, and a block holds its slots until its slowest wave ends, so smaller blocks
    // pay off most with one item per wave (the largest grid, clipped to the item count)
    {
        const Cfg start = best;
        for (int w : {1, 2, 4})
            for (int g : {p->n_cu, 4 * p->n_cu, 16 * p->n_cu, 64 * p->n_cu, 128 * p->n_cu, 1 << 20}) {
                c = start;
                c.wpb = w;
                c.grid = g;
                if (c.wpb != start.wpb || c.grid != start.grid) trial(c);
            }
    }
    for (int d : {0, 1}) { c = best; c.dyn = d; trial(c); }
    if (best.rmode == 1 || best.rmode == 2) {
        const int tiles[5][2] = {{8, 8}, {4, 16}, {16, 8}, {8, 16}, {16, 16}};
        for (auto& tl : tiles) { c = best; c.th = tl[0]; c.tw = tl[1]; trial(c); }
    }
    mode_rows();
    if (rc == CELESTE_OK)
        rc = celeste_plan_set_launch(p, best.chunk, best.wpb, best.grid, best.dyn, best.th, best.tw, best.rows,
                                     best.rmode);
    p->use_graph = graph;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_elbo);
    (void)hipFree(d_grad);
    if (best_ms) *best_ms = best_t;
    return rc;
}

}  // extern "C"
