// Internal layouts shared by the HIP kernels and the host side of libceleste.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "celeste.h"
#include "dual.h"

namespace cel {

constexpr int NPSF = 3;
constexpr int NDEV = 8;
constexpr int NEXP = 6;
constexpr int NGAL_PER_PSF = NDEV + NEXP;                 // 14
constexpr int NCOMP = NPSF * (1 + NGAL_PER_PSF);           // 45 Gaussians per (source, image)
constexpr int CST = 10;                                    // fields per component entry
constexpr int NP = 27;                                     // parameters the pixel terms depend on
constexpr int NMIX = 8;                                    // components of a type's colour-prior mixture
constexpr int NPK = NP + 2 * NMIX;                         // parameters with the mixture responsibilities
constexpr int ROW = 48;                                    // padded row of theta / grad
constexpr int MIXF = 24;                                   // fields of one colour-prior mixture component
constexpr int NCOEF = 4;                                   // per-(source, image) brightness factors

// Fields of one component entry of a (source, image) table.  For the Gaussian
// N(p; mean, S) scaled by a weight w: log_w = log(w / (2 pi sqrt(det S))), P = S^-1.
enum CompField {
    F_CX = 0, F_CY, F_PXX, F_PXY, F_PYY, F_LOGW,
    F_WT,    // galaxy: frac_dev (de Vaucouleurs) or 1 - frac_dev (exponential); star: 1
    F_WNU,   // galaxy: F_WT * nu_j (the component covariance is nu_j Sigma_shape + PSF)
    F_SGN,   // +1 de Vaucouleurs, -1 exponential, 0 star
    F_RDY    // exp(-P_yy): ratio of successive row-to-row factors down a column
};

// Per-(source, image) brightness factors: the source's expected light is
// k1 f_star + k2 f_gal and its second moment k3 f_star^2 + k4 f_gal^2 with
// k1 = iota q E[flux|star], k2 = iota (1-q) E[flux|gal],
// k3 = iota^2 q E[flux^2|star], k4 = iota^2 (1-q) E[flux^2|gal].
enum Coef { C_K1 = 0, C_K2, C_K3, C_K4 };

// Accumulators of one work item (sums over its pixels of the pixel term and of its
// derivatives with respect to the intermediate quantities of the own source).
enum AccField {
    A_VAL = 0,        // sum of pixel terms
    A_K1, A_K2, A_K3, A_K4,   // d/dk1..k4
    A_UX, A_UY,       // d/d position
    A_FDEV,           // d/d frac_dev
    A_SXX, A_SXY, A_SYY,      // 2 d/dSxx, d/dSxy, 2 d/dSyy of the galaxy shape covariance
    NACC
};

// Intermediate quantities of one (source, image) pair through which the pixel terms depend
// on the source's parameters: the brightness factors k1..k4, the position, frac_dev and the
// galaxy shape covariance.  The order matches the accumulators A_K1..A_SYY (index + 1).
enum WField { W_K1 = 0, W_K2, W_K3, W_K4, W_UX, W_UY, W_FDEV, W_SXX, W_SXY, W_SYY, NW };

// Second derivatives of a box's pixel sum in its brightness factors k1..k4 and frac_dev f
// (the pixel-level rows of the intermediate Hessian): (k1k1, k1k2, k2k2, k1k3, k1k4, k2k3,
// k2k4, fk1, fk2, fk3, fk4, ff); the (k3, k4) block is zero.  Stored per work item, padded.
enum KKField { KK_11, KK_12, KK_22, KK_13, KK_14, KK_23, KK_24, KK_F1, KK_F2, KK_F3, KK_F4, KK_FF, NKK_USED,
               NKK = 16 };

// Closed-form block of a box's intermediate Hessian (k_hess_geom), in the accumulator
// scaling (s_ij = c_ij d/dS_ij, c = 2 on the diagonal): NHG_GEO entries between the
// geometric intermediates (ux, uy, frac_dev, Sxx, Sxy, Syy) = 0..5, every pair but
// (frac_dev, frac_dev), then 4 entries (k1..k4) for each of ux, uy, Sxx, Sxy, Syy.
enum HGField {
    HG_XX, HG_XY, HG_YY, HG_XF, HG_YF,
    HG_X_SXX, HG_X_SXY, HG_X_SYY, HG_Y_SXX, HG_Y_SXY, HG_Y_SYY,
    HG_F_SXX, HG_F_SXY, HG_F_SYY,
    HG_SXX_SXX, HG_SXX_SXY, HG_SXX_SYY, HG_SXY_SXY, HG_SXY_SYY, HG_SYY_SYY,
    NHG_GEO,
    NHG = NHG_GEO + 20
};
constexpr int NGAL = NPSF * NGAL_PER_PSF;   // 42 galaxy components per box

__host__ __device__ constexpr int hg_row(int q) {
    constexpr int r[NHG_GEO] = {0, 0, 1, 0, 1, 0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 5};
    return r[q];
}
__host__ __device__ constexpr int hg_col(int q) {
    constexpr int c[NHG_GEO] = {0, 1, 1, 2, 2, 3, 4, 5, 3, 4, 5, 3, 4, 5, 3, 4, 5, 4, 5, 5};
    return c[q];
}

struct PairDev {              // one box (source, image)
    int32_t src, img, r0, c0, h, w;
    int64_t visit_off;        // first visit of the box in the global visit numbering
    int32_t item_begin, item_end;   // work items of this box in the full item list
    int32_t nbr_begin, nbr_end;     // other boxes of the same image that intersect it
};

struct Item {                 // a run of strips of one box: strips start .. start + count - 1
    int32_t pair, start, count, pad;
};

struct TileDev {              // a tile_h x tile_w render tile and its box list
    int32_t img, r0, c0, list_begin, list_end, pad;
};

// One component of a type's colour-prior mixture, [2][NMIX][MIXF] in device memory: weight,
// its log, mean[4], precision P = S^-1 (row-major 4 x 4), log det S, padding.
enum MixField { MX_W = 0, MX_LOGW, MX_MEAN, MX_P = MX_MEAN + 4, MX_LOGDET = MX_P + 16 };

struct Consts {
    double exp_alpha[NEXP], exp_nu[NEXP], dev_alpha[NDEV], dev_nu[NDEV];
    double prior_phi, prior_r[2][2], prior_c[2][2][4];
    const double* mix;         // colour-prior mixture table (CELESTE_COLOR_MIXTURE), or null
    uint32_t flags;
    int32_t npar;              // parameters per source: NP, or NPK with the mixture
};

// A subset of sources / boxes / items: entry j is ids[j] if ids is set, else base + j.
struct Sel {
    const int32_t* ids;
    int32_t base, n;
};
__host__ __device__ inline int32_t sel_at(const Sel& s, int32_t j) { return s.ids ? s.ids[j] : s.base + j; }

enum BaseMode {
    BASE_PLANES = 0,   // E, V planes of all sources (own included)
    BASE_BG = 1,       // per-visit background excluding the own source
    BASE_NBR = 2,      // background evaluated on the fly from the overlapping boxes
    BASE_FG = 3        // background from the overlapping boxes' stored profile values
};

// Direction seeding of the tangent pass: a vector in parameter space, a parameter unit
// vector, or a unit vector of a pair's intermediates (see WField in model.h).
enum DirMode { DIR_NONE = 0, DIR_VEC = 1, DIR_UNIT = 2, DIR_W = 3 };

struct Geometry {
    const celeste_image* images;
    const PairDev* pairs;
    const Item* items;
    const int32_t* nbr;
    const double* x;
    Consts consts;
};

struct PrepArgs {
    Geometry g;
    const double* theta;       // [S][32]
    const double* dir;         // [S][32] when dir_mode == DIR_VEC
    int32_t dir_mode, dir_unit;
    Sel pairs;
    double* tab;               // [n_pairs][NCOMP][CST] of T
    double* coef;              // [n_pairs][NCOEF] of T
    const int* status;
};

struct RenderArgs {
    Geometry g;
    const TileDev* tiles;
    const int32_t* tile_list;
    int32_t n_tiles, tile_h, tile_w, pad;
    const double* tab;         // double tables
    const double* coef;
    double* E;
    double* V;
    double* tile_sums;         // [n_tiles] pixel-term sums of covered pixels, or null
    const int* status;
};

struct AdjArgs {
    Geometry g;
    Sel items;
    const uint8_t* active;     // [S] or null
    const double* tab;         // T tables
    const double* coef;
    const double* tab_val;     // double tables used for overlapping boxes (BASE_NBR)
    const double* coef_val;
    int32_t dynamic;
    int* counter;
    const double* E;
    const double* V;
    const double* bg;          // [n_visits][2]
    const double* fg;          // [n_visits][2] own profile values from the render, or null
    double* partials;          // [n_items_total][NACC] of T
    double* kk;                // [n_items_total][NKK]: brightness-factor block of the box's
                               // intermediate Hessian (double gradient passes), or null
    double* fg_out;            // [n_visits][2]: own profile values written by the passes that
                               // fill kk, or null
    const int* status;
};

struct BgArgs {
    Geometry g;
    Sel items;
    const double* tab_val;
    const double* coef_val;
    const double* fg;          // [n_visits][2] current stored own values: background from them, or null
    double* bg;
    const int* status;
};

struct FinArgs {
    Geometry g;
    Sel srcs;
    const uint8_t* active;
    const double* theta;
    const double* dir;
    int32_t dir_mode, dir_unit;
    const int32_t* patch_ptr;  // device [S+1]
    const double* pair_lgamma; // [n_pairs] sum of log(x!) over each box, or null
    const double* partials;
    int32_t deriv;             // 0: value only
    double* elbo;              // [S] or null
    double* grad;              // [S][32] or null: value parts of the gradient
    double* tangent;           // [S][32] or null: tangent parts (Hessian-vector product)
    int64_t tangent_stride;    // row stride of `tangent` in doubles
    int32_t tangent_by_list;   // 1: row j of `tangent` is list entry j (not source id)
    int32_t tangent_pad;       // 1: also zero entries 27..31 of each row
    const int* status;
};

// Kernel launchers (kernels.hip)
hipError_t launch_validate(const double* theta, const uint8_t* active, const int32_t* list, int n,
                           int S, int npar, int* status, hipStream_t st);
hipError_t launch_prep(const PrepArgs& a, bool tangent, hipStream_t st);
hipError_t launch_render(const RenderArgs& a, int waves_per_block, hipStream_t st);
// strips.hip
hipError_t launch_adjoint(const AdjArgs& a, bool tangent, int base_mode, bool deriv, int grid,
                          int waves_per_block, int strip_rows, hipStream_t st);
hipError_t launch_background(const BgArgs& a, int grid, int waves_per_block, int strip_rows, hipStream_t st);
// Closed-form geometric block of each listed item's box Hessian into hg[item][NHG]
// (tables a.tab / a.coef in double, stored backgrounds a.bg, own values a.fg; nu[NGAL] the
// nu of each galaxy component): k_hess_second, then k_hess_geom.
hipError_t launch_hess_geom(const AdjArgs& a, const double* nu, double* hg, int grid, int waves_per_block,
                            int strip_rows, hipStream_t st);
hipError_t launch_debug_math(int fn, const double* x, double* y, int n, hipStream_t st);
hipError_t launch_pair_lgamma(const Geometry& g, int n_pairs, double* out, hipStream_t st);
hipError_t launch_fill_planes(const celeste_image* images, int n_img, int max_pix, double* E, double* V,
                              const int* status, hipStream_t st);
hipError_t launch_strip_fg(const Sel& items, const Geometry& g, const double* tab, double* fg, int strip_rows, int grid,
                           int waves_per_block, const int* status, hipStream_t st);
hipError_t launch_gather_planes(const RenderArgs& a, const double* fg, int waves_per_block, hipStream_t st);
hipError_t launch_render_strips(const Sel& items, const Geometry& g, const double* tab, const double* coef,
                                double* E, double* V, int strip_rows, int grid, int waves_per_block,
                                const int* status, hipStream_t st);
hipError_t launch_finalize(const FinArgs& a, bool tangent, hipStream_t st);
// Total ELBO from the per-tile sums and every KL; part: device scratch of 1024 doubles.
hipError_t launch_tile_total(const double* tile_sums, int n_tiles, const double* theta, const Consts& c,
                             int S, double* part, double* out, const int* status, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st);
// Work counts of the strip passes under the component culling (k_live_counts): strips,
// visits, evaluated PSF groups, live stars, live galaxy components and zero-component pads,
// the last four per strip and per visit.
constexpr int NLIVE_COUNTS = 9;
hipError_t launch_live_counts(const Sel& sel, const Geometry& g, const double* tab, int L,
                              unsigned long long* out, const int* status, hipStream_t st);

hipError_t launch_fill_u8_sel(uint8_t* p, const Sel& s, uint8_t v, hipStream_t st);
hipError_t launch_fill_f64_sel(double* p, const Sel& s, double v, hipStream_t st);

// Per-box sums of item partials: value parts into gw[pair][NACC] and, with kk, the k-block
// hw[pair][0..3][0..3] (double pass), or the tangent parts of accumulators 1..10 into
// hw[pair][dir][10] (tangent pass along a pair-intermediate direction).
hipError_t launch_pair_reduce(const Sel& pairs, const PairDev* dpairs, const double* partials, const double* kk,
                              bool tangent, int dir, double* gw, double* hw, const int* status, hipStream_t st);
// Per-box sums of hg into the position and shape rows of hw[pair] (hw[pair][dir][f] =
// c_f d2L / dw_dir dw_f, as the tangent passes give them).
hipError_t launch_pair_hess(const Sel& pairs, const PairDev* dpairs, const double* hg, double* hw, const int* status,
                            hipStream_t st);
// 27x27 Hessians of the listed sources (hess by list position) from gw, hw and the KL.
hipError_t launch_assemble_hessian(const Sel& srcs, const Geometry& g, const int32_t* patch_ptr,
                                   const double* theta, const double* gw, const double* hw, double* hess,
                                   const int* status, hipStream_t st);

// Entry point without allocation (noalloc.hip): the batched ELBO + gradient of api.cpp with
// the per-item partial sums and the work-queue counter at the given device addresses.
int batched_elbo_grad_scratch(celeste_plan* p, const double* theta, const uint8_t* active, double* elbo,
                              double* grad, double* partials, int* counter, hipStream_t st);
int64_t plan_item_count(const celeste_plan* p);
int plan_device(const celeste_plan* p);
// Looks up (once per device, with that device current) the device address of the static
// scratch array of noalloc.hip; CELESTE_OK or CELESTE_EHIP.
int noalloc_attach(int device);

// Trust region (tr.hip)
struct TrArgs {
    Sel srcs;
    double* theta;             // [S][32] current point, updated by tr_update
    double* grad;              // [S][32] natural-space gradient at theta
    double* hess;              // [n][27][27] by list position
    const double* grad_trial;  // [S][32] gradient at the trial point, or null
    const double* hess_trial;  // [n][27][27] Hessian at the trial point, or null
    uint8_t* accepted;         // [S] set by tr_update: the trial point became the current one
    double* radius;            // [S]
    double* theta_trial;       // [S][32]
    double* pred;              // [S] predicted increase
    double* elbo_cur;          // [S]
    const double* elbo_trial;  // [S]
    uint8_t* done;             // [S]
    uint8_t* live;             // [S] set by tr_solve: the source takes a step this iteration
    double eta_accept, radius_max, gtol;
    int32_t npar;              // NP, or NPK with the colour-prior mixture (Hessian rows and columns)
    int* status;
};
hipError_t launch_tr_solve(const TrArgs& a, hipStream_t st);
hipError_t launch_tr_update(const TrArgs& a, hipStream_t st);
// Gradient and Hessian of the trial point become the current ones where it was accepted.
hipError_t launch_tr_adopt(const TrArgs& a, hipStream_t st);

}  // namespace cel
