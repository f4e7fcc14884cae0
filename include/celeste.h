/*
 * celeste.h - C ABI of the MI355X FP64 ELBO library (libceleste.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the variational lower
 * bound of the Celeste astronomical-catalog model (Regier et al. 2018, Section III,
 * Eq. (1)) per light source, its gradient (a hand-written adjoint), its per-source
 * Hessian-vector product (the tangent of that adjoint), batched Newton trust-region
 * steps for many sources at once (Section IV-D) and block-coordinate-ascent sweeps
 * over conflict-free batches of sources (Section IV-D).
 *
 * Model, per image n (band b_n, sky level eps_n(m), calibration iota_n, 3-component
 * Gaussian PSF in the image frame, local linear astrometry: a world point u is at
 * image-frame position wcs_n (u - origin_n)) and pixel m (centre (x = col, y = row) in
 * the image frame) - the image metadata of Section III read this way:
 *   E_s(m)   = iota_n [q a_star f_star(m) + (1-q) a_gal f_gal(m)]
 *   Var_s(m) = iota_n^2 [q b_star f_star^2 + (1-q) b_gal f_gal^2] - E_s(m)^2
 *   E(m) = eps_n(m) + sum_t E_t(m),  V(m) = sum_t Var_t(m)   over sources t whose box
 *   in image n contains m;  a = E[flux_b], b = E[flux_b^2] of the log-normal band flux;
 *   pixel term  l(m) = x_m (log E - V / (2 E^2)) - E   (second-order expansion of
 *   E[log F] about E[F]);  ELBO_s = sum over s's own boxes of l(m) - KL_s.
 * f_star is the PSF; f_gal mixes an exponential and a de Vaucouleurs profile (each a
 * Gaussian mixture given in the problem description) sheared by the galaxy shape
 * radius^2 R(angle) diag(1, ratio^2) R(angle)^T (world frame; wcs S wcs^T in the image)
 * and convolved with the PSF.
 *
 * Parameters: theta is a device array [n_src][48] of float64, one row per source:
 *   0 u_x, 1 u_y (world pixels), 2 frac_dev in [0,1], 3 axis ratio in (0,1],
 *   4 angle (rad, counter-clockwise from +x to the major axis), 5 half-light radius
 *   (px, > 0), 6 q = probability of a star in (0,1),
 *   7..16 star: r_mu, r_var, c_mu[4], c_var[4];  17..26 galaxy: same;
 *   27..34 star, 35..42 galaxy: responsibilities kappa[8] of the colour-prior mixture
 *   components (CELESTE_COLOR_MIXTURE only: each type's eight positive, summing to 1;
 *   ignored otherwise);  43..47 unused.
 *   r is the log reference-band (r) flux, c_k = log(flux_{k+1}/flux_k) over u,g,r,i,z;
 *   *_var are variances (> 0).  A source has n_params = 27 parameters, or 43 with the
 *   colour-prior mixture (the paper's 44 count the type as a two-entry simplex; here
 *   q_gal = 1 - q).  Gradients are taken with respect to these entries.
 *
 * Conventions for every call:
 *  - Pointers documented "device" must be device memory of the current HIP device;
 *    "host" pointers are read during the call only.  The caller owns all of them.
 *  - Calls are stream-ordered and asynchronous unless documented otherwise.  Domain
 *    checks of theta run on the device; a failure leaves the outputs of that call
 *    untouched and is reported by celeste_plan_status().
 *  - Return value: CELESTE_OK or a negative CELESTE_E* code.  Nothing is thrown.
 *  - A plan is used from one host thread and one stream at a time; distinct plans
 *    are independent.  Calls on one plan must not overlap.
 */
#ifndef CELESTE_H
#define CELESTE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CELESTE_ABI_VERSION 7

enum celeste_status {
    CELESTE_OK = 0,
    CELESTE_EINVAL = -1,     /* bad size, pointer, geometry or parameter */
    CELESTE_ECONFLICT = -2,  /* two members of one batch share a pixel */
    CELESTE_EHIP = -3,       /* a HIP runtime call failed (detail: celeste_last_hip_error) */
    CELESTE_ENOMEM = -4,     /* device allocation failed */
    CELESTE_EDOMAIN = -5,    /* theta (or a trust-region trial) left the parameter domain */
    CELESTE_ESCRATCH = -6    /* the problem needs more than celeste_elbo_grad_noalloc's static scratch */
};

enum celeste_mode {
    CELESTE_PLAIN = 0,    /* one launch per source, overlapping sources evaluated on the fly */
    CELESTE_BATCHED = 1   /* all sources: render pass + one grid-stride fused adjoint launch */
};

enum celeste_flags {
    CELESTE_INCLUDE_KL = 1,       /* subtract KL(q || prior) from each ELBO_s */
    CELESTE_INCLUDE_LGAMMA = 2,   /* include the -log(x!) constant in every pixel term */
    CELESTE_COLOR_MIXTURE = 4     /* colour prior: a Gaussian mixture per type (color_mix_*), with
                                     the component responsibilities kappa in theta (43 parameters):
                                     a type's colour KL term is KL(Cat(kappa) || Cat(w)) +
                                     sum_d kappa_d KL(N(c_mu, diag c_var) || N(mean_d, cov_d)) */
};

/* One image: header of a row-major H x W plane of float64 counts inside x (H * W < 2^29). */
typedef struct celeste_image {
    int32_t band;         /* 0..4 = u, g, r, i, z */
    int32_t H, W;
    int32_t reserved;
    int64_t pix_offset;   /* offset of pixel (0, 0) in x */
    double sky;           /* eps_n > 0, expected sky counts per pixel (when sky_map is NULL) */
    double iota;          /* iota_n > 0, counts per unit flux */
    double origin_x, origin_y;   /* world coordinates mapped to pixel (row 0, col 0) */
    double psf[3][6];     /* per component: weight > 0, mean offset x, y, covariance xx, xy, yy
                             (image frame) */
    const double* sky_map;   /* device [H][W] row-major sky level of every pixel (> 0), or NULL:
                                `sky` everywhere.  Owned by the caller, alive as long as the plan */
    double wcs[2][2];     /* local linear astrometry: image-frame offset (x = col, y = row) =
                             wcs * (world point - origin); identity for a pure translation.
                             A galaxy's world-frame shape covariance S appears as wcs S wcs^T */
} celeste_image;

/* A source's patch ("active pixels") in one image: rows r0..r0+h-1, cols c0..c0+w-1
   (h * w < 2^28). */
typedef struct celeste_box {
    int32_t img, r0, c0, h, w;
} celeste_box;

typedef struct celeste_problem_desc {
    int32_t n_img;
    int32_t n_src;
    const celeste_image* images;   /* host [n_img] */
    const double* x;               /* device [n_pix]; NaN marks a masked pixel */
    int64_t n_pix;
    const int32_t* patch_ptr;      /* host [n_src + 1], CSR into boxes */
    const celeste_box* boxes;      /* host [patch_ptr[n_src]]; at most one box per (source, image) */
    double exp_alpha[6], exp_nu[6];    /* exponential profile: weights (sum 1) and variances */
    double dev_alpha[8], dev_nu[8];    /* de Vaucouleurs profile */
    double prior_phi;              /* prior probability of a star, (0, 1) */
    double prior_r[2][2];          /* [star, galaxy][mean, variance] of log r-band flux */
    double prior_c[2][2][4];       /* [star, galaxy][mean, variance][colour k] (without the mixture) */
    uint32_t flags;                /* celeste_flags */
    int32_t reserved;
    /* colour-prior mixture (read with CELESTE_COLOR_MIXTURE only): per type 8 components with
       weights > 0 summing to 1, means and symmetric positive definite covariances */
    double color_mix_w[2][8];
    double color_mix_mean[2][8][4];
    double color_mix_cov[2][8][4][4];
} celeste_problem_desc;

/* Trust-region constants (Nocedal & Wright, Ch. 4) for celeste_newton / celeste_sweep. */
typedef struct celeste_tr_params {
    double radius0;        /* initial radius (unconstrained coordinates), e.g. 1 */
    double radius_max;     /* e.g. 1e3 */
    double eta_accept;     /* accept the step if actual/predicted > eta_accept, e.g. 0.1 */
    double gtol;           /* a source stops once max |grad| in unconstrained space < gtol */
    int32_t newton_steps;  /* Newton iterations per source per batch visit (celeste_sweep) */
    int32_t reserved;
} celeste_tr_params;

typedef struct celeste_plan_info {
    int64_t n_visits;      /* sum over boxes of h*w: (source, pixel) pairs of one evaluation */
    int64_t n_pairs;       /* boxes */
    int64_t n_items;       /* work items of the fused adjoint launch */
    int64_t n_tiles;       /* render tiles touched by at least one box */
    int64_t n_nbr;         /* entries of the box-overlap lists used by the plain form */
    int32_t chunk;         /* strips per adjoint work item */
    int32_t waves_per_block;
    int32_t grid_blocks;   /* grid size (blocks) of the grid-stride strip and adjoint launches */
    int32_t tile_h, tile_w;
    int32_t dynamic_queue; /* 1: items popped from a device counter; 0: static round robin */
    int32_t strip_rows;    /* pixels per strip: a lane walks one column of a box this many rows */
    int32_t render_mode;   /* 0: strips per conflict-free class of boxes; 1: binned tiles evaluating
                              the Gaussians; 2 (default): one strip pass storing each visit's own
                              profile values, then a binned-tile gather (the fused adjoint reuses
                              them); 3: the stored values only - the fused adjoint sums each
                              pixel's background from the overlapping boxes' values, no planes */
    int32_t n_classes;     /* conflict-free classes of boxes (render launches) */
    int32_t n_params;      /* parameters per source: 27, or 43 with CELESTE_COLOR_MIXTURE */
    int64_t workspace_bytes;
} celeste_plan_info;

typedef struct celeste_plan celeste_plan;

/* Validates the problem (Section III model: boxes inside images, positive PSF
 * covariances (eigenvalues >= 0.01 px^2) and weights, sky (every sky-map entry) and
 * iota > 0, invertible astrometry, mixture variances > 0, one box per (source, image)),
 * bins boxes into render tiles and work items, and allocates the plan-owned device
 * workspace, sized for every later evaluation, Hessian, Newton and sweep call.  Besides
 * this call only celeste_plan_set_launch (grown tile buffers for smaller tiles),
 * celeste_autotune (its own timing outputs) and celeste_sweep (grown list buffers when a
 * schedule lists sources more often than once in total) allocate device memory;
 * celeste_elbo_grad_noalloc never does.  Synchronous.  *out receives the plan.
 * Returns CELESTE_EINVAL (nothing allocated), CELESTE_ENOMEM or CELESTE_EHIP. */
int celeste_plan_create(const celeste_problem_desc* desc, celeste_plan** out);

/* Frees the plan's own memory (never the caller's).  NULL is a no-op. */
void celeste_plan_destroy(celeste_plan* plan);

/* Sizes and the current launch configuration (host *info). */
int celeste_plan_get_info(const celeste_plan* plan, celeste_plan_info* info);

/* Per-source ELBO_s (Eq. (1) restricted to s's boxes, other sources fixed) into
 * elbo[n_src] (device).  active: device [n_src] bytes, nonzero = evaluate, or NULL
 * for all; entries of inactive sources are left untouched.  mode: celeste_mode. */
int celeste_elbo(celeste_plan* plan, const double* theta, const uint8_t* active, int mode,
                 double* elbo, hipStream_t stream);

/* ELBO_s and its gradient with respect to theta[s][0..n_params-1] (device
 * grad[n_src][48], the other entries set to 0), from the hand-written adjoint of Eq. (1)'s pixel terms
 * (Section III model) plus the KL's closed-form gradient.  No per-pixel tape: with
 * render modes 0 and 1 the fused adjoint recomputes each visit's own profile values; with
 * modes 2 (the default) and 3 the render stores them (16 B per visit in plan memory) and
 * the adjoint reads them back instead of evaluating the 45 Gaussians a second time.  The
 * strip kernels leave out of a work item every Gaussian that stays below exp(-50) of its
 * own peak on all of the item's pixels (celeste_work_counts): a change far below the
 * rounding of any pixel's expected count, which holds the sky. */
int celeste_elbo_grad(celeste_plan* plan, const double* theta, const uint8_t* active, int mode,
                      double* elbo, double* grad, hipStream_t stream);

/* Size of the static device scratch of celeste_elbo_grad_noalloc (bytes, per device). */
#define CELESTE_NOALLOC_SCRATCH_BYTES (8u << 20)

/* For callers that cannot allocate device memory at the time of the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): celeste_elbo_grad
 * in the batched form (same kernels, bitwise the same results, never a graph replay), with
 * its per-work-item partial sums and work-queue counter in a static device array of
 * CELESTE_NOALLOC_SCRATCH_BYTES per device instead of plan memory.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the array's address is
 * looked up once per device by celeste_plan_create, and the array lives until the process
 * ends.  Plans whose work items need more than 8 MiB - 256 B of partial sums (88 B per work
 * item: 95 322 items, e.g. the 2000-source field at 16- or 8-row strips but not at 4-row
 * strips) get CELESTE_ESCRATCH with nothing launched and the outputs untouched.  Every call
 * on one device shares that device's array: calls that overlap on one device (on any plans,
 * streams or threads) race and must be serialised by the caller.  Otherwise as
 * celeste_elbo_grad with mode CELESTE_BATCHED. */
int celeste_elbo_grad_noalloc(celeste_plan* plan, const double* theta, const uint8_t* active, double* elbo,
                              double* grad, hipStream_t stream);

/* Block-diagonal Hessian-vector product (the exact second derivatives Newton's method
 * needs, Section IV-D): hv[s] = (d^2 ELBO_s / d theta_s^2) v[s] (device [n_src][48];
 * entries from n_params on ignored in v and set to 0 in hv).  Computed as the forward-mode tangent of
 * the adjoint.  grad (device [n_src][48] or NULL) receives the gradient as a by-product.
 * All sources, batched form. */
int celeste_hvp(celeste_plan* plan, const double* theta, const double* v, double* hv,
                double* grad, hipStream_t stream);

/* Dense per-source Hessians hess[k][n_params][n_params] (device, row-major) of the n listed
 * sources src[k] (host list of distinct ids; CELESTE_EINVAL otherwise), the exact
 * second derivatives of Section IV-D: each box's Hessian in its ten intermediates
 * (brightness factors and frac_dev from the gradient pass, position and shape from a
 * closed-form pass, or from tangent-adjoint passes: celeste_plan_set_hessian_mode)
 * pushed through the chain rule and its tangent, plus the KL.  Stream-ordered: the source,
 * box and item lists go up through the plan's pinned staging on `stream` (the host waits
 * only if the previous list upload of this plan is still being copied; a longer list than
 * before grows the staging, a pinned host allocation). */
int celeste_hessian(celeste_plan* plan, const double* theta, const int32_t* src, int n,
                    double* hess, hipStream_t stream);

/* Newton trust-region iterations (Section IV-D) for the n sources src[] (host list,
 * distinct).  Each listed source is optimised with every other source held at its
 * value in theta at entry.  Per iteration: gradient, dense Hessian (27 x 27, or 43 x 43
 * with the colour-prior mixture), exact trust-region subproblem in unconstrained
 * coordinates (logit of q, frac_dev, axis ratio; log of radius and variances; with the
 * mixture, each type's responsibilities through a softmax whose last logit is fixed at 0:
 * 41 coordinates) on the Householder tridiagonal form of the Hessian (secular equation;
 * the eigendecomposition near the hard case), trial evaluation, accept/reject and radius
 * update - all on the device.
 * theta_inout (device [n_src][48]) is updated in place; radius (device [n_src]) is
 * read and written (initialise with params->radius0); elbo_out (device [n_src] or
 * NULL) receives the final ELBO_s of the listed sources.  Stream-ordered, with the list
 * upload of celeste_hessian; no host synchronisation between iterations. */
int celeste_newton(celeste_plan* plan, double* theta_inout, const int32_t* src, int n,
                   int n_steps, const celeste_tr_params* params, double* radius,
                   double* elbo_out, hipStream_t stream);

/* Work of the batched path's strip passes at theta (device [n_src][48]) under the
 * component culling of the strip kernels (a Gaussian whose quadratic form exceeds 100 on
 * every pixel of a work item, i.e. below exp(-50) of its own peak there, is left out of
 * that item's strips), for FLOP counts: counts (host int64[9]) = strips, visits, PSF groups
 * evaluated x strips, live star components x strips, live galaxy components x strips,
 * zero-component pads x strips (an odd number of live galaxy components in a group is
 * padded to a pair), then live stars, live galaxy components and pads x visits, all
 * summed over the work items of the current launch configuration.  Builds the tables,
 * counts with the kernels' own test and synchronises the stream; CELESTE_EDOMAIN if theta
 * leaves the parameter domain. */
int celeste_work_counts(celeste_plan* plan, const double* theta, int64_t* counts, hipStream_t stream);

/* Total ELBO of the field (each covered pixel counted once, minus every KL) into
 * out[0] (device). */
int celeste_total_elbo(celeste_plan* plan, const double* theta, double* out, hipStream_t stream);

/* How celeste_hessian, celeste_newton and celeste_sweep form the position and shape rows
 * of each box's Hessian in its intermediates (Section IV-D: exact Hessians).  mode 0 (the
 * default): one pass evaluating those second derivatives in closed form pixel by pixel;
 * mode 1: five tangent (dual-number) passes of the adjoint along the position and shape
 * intermediates.  Both give the same Hessian up to rounding.  CELESTE_EINVAL for another
 * mode.  Host call; affects later calls only. */
int celeste_plan_set_hessian_mode(celeste_plan* plan, int mode);

/* Greedy colouring of the box-overlap graph in a seeded random order: every batch is
 * a set of sources no two of which share a pixel of any image (the conflict-free
 * schedule of Section IV-D).  Host call.  batch_ptr (host [n_src + 1]) and
 * batch_src (host [n_src]) receive the CSR schedule, *n_batches its length. */
int celeste_color_batches(const celeste_plan* plan, uint64_t seed, int32_t* batch_ptr,
                          int32_t* batch_src, int32_t* n_batches);

/* Conflict graph of Section IV-D: sources s != t are adjacent when a patch box of s and
 * a patch box of t lie on the same image and share a pixel.  Host call.  adj_ptr (host
 * [n_src + 1]) and adj (host [cap]) receive it as CSR, each row sorted ascending without
 * repeats; *n_adj (host) receives the number of entries (twice the edge count).  If cap
 * is smaller than that, nothing is written but *n_adj and the call returns
 * CELESTE_EINVAL, so a first call with cap = 0 sizes the buffer. */
int celeste_conflict_graph(const celeste_plan* plan, int32_t* adj_ptr, int32_t* adj, int64_t cap,
                           int64_t* n_adj);

/* Cyclades schedule (Section IV-D, after Pan et al. 2016) as conflict-free batches for
 * celeste_sweep.  Pure host code: needs no plan and no GPU.
 *   n, adj_ptr [n + 1], adj: an undirected conflict graph as CSR (host; each edge in
 *     both rows; repeats allowed).
 *   order [n] (host): a permutation of 0..n-1, the random sampling order drawn by the
 *     caller.  It is cut into consecutive samples of sample_size sources (the last one
 *     shorter); every source is sampled once (without replacement).
 *   Within a sample, the conflict graph restricted to the sample splits into connected
 *   components.  Components run side by side; the members of one component run one
 *   after another in sample order.  Batch r of a sample (a "round") holds the r-th member
 *   of every component that has more than r members, listed in sample order, so a
 *   sample of largest component size R yields R batches, and the batches of a sample
 *   precede those of the next.  No two members of a batch are adjacent, and the result
 *   of celeste_sweep over one epoch equals serial block coordinate ascent in `order`.
 *   batch_ptr (host [n + 1]) and batch_src (host [n]) receive the CSR schedule,
 *   *n_batches its length, *n_components (host, or NULL) the number of components
 *   summed over samples.
 * CELESTE_EINVAL for n < 0, sample_size < 1, a row pointer that is not non-decreasing
 * from 0, a neighbour outside 0..n-1, or an order that is not a permutation (outputs
 * untouched). */
int celeste_cyclades_batches(int32_t n, const int32_t* adj_ptr, const int32_t* adj,
                             const int32_t* order, int32_t sample_size, int32_t* batch_ptr,
                             int32_t* batch_src, int32_t* n_batches, int32_t* n_components);

/* Block coordinate ascent (Section IV-D: each source's parameters form a block, optimised
 * by Newton's method with the overlapping sources held fixed; conflict-free batches of
 * sources run together): n_sweeps passes over the batches (host CSR batch_ptr,
 * batch_src), each batch optimised by params->newton_steps Newton trust-region
 * iterations with all other sources fixed.  Batches must be conflict-free
 * (CELESTE_ECONFLICT otherwise, nothing run).  elbo_trace (device [n_sweeps + 1])
 * receives the total ELBO before the first sweep and after each sweep.  Every batch's
 * lists go up once per call, stream-ordered as in celeste_hessian; when a schedule lists
 * sources more often than the plan's list buffers hold (each source once), the call waits
 * for `stream` and grows them (device allocation, kept by the plan).  No host
 * synchronisation between batches or sweeps.  With celeste_plan_use_graph enabled, one
 * sweep is captured into a HIP graph per call and replayed n_sweeps times (the same
 * kernels in the same order: the same results). */
int celeste_sweep(celeste_plan* plan, double* theta_inout, const int32_t* batch_ptr,
                  const int32_t* batch_src, int n_batches, int n_sweeps,
                  const celeste_tr_params* params, double* elbo_trace, hipStream_t stream);

/* Launch configuration: strips per work item (multiple of 64, at most 1024), waves per
 * block (1, 2 or 4), grid size of the grid-stride launches (blocks; 0 = 64 per compute
 * unit), dynamic_queue (0/1), render tile tile_h x tile_w (tile_w divides 64; tile_h * tile_w = 64, 128 or 256),
 * strip_rows (4, 8 or 16 pixels per strip) and render_mode (see celeste_plan_info).  A new
 * plan starts at chunk 64, 4 waves per block, grid 0, static queue, 16 x 16 tiles, 16-row
 * strips, render mode 2.  Rebuilds work items and render tiles (synchronous).  If grown
 * tile buffers cannot be allocated it returns CELESTE_ENOMEM and the plan keeps its
 * previous configuration. */
int celeste_plan_set_launch(celeste_plan* plan, int chunk, int waves_per_block, int grid_blocks,
                            int dynamic_queue, int tile_h, int tile_w, int strip_rows, int render_mode);

/* Times candidate launch configurations of celeste_elbo_grad (batched) on theta with
 * HIP events (median of `reps` runs each) and keeps the fastest (a candidate replaces the
 * current choice only when at least 1% faster).  Synchronous.
 * best_ms (host, or NULL) receives its time. */
int celeste_autotune(celeste_plan* plan, const double* theta, int reps, double* best_ms,
                     hipStream_t stream);

/* Capture the batched celeste_elbo_grad sequence for these exact pointers in a HIP
 * graph on first use and replay it afterwards, and run celeste_sweep's sweeps as replays
 * of a captured sweep (0 = off, the default). */
int celeste_plan_use_graph(celeste_plan* plan, int enable);

/* Per-phase device time of the batched evaluation (celeste_elbo / celeste_elbo_grad,
 * batched, outside a graph), measured with HIP events on the caller's stream while
 * enabled; each instrumented call then synchronises its stream.  ms (host [4], or
 * NULL) receives the summed milliseconds of (tables, render, fused adjoint, finalize)
 * since the last reset and *calls their count; reset != 0 clears both afterwards. */
int celeste_plan_profile(celeste_plan* plan, int enable, double* ms, int64_t* calls, int reset);

/* Synchronises `stream` and returns the domain status of the last call on this plan
 * (CELESTE_OK or CELESTE_EDOMAIN), then clears it. */
int celeste_plan_status(celeste_plan* plan, hipStream_t stream);

/* HIP error string of the last CELESTE_EHIP on this thread. */
const char* celeste_last_hip_error(void);

/* Diagnostic: the elementary functions of the strip kernels applied elementwise to device
 * arrays of n, for comparison with a reference libm.  fn = CELESTE_FN_EXP: table-driven
 * exp (Tang's method: 256-entry 2^(j/256) table, |r| <= ln2/512, degree-4 polynomial),
 * x[i] <= 709 and not NaN; CELESTE_FN_LOG: table-driven log (Tang's method: 128 breakpoints
 * in [1/2, 1), degree-6 log1p), finite x[i] > 0; CELESTE_FN_RCP: 1/x by the hardware estimate
 * and two Newton steps, x[i] finite with a normal reciprocal.  Other fn: CELESTE_EINVAL. */
enum { CELESTE_FN_EXP = 0, CELESTE_FN_LOG = 1, CELESTE_FN_RCP = 2 };
int celeste_debug_math(int fn, const double* x, double* y, int n, hipStream_t stream);

/* Text of a status code (static storage). */
const char* celeste_status_string(int status);
/* CELESTE_ABI_VERSION of the library. */
int celeste_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CELESTE_H */
