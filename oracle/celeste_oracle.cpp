// Celeste ELBO oracle: a plain, slow FP64 CPU implementation of the per-source
// variational lower bound and its derivatives.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do.  It shares no code, header or table generator with the HIP library.
//
// What it computes (Regier et al. 2018, Section III and Eq. (1)): pixel counts are
// Poisson with a rate that is the sky level plus the calibrated light of every
// source covering the pixel; the variational family makes the expectation of the
// log-likelihood analytic up to a second-order (delta-method) expansion of
// E[log F].  Everything the paper leaves to the cited model is taken from an
// explicit, listed reading (the model constants below, the parameter layout, the
// mixture tables passed in as inputs).  An image's metadata (its sky location and
// observing conditions, Section III) is read as: a sky level per pixel (a constant or a
// map), a calibration factor, a PSF mixture in the image frame, and a local linear
// astrometry (origin and 2x2 matrix) from world to image coordinates.
//
// Structure: every pixel quantity is written once, as a template on the scalar
// type.  T = double gives values; T = Dual<double,N> (forward-mode AD over the N
// parameters of one source: 27, or 43 with the colour-prior mixture) gives the exact
// gradient; T = Dual<Dual<double,N>,1> (forward over forward) gives a Hessian-vector
// product.  No derivative is derived
// by hand here.  Loops are the naive definition: for a pixel, every other source
// whose box in that image contains the pixel is evaluated from scratch.  Sums over
// pixels use Neumaier compensation.  Build with -O2 -ffp-contract=off, no fast-math.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace oracle {

// plain double math visible to unqualified calls inside the templates
inline double exp(double x) { return std::exp(x); }
inline double log(double x) { return std::log(x); }
inline double sqrt(double x) { return std::sqrt(x); }
inline double sin(double x) { return std::sin(x); }
inline double cos(double x) { return std::cos(x); }

// ---------------------------------------------------------------- dual numbers
template <class T, int N>
struct Dual {
    T v;
    T d[N];
    Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
    Dual(double c) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
};

template <class T, int N>
Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
    Dual<T, N> r; r.v = a.v + b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
    Dual<T, N> r; r.v = a.v - b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a) {
    Dual<T, N> r; r.v = -a.v;
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
    Dual<T, N> r; r.v = a.v * b.v;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
    Dual<T, N> r; r.v = a.v / b.v;
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, double b) { return a + Dual<T, N>(b); }
template <class T, int N> Dual<T, N> operator+(double a, const Dual<T, N>& b) { return Dual<T, N>(a) + b; }
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, double b) { return a - Dual<T, N>(b); }
template <class T, int N> Dual<T, N> operator-(double a, const Dual<T, N>& b) { return Dual<T, N>(a) - b; }
template <class T, int N>
Dual<T, N> operator*(const Dual<T, N>& a, double b) {
    Dual<T, N> r; r.v = a.v * b;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <class T, int N> Dual<T, N> operator*(double a, const Dual<T, N>& b) { return b * a; }
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, double b) { return a / Dual<T, N>(b); }
template <class T, int N> Dual<T, N> operator/(double a, const Dual<T, N>& b) { return Dual<T, N>(a) / b; }

template <class T, int N>
Dual<T, N> exp(const Dual<T, N>& a) {
    using std::exp;
    Dual<T, N> r; r.v = exp(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = r.v * a.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> log(const Dual<T, N>& a) {
    using std::log;
    Dual<T, N> r; r.v = log(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / a.v;
    return r;
}
template <class T, int N>
Dual<T, N> sqrt(const Dual<T, N>& a) {
    using std::sqrt;
    Dual<T, N> r; r.v = sqrt(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
    return r;
}
template <class T, int N>
Dual<T, N> sin(const Dual<T, N>& a) {
    using std::sin; using std::cos;
    Dual<T, N> r; r.v = sin(a.v);
    T c = cos(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = c * a.d[i];
    return r;
}
template <class T, int N>
Dual<T, N> cos(const Dual<T, N>& a) {
    using std::sin; using std::cos;
    Dual<T, N> r; r.v = cos(a.v);
    T s = sin(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -(s * a.d[i]);
    return r;
}

// flattening to doubles (for compensated accumulation of every component)
inline int flat_size(const double*) { return 1; }
template <class T, int N> int flat_size(const Dual<T, N>*) { return (N + 1) * flat_size((const T*)nullptr); }
inline void flatten(const double& x, double* out) { out[0] = x; }
template <class T, int N>
void flatten(const Dual<T, N>& x, double* out) {
    const int k = flat_size((const T*)nullptr);
    flatten(x.v, out);
    for (int i = 0; i < N; ++i) flatten(x.d[i], out + (i + 1) * k);
}

// Neumaier-compensated running sums of a vector of doubles, plus sums of |terms|.
struct Acc {
    std::vector<double> s, c, a;
    explicit Acc(int n) : s(n, 0.0), c(n, 0.0), a(n, 0.0) {}
    void add(const double* x) {
        for (size_t i = 0; i < s.size(); ++i) {
            double t = s[i] + x[i];
            if (std::fabs(s[i]) >= std::fabs(x[i])) c[i] += (s[i] - t) + x[i];
            else c[i] += (x[i] - t) + s[i];
            s[i] = t;
            a[i] += std::fabs(x[i]);
        }
    }
    double get(int i) const { return s[i] + c[i]; }
};

// ---------------------------------------------------------------- problem input
struct OImage {
    int32_t band, H, W, pad;
    int64_t off;                 // offset of the image in x
    double sky, iota, ox, oy;    // sky level, calibration, world (x, y) of pixel (0, 0)
    double psf[3][6];            // (w, xi_x, xi_y, S_xx, S_xy, S_yy) per PSF component
    const double* sky_map;       // sky level of every pixel [H][W], or null: `sky` everywhere
    double wcs[2][2];            // image-frame offset = wcs * (world offset from the origin)
};

// Sky level of pixel (r, c) of an image: the per-pixel map when the image has one.
inline double sky_at(const OImage& im, int r, int c) {
    return im.sky_map ? im.sky_map[(int64_t)r * im.W + c] : im.sky;
}
struct OBox { int32_t img, r0, c0, h, w; };
const int ROW = 48;              // theta row: 27 model parameters, 16 mixture responsibilities, padding
const int NMIX = 8;              // components of each type's colour-prior mixture
struct OProblem {
    int32_t n_img, n_src;
    const OImage* img;
    const double* x;             // pixel counts; NaN marks a masked pixel
    const int32_t* patch_ptr;    // [n_src + 1]
    const OBox* box;
    const double* theta;         // [n_src][32]
    double exp_alpha[6], exp_nu[6], dev_alpha[8], dev_nu[8];
    double prior_phi;            // prior probability of a star
    double prior_r[2][2];        // [type][mean, var] of log reference-band brightness
    double prior_c[2][2][4];     // [type][mean, var][colour]
    int32_t flags, pad;
    // colour prior as a Gaussian mixture per type (with FLAG_MIX): weights, means and
    // full covariances of its NMIX components
    double mix_w[2][NMIX], mix_mean[2][NMIX][4], mix_cov[2][NMIX][4][4];
};
enum { FLAG_KL = 1, FLAG_LGAMMA = 2, FLAG_MIX = 4 };

const double PI = 3.14159265358979323846;

// Colour c_k = log(flux_{k+1} / flux_k) over bands u,g,r,i,z; reference band r.
// log flux_b = log r + sum_k BSIGN[b][k] c_k.
const int BSIGN[5][4] = {{-1, -1, 0, 0}, {0, -1, 0, 0}, {0, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 1, 1}};

template <class T>
struct Src {
    T ux, uy, fdev, rho, phi, re, q;
    T rmu[2], rvar[2], cmu[2][4], cvar[2][4];   // type 0 star, 1 galaxy
    T kap[2][NMIX];   // responsibilities of the colour-prior mixture components (row 27..42)
};

template <class T>
Src<T> load_src(const T* p) {
    Src<T> s;
    s.ux = p[0]; s.uy = p[1]; s.fdev = p[2]; s.rho = p[3]; s.phi = p[4]; s.re = p[5]; s.q = p[6];
    for (int a = 0; a < 2; ++a) {
        const T* b = p + 7 + 10 * a;
        s.rmu[a] = b[0]; s.rvar[a] = b[1];
        for (int k = 0; k < 4; ++k) { s.cmu[a][k] = b[2 + k]; s.cvar[a][k] = b[6 + k]; }
        for (int d = 0; d < NMIX; ++d) s.kap[a][d] = p[27 + NMIX * a + d];
    }
    return s;
}

// log flux_b | type a ~ N(m, v); returns E[flux] and E[flux^2] (log-normal moments).
template <class T>
void flux_moments(const Src<T>& s, int a, int b, T& m1, T& m2) {
    T m = s.rmu[a];
    T v = s.rvar[a];
    for (int k = 0; k < 4; ++k) {
        const double sg = BSIGN[b][k];
        m = m + sg * s.cmu[a][k];
        v = v + (sg * sg) * s.cvar[a][k];
    }
    m1 = exp(m + 0.5 * v);
    m2 = exp(2.0 * m + 2.0 * v);
}

// Galaxy shape covariance: radius^2 R(angle) diag(1, ratio^2) R(angle)^T.
template <class T>
void galaxy_cov(const Src<T>& s, T& sxx, T& sxy, T& syy) {
    T c = cos(s.phi), sn = sin(s.phi);
    T r2 = s.re * s.re, p2 = s.rho * s.rho;
    sxx = r2 * (c * c + p2 * sn * sn);
    sxy = r2 * (c * sn - p2 * c * sn);
    syy = r2 * (sn * sn + p2 * c * c);
}

// Bivariate normal density at (px, py).
template <class T>
T normal2(double px, double py, const T& mx, const T& my, const T& sxx, const T& sxy, const T& syy) {
    T det = sxx * syy - sxy * sxy;
    T dx = px - mx, dy = py - my;
    T quad = (syy * dx * dx - 2.0 * sxy * dx * dy + sxx * dy * dy) / det;
    return exp(-0.5 * quad) / (2.0 * PI * sqrt(det));
}

// PSF-convolved star and galaxy profiles of a source at the centre of pixel
// (row, col) of image im: pixel centre is (x = col, y = row) in the image frame.  A
// world point u maps to the image frame as wcs (u - origin), the image's local linear
// astrometry, so a world-frame galaxy covariance S appears as wcs S wcs^T; the PSF is
// given in the image frame.
template <class T>
void profiles(const OProblem& P, const OImage& im, const Src<T>& s, double px, double py,
              T& fstar, T& fgal) {
    const double(&A)[2][2] = im.wcs;
    T wx = s.ux - im.ox, wy = s.uy - im.oy;
    T mx0 = A[0][0] * wx + A[0][1] * wy, my0 = A[1][0] * wx + A[1][1] * wy;
    T wxx, wxy, wyy;
    galaxy_cov(s, wxx, wxy, wyy);
    // wcs S wcs^T
    T sxx = (A[0][0] * A[0][0]) * wxx + (2.0 * A[0][0] * A[0][1]) * wxy + (A[0][1] * A[0][1]) * wyy;
    T sxy = (A[0][0] * A[1][0]) * wxx + (A[0][0] * A[1][1] + A[0][1] * A[1][0]) * wxy +
            (A[0][1] * A[1][1]) * wyy;
    T syy = (A[1][0] * A[1][0]) * wxx + (2.0 * A[1][0] * A[1][1]) * wxy + (A[1][1] * A[1][1]) * wyy;
    fstar = T(0.0);
    T fdev(0.0), fexp(0.0);
    for (int k = 0; k < 3; ++k) {
        const double* ps = im.psf[k];
        T mx = mx0 + ps[1], my = my0 + ps[2];
        fstar = fstar + ps[0] * normal2(px, py, mx, my, T(ps[3]), T(ps[4]), T(ps[5]));
        for (int j = 0; j < 8; ++j) {
            const double nu = P.dev_nu[j];
            fdev = fdev + (ps[0] * P.dev_alpha[j]) *
                   normal2(px, py, mx, my, nu * sxx + ps[3], nu * sxy + ps[4], nu * syy + ps[5]);
        }
        for (int j = 0; j < 6; ++j) {
            const double nu = P.exp_nu[j];
            fexp = fexp + (ps[0] * P.exp_alpha[j]) *
                   normal2(px, py, mx, my, nu * sxx + ps[3], nu * sxy + ps[4], nu * syy + ps[5]);
        }
    }
    fgal = s.fdev * fdev + (1.0 - s.fdev) * fexp;
}

// Mean and variance of one source's light in a pixel under q: the source is a star
// with probability q, its band flux is log-normal given the type.
template <class T>
void source_moments(const OProblem& P, const OImage& im, const Src<T>& s, double px, double py,
                    T& Es, T& Vs) {
    T fstar, fgal;
    profiles(P, im, s, px, py, fstar, fgal);
    T m1s, m2s, m1g, m2g;
    flux_moments(s, 0, im.band, m1s, m2s);
    flux_moments(s, 1, im.band, m1g, m2g);
    Es = im.iota * (s.q * m1s * fstar + (1.0 - s.q) * m1g * fgal);
    Vs = (im.iota * im.iota) * (s.q * m2s * fstar * fstar + (1.0 - s.q) * m2g * fgal * fgal) - Es * Es;
}

// Delta-method expected Poisson log-likelihood of count x given E[F] and Var[F].
template <class T>
T pixel_term(double x, const T& E, const T& V, int flags) {
    T l = x * (log(E) - V / (2.0 * E * E)) - E;
    if (flags & FLAG_LGAMMA) l = l - std::lgamma(x + 1.0);
    return l;
}

inline bool box_has(const OBox& b, int r, int c) {
    return r >= b.r0 && r < b.r0 + b.h && c >= b.c0 && c < b.c0 + b.w;
}

// Sky plus the light of every source other than `skip` whose box in image n covers
// (r, c); `skip` = -1 includes all sources.
void background(const OProblem& P, int n, int r, int c, int skip, double& E, double& V) {
    const OImage& im = P.img[n];
    E = sky_at(im, r, c);
    V = 0.0;
    for (int t = 0; t < P.n_src; ++t) {
        if (t == skip) continue;
        for (int b = P.patch_ptr[t]; b < P.patch_ptr[t + 1]; ++b) {
            if (P.box[b].img != n || !box_has(P.box[b], r, c)) continue;
            Src<double> st = load_src(P.theta + ROW * (size_t)t);
            double Et, Vt;
            source_moments(P, im, st, (double)c, (double)r, Et, Vt);
            E += Et;
            V += Vt;
            break;
        }
    }
}

template <class T>
T kl_normal(const T& m1, const T& v1, double m2, double v2) {
    T dm = m1 - m2;
    return 0.5 * (std::log(v2) - log(v1) + (v1 + dm * dm) / v2 - 1.0);
}

// Inverse and log-determinant of a symmetric positive definite 4 x 4 matrix by its
// Cholesky factor (prior constants only, plain double).
void spd4_inverse(const double (&S)[4][4], double (&Pinv)[4][4], double& logdet) {
    double L[4][4] = {};
    logdet = 0.0;
    for (int j = 0; j < 4; ++j) {
        double d = S[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        L[j][j] = std::sqrt(d);
        logdet += 2.0 * std::log(L[j][j]);
        for (int i = j + 1; i < 4; ++i) {
            double v = S[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    // columns of S^-1 from L L^T x = e_c
    for (int c = 0; c < 4; ++c) {
        double y[4], x[4];
        for (int i = 0; i < 4; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
            y[i] = v / L[i][i];
        }
        for (int i = 3; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 4; ++k) v -= L[k][i] * x[k];
            x[i] = v / L[i][i];
        }
        for (int i = 0; i < 4; ++i) Pinv[i][c] = x[i];
    }
}

// KL(N(m, diag v) || N(mu, S)) in 4 dimensions:
// (tr(S^-1 diag v) + (m - mu)^T S^-1 (m - mu) - 4 + log det S - sum log v) / 2.
template <class T>
T kl_diag_full(const T* m, const T* v, const double* mu, const double (&S)[4][4]) {
    double Pm[4][4], logdet;
    spd4_inverse(S, Pm, logdet);
    T d[4];
    for (int k = 0; k < 4; ++k) d[k] = m[k] - mu[k];
    T acc = T(logdet - 4.0);
    for (int k = 0; k < 4; ++k) {
        acc = acc + Pm[k][k] * v[k] - log(v[k]);
        for (int l = 0; l < 4; ++l) acc = acc + Pm[k][l] * (d[k] * d[l]);
    }
    return 0.5 * acc;
}

// KL(q(a, r, c) || prior): Bernoulli on the type plus, per type weighted by its
// probability, the Gaussian KL of log brightness and that of the colours.  With the
// colour-prior mixture (FLAG_MIX) the colours' prior is sum_d w_d N(mu_d, S_d); the
// variational family adds the component indicator z ~ Cat(kappa) per type, independent of
// the colours, and the colour term becomes KL(q(c, z) || p(c, z)) =
// KL(Cat(kappa) || Cat(w)) + sum_d kappa_d KL(N(c_mu, diag c_var) || N(mu_d, S_d)).
template <class T>
T kl_source(const OProblem& P, const Src<T>& s) {
    const double phi = P.prior_phi;
    T q = s.q;
    T kl = q * log(q / phi) + (1.0 - q) * log((1.0 - q) / (1.0 - phi));
    for (int a = 0; a < 2; ++a) {
        T k = kl_normal(s.rmu[a], s.rvar[a], P.prior_r[a][0], P.prior_r[a][1]);
        if (P.flags & FLAG_MIX) {
            for (int d = 0; d < NMIX; ++d) {
                const T kd = s.kap[a][d];
                k = k + kd * (log(kd / P.mix_w[a][d]) +
                              kl_diag_full(s.cmu[a], s.cvar[a], P.mix_mean[a][d], P.mix_cov[a][d]));
            }
        } else {
            for (int j = 0; j < 4; ++j)
                k = k + kl_normal(s.cmu[a][j], s.cvar[a][j], P.prior_c[a][0][j], P.prior_c[a][1][j]);
        }
        kl = kl + (a == 0 ? q : 1.0 - q) * k;
    }
    return kl;
}

// Per-source ELBO: sum of pixel terms over the source's own boxes (other sources
// fixed), minus its KL.  Returns value/derivatives through a flattened accumulator.
template <class T>
void source_elbo(const OProblem& P, int s, const T* p27, Acc& acc, Acc& kl_acc) {
    const int K = flat_size((const T*)nullptr);
    std::vector<double> buf(K);
    Src<T> own = load_src(p27);
    for (int b = P.patch_ptr[s]; b < P.patch_ptr[s + 1]; ++b) {
        const OBox& bx = P.box[b];
        const OImage& im = P.img[bx.img];
        for (int r = bx.r0; r < bx.r0 + bx.h; ++r) {
            for (int c = bx.c0; c < bx.c0 + bx.w; ++c) {
                const double x = P.x[im.off + (int64_t)r * im.W + c];
                if (std::isnan(x)) continue;
                double Eb, Vb;
                background(P, bx.img, r, c, s, Eb, Vb);
                T Es, Vs;
                source_moments(P, im, own, (double)c, (double)r, Es, Vs);
                T l = pixel_term(x, Es + Eb, Vs + Vb, P.flags);
                flatten(l, buf.data());
                acc.add(buf.data());
            }
        }
    }
    if (P.flags & FLAG_KL) {
        T kl = kl_source(P, own);
        flatten(-kl, buf.data());
        kl_acc.add(buf.data());
    }
}

}  // namespace oracle

using namespace oracle;

// Number of parameters a source's ELBO depends on: 27, or 43 with the colour-prior mixture
// (the 16 responsibilities enter the KL only).
inline int n_params(const OProblem* P) { return (P->flags & FLAG_MIX) ? 43 : 27; }

template <int N>
void source_grad_n(const OProblem* P, int s, double* val, double* grad, double* gabs) {
    typedef Dual<double, N> D;
    D p[ROW];
    const double* th = P->theta + ROW * (size_t)s;
    for (int i = 0; i < ROW; ++i) {
        p[i] = D(th[i]);
        if (i < N) p[i].d[i] = 1.0;
    }
    Acc acc(N + 1), kl(N + 1);
    source_elbo<D>(*P, s, p, acc, kl);
    val[0] = acc.get(0);
    val[1] = kl.get(0);
    val[2] = acc.a[0];
    for (int i = 0; i < N; ++i) {
        grad[i] = acc.get(1 + i) + kl.get(1 + i);
        gabs[i] = acc.a[1 + i] + kl.a[1 + i];
    }
}

template <int N>
void source_hvp_n(const OProblem* P, int s, const double* v, double* hv, double* habs) {
    typedef Dual<double, N> D;
    typedef Dual<D, 1> DD;
    DD p[ROW];
    const double* th = P->theta + ROW * (size_t)s;
    for (int i = 0; i < ROW; ++i) {
        p[i] = DD(th[i]);
        if (i < N) {
            p[i].v.d[i] = 1.0;
            p[i].d[0] = D(v[i]);
        }
    }
    Acc acc(2 * (N + 1)), kl(2 * (N + 1));
    source_elbo<DD>(*P, s, p, acc, kl);
    // layout: [v.v, v.d[0..N-1], d0.v, d0.d[0..N-1]]
    for (int i = 0; i < N; ++i) {
        hv[i] = acc.get(N + 1 + 1 + i) + kl.get(N + 1 + 1 + i);
        habs[i] = acc.a[N + 1 + 1 + i] + kl.a[N + 1 + 1 + i];
    }
}


extern "C" {

int oracle_version() { return 1; }
int oracle_sizeof_image() { return (int)sizeof(OImage); }
int oracle_sizeof_problem() { return (int)sizeof(OProblem); }

// Per-source ELBO value.  out[0] = pixel sum, out[1] = -KL (0 without the KL flag),
// out[2] = sum over visits of |pixel term|.
int oracle_source_value(const OProblem* P, int s, double* out) {
    Acc acc(1), kl(1);
    source_elbo<double>(*P, s, P->theta + ROW * (size_t)s, acc, kl);
    out[0] = acc.get(0);
    out[1] = kl.get(0);
    out[2] = acc.a[0];
    return 0;
}

int oracle_n_params(const OProblem* P) { return n_params(P); }

// Per-source ELBO gradient w.r.t. its own parameters (forward-mode duals).
// val[0..2] as oracle_source_value; grad[n] = d(pixel sum - KL)/d theta_s;
// gabs[n] = sum over visits of |d pixel term / d theta_s| (plus |d KL|); n = n_params.
int oracle_source_grad(const OProblem* P, int s, double* val, double* grad, double* gabs) {
    if (n_params(P) == 43) source_grad_n<43>(P, s, val, grad, gabs);
    else source_grad_n<27>(P, s, val, grad, gabs);
    return 0;
}

// Hessian-vector product of the per-source ELBO in direction v (forward over forward).
// hv[n] = H v, habs[n] = sum over visits of |(H_visit v)_i| (plus the KL term's).
int oracle_source_hvp(const OProblem* P, int s, const double* v, double* hv, double* habs) {
    if (n_params(P) == 43) source_hvp_n<43>(P, s, v, hv, habs);
    else source_hvp_n<27>(P, s, v, hv, habs);
    return 0;
}

// Dense Hessian of the per-source ELBO: column d is the Hessian-vector product along the
// unit vector e_d (the n columns run in parallel, OpenMP); habs[i][d] is that product's
// sum of |per-visit terms| for entry i.  Row-major n x n H[i][d] and habs[i][d].
int oracle_source_hessian(const OProblem* P, int s, double* H, double* habs) {
    const int n = n_params(P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < n; ++d) {
        double e[43], hv[43], ha[43];
        for (int i = 0; i < n; ++i) e[i] = (i == d) ? 1.0 : 0.0;
        oracle_source_hvp(P, s, e, hv, ha);
        for (int i = 0; i < n; ++i) {
            H[i * n + d] = hv[i];
            habs[i * n + d] = ha[i];
        }
    }
    return 0;
}

// E[F] and Var[F] at every pixel of image n (sky + all covering sources).
int oracle_render(const OProblem* P, int n, double* E, double* V) {
    const OImage& im = P->img[n];
    for (int r = 0; r < im.H; ++r)
        for (int c = 0; c < im.W; ++c)
            background(*P, n, r, c, -1, E[(int64_t)r * im.W + c], V[(int64_t)r * im.W + c]);
    return 0;
}

// One source's own E_s and Var_s at every pixel of image n, ignoring boxes
// (used by the mass and symmetry checks).
int oracle_source_light(const OProblem* P, int s, int n, double* E, double* V) {
    const OImage& im = P->img[n];
    Src<double> st = load_src(P->theta + ROW * (size_t)s);
    for (int r = 0; r < im.H; ++r)
        for (int c = 0; c < im.W; ++c)
            source_moments(*P, im, st, (double)c, (double)r, E[(int64_t)r * im.W + c],
                           V[(int64_t)r * im.W + c]);
    return 0;
}

// Star and galaxy profile of source s at image-frame point (px, py) of image n.
int oracle_profiles(const OProblem* P, int s, int n, double px, double py, double* out) {
    Src<double> st = load_src(P->theta + ROW * (size_t)s);
    profiles(*P, P->img[n], st, px, py, out[0], out[1]);
    return 0;
}

// E[flux] and E[flux^2] of source s for type a in band b.
int oracle_flux_moments(const OProblem* P, int s, int a, int b, double* out) {
    Src<double> st = load_src(P->theta + ROW * (size_t)s);
    flux_moments(st, a, b, out[0], out[1]);
    return 0;
}

double oracle_kl(const OProblem* P, int s) {
    Src<double> st = load_src(P->theta + ROW * (size_t)s);
    return kl_source(*P, st);
}

// Total ELBO: pixel terms over the union of all boxes (each pixel once) minus the
// sum of every source's KL.
double oracle_total_elbo(const OProblem* P) {
    Acc acc(1);
    for (int n = 0; n < P->n_img; ++n) {
        const OImage& im = P->img[n];
        std::vector<char> cov((size_t)im.H * im.W, 0);
        for (int b = 0; b < P->patch_ptr[P->n_src]; ++b) {
            const OBox& bx = P->box[b];
            if (bx.img != n) continue;
            for (int r = bx.r0; r < bx.r0 + bx.h; ++r)
                for (int c = bx.c0; c < bx.c0 + bx.w; ++c) cov[(size_t)r * im.W + c] = 1;
        }
        for (int r = 0; r < im.H; ++r)
            for (int c = 0; c < im.W; ++c) {
                if (!cov[(size_t)r * im.W + c]) continue;
                const double x = P->x[im.off + (int64_t)r * im.W + c];
                if (std::isnan(x)) continue;
                double E, V;
                background(*P, n, r, c, -1, E, V);
                double l = pixel_term(x, E, V, P->flags);
                acc.add(&l);
            }
    }
    double tot = acc.get(0);
    if (P->flags & FLAG_KL) {
        Acc k(1);
        for (int s = 0; s < P->n_src; ++s) {
            double v = -oracle_kl(P, s);
            k.add(&v);
        }
        tot += k.get(0);
    }
    return tot;
}

// Gradients of many sources (the CPU baseline): OpenMP over the listed sources.
int oracle_grad_many(const OProblem* P, int n, const int32_t* src, double* val3, double* grad) {
    const int np = n_params(P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        double gabs[43];
        oracle_source_grad(P, src[i], val3 + 3 * (size_t)i, grad + np * (size_t)i, gabs);
    }
    return 0;
}

}  // extern "C"
