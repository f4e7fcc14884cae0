// First-order dual number (value, tangent) for the forward-mode tangent of the
// hand-written adjoint: running the gradient code on `dual` inputs seeded with a
// direction v yields the gradient (value parts) and the Hessian-vector product
// (tangent parts) in one pass.
#pragma once
#include <hip/hip_runtime.h>

struct dual {
    double v, t;
};

__host__ __device__ inline dual mkd(double v, double t = 0.0) { dual r; r.v = v; r.t = t; return r; }

__host__ __device__ inline dual operator+(dual a, dual b) { return mkd(a.v + b.v, a.t + b.t); }
__host__ __device__ inline dual operator-(dual a, dual b) { return mkd(a.v - b.v, a.t - b.t); }
__host__ __device__ inline dual operator-(dual a) { return mkd(-a.v, -a.t); }
__host__ __device__ inline dual operator*(dual a, dual b) { return mkd(a.v * b.v, a.t * b.v + a.v * b.t); }
__host__ __device__ inline dual operator/(dual a, dual b) {
    const double q = a.v / b.v;
    return mkd(q, (a.t - q * b.t) / b.v);
}
__host__ __device__ inline dual operator+(dual a, double b) { return mkd(a.v + b, a.t); }
__host__ __device__ inline dual operator+(double a, dual b) { return mkd(a + b.v, b.t); }
__host__ __device__ inline dual operator-(dual a, double b) { return mkd(a.v - b, a.t); }
__host__ __device__ inline dual operator-(double a, dual b) { return mkd(a - b.v, -b.t); }
__host__ __device__ inline dual operator*(dual a, double b) { return mkd(a.v * b, a.t * b); }
__host__ __device__ inline dual operator*(double a, dual b) { return mkd(a * b.v, a * b.t); }
__host__ __device__ inline dual operator/(dual a, double b) { return mkd(a.v / b, a.t / b); }
__host__ __device__ inline dual operator/(double a, dual b) {
    const double q = a / b.v;
    return mkd(q, -q * b.t / b.v);
}
__host__ __device__ inline dual& operator+=(dual& a, dual b) { a = a + b; return a; }
__host__ __device__ inline dual& operator-=(dual& a, dual b) { a = a - b; return a; }

__device__ inline dual exp(dual a) { const double e = exp(a.v); return mkd(e, e * a.t); }
__device__ inline dual log(dual a) { return mkd(log(a.v), a.t / a.v); }
__device__ inline dual sqrt(dual a) { const double s = sqrt(a.v); return mkd(s, a.t / (2.0 * s)); }
__device__ inline dual sin(dual a) { return mkd(sin(a.v), cos(a.v) * a.t); }
__device__ inline dual cos(dual a) { return mkd(cos(a.v), -sin(a.v) * a.t); }

// Scalar traits used by the templated model code.
__host__ __device__ inline double value_of(double x) { return x; }
__host__ __device__ inline double value_of(dual x) { return x.v; }
__host__ __device__ inline double tangent_of(double) { return 0.0; }
__host__ __device__ inline double tangent_of(dual x) { return x.t; }

// A quantity whose value is `base` and whose tangent is that of `own` (used when a
// stored total already contains the source's own value but not its tangent).
__host__ __device__ inline double value_with_tangent(double base, double) { return base; }
__host__ __device__ inline dual value_with_tangent(double base, dual own) { return mkd(base, own.t); }

// Unroll factor of the loops over the 42 galaxy Gaussians.  Value arithmetic: two at a
// time, so that one component's table loads and seed overlap the other's rows (measured
// best of 1, 2, 3, 6).  Dual (value + tangent) arithmetic keeps one.  At two, the tangent
// products of the streamed passes (own values recomputed, planes or stored backgrounds)
// came out bitwise equal to those at one, but the pass that recomputes both the own values
// and the neighbours' background per strip (stored neighbour values, 16-row strips) returned
// tangents off by up to a factor of four in the position and shape directions while its
// values and gradients agreed to 1e-12; the source changes no index or lane assignment with
// this factor, and the cause in the generated code is not identified (its kernels spill a
// few hundred bytes per lane at either factor).
#ifndef CELESTE_GAL_UNROLL
#define CELESTE_GAL_UNROLL 2
#endif
#ifndef CELESTE_DUAL_GAL_UNROLL
#define CELESTE_DUAL_GAL_UNROLL 1
#endif

template <class T> struct scalar_traits;
template <> struct scalar_traits<double> {
    static constexpr int width = 1;
    static constexpr int gal_unroll = CELESTE_GAL_UNROLL;
    __host__ __device__ static double make(double v, double) { return v; }
};
template <> struct scalar_traits<dual> {
    static constexpr int width = 2;
    static constexpr int gal_unroll = CELESTE_DUAL_GAL_UNROLL;
    __host__ __device__ static dual make(double v, double t) { return mkd(v, t); }
};
