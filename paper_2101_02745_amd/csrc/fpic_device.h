// Device helpers shared by the HIP kernels of libflavorpic: stage times,
// the commutator slope, the quadratic shape weights, slope storage and
// global-memory accessors.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fpic {

// Stage time t = n dt + c dt, each operation rounded once (the CPU
// reference forms it the same way).
__device__ __forceinline__ double stage_time(int64_t n, double dt, double c)
{
#pragma clang fp contract(off)
    const double tn = (double)n * dt;
    return tn + c * dt;
}

// Quadratic (triangular-shaped cloud) weights from the fraction phi of the
// way between the centres of cells L and L + 1: the nearest centre is
// L + up, xi = x - x_(L+up) in [-1/2, 1/2), and cells L + up - 1, L + up,
// L + up + 1 get (1/2 - xi)^2 / 2, 3/4 - xi^2, (1/2 + xi)^2 / 2 (each
// operation rounded once, as the CPU reference forms them).
struct Quad {
    int up;
    double w0, w1, w2;
};

__device__ __forceinline__ Quad quad_weights(double phi)
{
#pragma clang fp contract(off)
    Quad q;
    q.up = phi < 0.5 ? 0 : 1;
    const double xi = q.up ? phi - 1.0 : phi;
    q.w0 = 0.5 * ((0.5 - xi) * (0.5 - xi));
    q.w1 = 0.75 - xi * xi;
    q.w2 = 0.5 * ((0.5 + xi) * (0.5 + xi));
    return q;
}

// Component k of the source a particle deposits, N rho - Nbar conj(rhobar):
// rhobar enters conjugated, so its imaginary parts (components 4, 6, 8)
// add.  Written as one explicit fused multiply-add, so that every kernel
// that forms a source (a stage forming the next stage's, the deposit of a
// state handed over by the caller) rounds it the same way and a run resumed
// from a saved state continues bitwise; left to the compiler, which of the
// two products is fused can differ from one kernel to the next.
__device__ __forceinline__ double source_comp(int k, double wN, double y, double wNb, double yb)
{
    const double b = wNb * yb;
    return __builtin_fma(wN, y, (k == 4 || k == 6 || k == 8) ? b : -b);
}

// Shape-weighted sums of two and three values, w0 a + w1 b (+ w2 c), with
// the rounding fixed by explicit fused multiply-adds in the order written,
// for the same reason.
__device__ __forceinline__ double wsum2(double w0, double a, double w1, double b)
{
    return __builtin_fma(w1, b, w0 * a);
}

__device__ __forceinline__ double wsum3(double w0, double a, double w1, double b, double w2, double c)
{
    return __builtin_fma(w2, c, __builtin_fma(w1, b, w0 * a));
}

// k = -i [H, rho] for Hermitian H, rho given as 9 packed reals (diagonal,
// then Re/Im of the (0,1), (0,2), (1,2) entries).  With C = H rho:
// k_aa = 2 Im C_aa and k_ab = -i (C_ab - conj(C_ba)) for a < b.  The trace
// of a commutator vanishes: k_00 is formed as -(k_11 + k_22), which is what
// lets a stored slope drop it (NK).
__device__ __forceinline__ void commutator(const double h[9], const double r[9], double k[9])
{
    const double h0 = h[0], h1 = h[1], h2 = h[2];
    const double ar = h[3], ai = h[4], br = h[5], bi = h[6], cr = h[7], ci = h[8];
    const double p0 = r[0], p1 = r[1], p2 = r[2];
    const double xr = r[3], xi = r[4], yr = r[5], yi = r[6], zr = r[7], zi = r[8];

    k[1] = 2.0 * ((ar * xi - ai * xr) + (ci * zr - cr * zi));
    k[2] = 2.0 * ((br * yi - bi * yr) + (cr * zi - ci * zr));
    k[0] = -(k[1] + k[2]);

    // C01 = h0 x + a p1 + b z^*,  C10 = a^* p0 + h1 x^* + c y^*
    const double c01r = h0 * xr + ar * p1 + (br * zr + bi * zi);
    const double c01i = h0 * xi + ai * p1 + (bi * zr - br * zi);
    const double c10r = ar * p0 + h1 * xr + (cr * yr + ci * yi);
    const double c10i = -ai * p0 - h1 * xi + (ci * yr - cr * yi);
    k[3] = c01i + c10i;
    k[4] = c10r - c01r;

    // C02 = h0 y + a z + b p2,  C20 = b^* p0 + c^* x^* + h2 y^*
    const double c02r = h0 * yr + (ar * zr - ai * zi) + br * p2;
    const double c02i = h0 * yi + (ar * zi + ai * zr) + bi * p2;
    const double c20r = br * p0 + (cr * xr - ci * xi) + h2 * yr;
    const double c20i = -bi * p0 - (cr * xi + ci * xr) - h2 * yi;
    k[5] = c02i + c20i;
    k[6] = c20r - c02r;

    // C12 = a^* y + h1 z + c p2,  C21 = b^* x + c^* p1 + h2 z^*
    const double c12r = (ar * yr + ai * yi) + h1 * zr + cr * p2;
    const double c12i = (ar * yi - ai * yr) + h1 * zi + ci * p2;
    const double c21r = (br * xr + bi * xi) + cr * p1 + h2 * zr;
    const double c21i = (br * xi - bi * xr) - ci * p1 - h2 * zi;
    k[7] = c12i + c21i;
    k[8] = c21r - c12r;
}

// Global-memory accesses through explicit address-space-1 pointers (the
// descriptor's pointers are generic, which would otherwise give flat loads).
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double gld(const double *p) { return *(const gdouble *)p; }
__device__ __forceinline__ void gst(double *p, double v) { *(gdouble *)p = v; }
// Nontemporal forms (streaming cache policy) for data not re-read soon.
__device__ __forceinline__ double gld_nt(const double *p)
{
    return __builtin_nontemporal_load((const gdouble *)p);
}
__device__ __forceinline__ void gst_nt(double *p, double v) { __builtin_nontemporal_store(v, (gdouble *)p); }
// Read-only tables (direction components, weights), which no kernel writes
// while another reads them: read through the constant address space, so at
// a wave-uniform index they become scalar loads.  A flat load (generic
// pointer) would make the wave wait for every vector load and store it has
// in flight, e.g. the previous direction's stores.
typedef const __attribute__((address_space(4))) double cdouble;
__device__ __forceinline__ double tld(const double *p, int64_t i) { return ((const cdouble *)p)[i]; }
// Device-scope relaxed atomics on global memory through address-space-1
// pointers: global_atomic_* instructions (a generic pointer gives flat
// atomics, with the same full waits as flat loads).
typedef __attribute__((address_space(1))) int32_t gint;
__device__ __forceinline__ void gatomic_add(double *p, double v)
{
    __hip_atomic_fetch_add((gdouble *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t gatomic_add(int32_t *p, int32_t v)
{
    return __hip_atomic_fetch_add((gint *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Slopes in memory: NK reals per particle, component c of the packed 18 at
// slot c - 1 (c = 1..8) or c - 2 (c = 10..17); components 0 and 9 are the
// negated sums of the next two.
__device__ __forceinline__ int kslot(int c) { return c < 9 ? c - 1 : c - 2; }

template <bool NT = false>
__device__ __forceinline__ void load_slope(const double *K, int64_t np, int64_t p, double k[18])
{
#pragma unroll
    for (int c = 1; c < 18; c++)
        if (c != 9)
            k[c] = NT ? gld_nt(K + kslot(c) * np + p) : gld(K + kslot(c) * np + p);
    k[0] = -(k[1] + k[2]);
    k[9] = -(k[10] + k[11]);
}

template <bool NT = false>
__device__ __forceinline__ void store_slope(double *K, int64_t np, int64_t p, const double k[18])
{
#pragma unroll
    for (int c = 1; c < 18; c++)
        if (c != 9) {
            if (NT)
                gst_nt(K + kslot(c) * np + p, k[c]);
            else
                gst(K + kslot(c) * np + p, k[c]);
        }
}

}  // namespace fpic
