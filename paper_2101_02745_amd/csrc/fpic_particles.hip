// General particle placement (include/fpic_particles.h): particles anywhere
// in the periodic box, any number per cell, each with its own position at
// t = 0, direction and weights.
//
// Layout.  Structure of arrays in two sets A and B: the state Y[18][np],
// positions pos[3][np], directions v[3][np], weights wN = N/dV, wNb = Nbar/dV
// and the caller's index pid.  The particles are kept sorted by cell: a
// counting sort (count, scan, scatter) moves every particle from the current
// set to the other one every `sort_every` steps.  Slopes K1..K3 keep 16
// reals per particle (the traceless form of fpic_internal.h).
//
// One launch per Runge-Kutta stage; a workgroup takes 256 consecutive
// particles (one per thread).  Per particle the thread forms the stage
// state, interpolates the combined moments of the grid at its stage
// position (the 32 traceless components, see pstage_kernel; from an LDS
// copy of the workgroup's cells in stages 1-3, through the caches in
// stage 4), builds H and
// Hbar (eq. potentials, Sec. II.A conventions), the commutator slopes
// (eq. eom) and the next stage state, and deposits that state with the
// next-stage weights (eq. pic_deposition).  Because the particles are sorted
// by cell, a workgroup's particles cover a small box of cells: it
// accumulates their deposits in LDS over that box and adds the box into the
// grid with global atomics.  A workgroup whose box does not fit its LDS
// (particles spread out) adds straight to the grid.
//
// Deposits are summed exactly, in integers: each contribution v is scaled
// by 2^S (S fixed per box from the particle count and the largest weight,
// so that no contribution and no cell's sum can pass 2^81) and split into
// two 64-bit limbs,
// hi = floor(V / 2^32) and lo = V - 2^32 hi in [0, 2^32), V = rint(v 2^S).
// Integer atomics add the
// limbs; integer addition is associative, so the sums do not depend on the
// order in which the atomics land or on the order of the particles within
// a cell (the counting sort leaves that order to its atomics): every run
// is bitwise reproducible.  A finalize pass turns each limb pair into a
// double (one rounding of the exact sum of the scaled contributions, each
// of which is off by at most 2^-(S+1), i.e. 2^-84 of 16 np max_p (|N_p| +
// |Nbar_p|)/dV) and clears the limbs.  Stage s of step n reads G[(4n+s-1) % 3] and its
// finalize writes G[(4n+s) % 3].
//
// Positions: x(t) = x0 + Omega t per axis, u = x / dx - 1/2, first cell
// floor(u), fraction u - floor(u); every operation rounded once, the same
// formulas as the CPU reference.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fpic_device.h"
#include "fpic_internal.h"
#include "fpic_particles.h"

namespace fpicp {

using fpic::commutator;
using fpic::fail;
using fpic::gatomic_add;
using fpic::gld;
using fpic::gst;
using fpic::load_slope;
using fpic::Quad;
using fpic::quad_weights;
using fpic::source_comp;
using fpic::stage_time;
using fpic::store_slope;

constexpr int NG = 36;
constexpr int NXT = 8;   // traceless source components (stage grids: 4 NXT)
constexpr int BLK = 256;            // particles (threads) per workgroup
constexpr int NWAVE = BLK / 64;
// LDS of the deposit box accumulators: 48 KB with floating-point atomics
// (three workgroups per CU when the stage kernel needs at most 168 VGPRs),
// 64 KB for the exact sums, whose limbs take twice the room
template <bool EXACT>
constexpr int acc_words() { return EXACT ? 8192 : 6144; }
constexpr int MAX_COPIES = 32;      // replicas of the box accumulator
constexpr int kRedBlk = 256;        // blocks of the diagnostic reductions
// scratch (8-byte words): [0, 32) results, then the totals partials
// (36 limbs per block), the check partials (3 per block), the weight sums
constexpr int kScratch1 = 32, kScratch2 = kScratch1 + 36 * kRedBlk, kScratch3 = kScratch2 + 3 * kRedBlk;

enum : int { PM_DEPOSIT = 5, PM_MOM_NU = 6, PM_MOM_NUBAR = 7, PM_S4_SORT = 8 };

struct PDesc {
    int32_t n[3];
    int32_t shape;
    int64_t ncell, np;
    double dt, dx[3];
    double hvac[9];   // constant part of H: vacuum + matter, packed
    double hvacb[9];  // of Hbar before conjugation: vacuum - matter
    // current particle set
    double *pos, *v, *wN, *wNb;
    int32_t *pid;
    double *Y;
    // the set the next sort writes
    double *pos2, *v2, *wN2, *wNb2, *Y2;
    int32_t *pid2;
    double *K1, *K2, *K3;
    double *G0, *G1, *G2;
    int64_t *step;
    int32_t *cnt, *cur;  // [ncell] sort counters
    long long *GL;       // [2][NG][ncell] deposit limbs: hi plane, then lo plane
    double qs, qi;       // 2^S and 2^-S: the fixed-point scale of the deposits
};

// ---- exact deposit sums -------------------------------------------------
// v 2^S as the limb pair (hi, lo) with rint(v 2^S) = 2^32 hi + lo and
// 0 <= lo < 2^32.  Valid for |v 2^S| < 2^83 (the scale keeps contributions
// below 2^81), so that -2^51 <= hi < 2^51; both limbs are read off the bits of a double: an integer-valued
// double in [2^52, 2^53) holds its value minus 2^52 in its mantissa bits
// (no double-to-64-bit-integer conversion exists on this GPU).  Every step
// is exact.
__device__ __forceinline__ void to_limbs(double v, double qs, long long &hi, long long &lo)
{
#pragma clang fp contract(off)
    const double V = rint(v * qs);
    const double h = floor(V * 0x1p-32);
    const double r = fma(h, -0x1p32, V);  // integer in [0, 2^32), exact
    const double M = 0x1.8p52;            // h + M in [2^52, 2^53)
    hi = __double_as_longlong(h + M) - __double_as_longlong(M);
    lo = (long long)(unsigned)__double2loint(r + 0x1p52);
}

// the double nearest to 2^-S (2^32 a1 + a0) for limb sums a1, a0 (a0 >= 0)
__device__ __forceinline__ double from_limbs(long long a1, long long a0, double qi)
{
#pragma clang fp contract(off)
    const long long t = a1 + (a0 >> 32);               // |t| < 2^62
    const long long r0 = a0 & 0xffffffffLL;
    const double th = (double)t;                       // rounded when |t| > 2^53
    const long long e = t - (long long)th;             // exact, |e| <= 2^9
    const double low = (double)(e * 4294967296LL + r0);  // exact, < 2^42
    return fma(th, 0x1p32, low) * qi;                  // one rounding
}

typedef __attribute__((address_space(1))) long long glong;
__device__ __forceinline__ void gatomic_add_ll(long long *p, long long v)
{
    __hip_atomic_fetch_add((glong *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lds_add_limbs(long long *hi_p, long long *lo_p, double v, double qs)
{
    long long hi, lo;
    to_limbs(v, qs, hi, lo);
    atomicAdd(reinterpret_cast<unsigned long long *>(hi_p), (unsigned long long)hi);
    atomicAdd(reinterpret_cast<unsigned long long *>(lo_p), (unsigned long long)lo);
}

__device__ __forceinline__ void global_add_limbs(long long *GL, int64_t plane, int64_t q, double v,
                                                 double qs)
{
    long long hi, lo;
    to_limbs(v, qs, hi, lo);
    gatomic_add_ll(GL + q, hi);
    gatomic_add_ll(GL + plane + q, lo);
}

// Limb sums of one box entry (LDS offset q of each of the R copies, hi
// limbs, then lo limbs half further on) added to grid entry g.
__device__ __forceinline__ void flush_limbs(const long long *lacc, int R, int cstride, int half, int q,
                                            long long *GL, int64_t g, int64_t plane)
{
    long long hi = 0, lo = 0;
#pragma unroll 4
    for (int r = 0; r < R; r++) {
        hi += lacc[r * cstride + q];
        lo += lacc[r * cstride + half + q];
    }
    if (hi != 0)
        gatomic_add_ll(GL + g, hi);
    if (lo != 0)
        gatomic_add_ll(GL + plane + g, lo);
}

// n-periodic index of an integer-valued double (|i| < 2^52)
__device__ __forceinline__ int wrap_cell(double i, int n)
{
    const double nd = (double)n;
    double r = i - nd * floor(i / nd);
    if (r < 0.0)
        r += nd;
    if (r >= nd)
        r -= nd;
    return (int)r;
}

// Along one axis at time t: first cell of the shape function's stencil
// (periodic) and its weights; SH = 1: cells L, L + 1 with (1 - phi, phi);
// SH = 2: cells L + up - 1 .. L + up + 1 with the quadratic weights.  An
// axis with one cell keeps every particle in cell 0 with weight 1.
template <int SH>
__device__ __forceinline__ void axis_stencil(double x0, double v, double t, double dx, int n,
                                             int *first, double w[3])
{
#pragma clang fp contract(off)
    if (n == 1) {
        *first = 0;
        w[0] = 1.0;
        w[1] = 0.0;
        w[2] = 0.0;
        return;
    }
    const double x = x0 + v * t;
    const double u = x / dx - 0.5;
    const double fl = floor(u);
    const double phi = u - fl;
    if (SH == 2) {
        const Quad q = quad_weights(phi);
        *first = wrap_cell(fl + (double)(q.up - 1), n);
        w[0] = q.w0;
        w[1] = q.w1;
        w[2] = q.w2;
    } else {
        *first = wrap_cell(fl, n);
        w[0] = 1.0 - phi;
        w[1] = phi;
        w[2] = 0.0;
    }
}

// offset of cell c from the reference cell r on an n-periodic axis, in
// (-n/2, n/2]
__device__ __forceinline__ int periodic_offset(int c, int r, int n)
{
    int o = c - r;
    if (2 * o > n)
        o -= n;
    else if (2 * o <= -n)
        o += n;
    return o;
}

__device__ __forceinline__ int wrap_int(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

// w[b] for a run-time b in 0..2, without indexing a private array
__device__ __forceinline__ double pick(const double w[3], int b)
{
    return b == 0 ? w[0] : (b == 1 ? w[1] : w[2]);
}

// Box of cells covered by the stencils of a workgroup's active particles
// (first cells f, SW cells per axis), as offsets from thread 0's first cell
// on each periodic axis.  Every thread of the workgroup must call it.
struct Box {
    int ref[3], lo[3], s[3];
    int64_t cells;
};

template <int SW, bool D3>
__device__ __forceinline__ Box block_box(const int f[3], bool active, const int n[3],
                                         int (*sred)[6], int *sref, int o[3])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // earlier readers of sref, sred and the LDS box are done
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; a++)
            sref[a] = f[a];
    __syncthreads();
    Box b;
    int m[6];
    for (int a = 0; a < 3; a++) {
        b.ref[a] = sref[a];
        o[a] = periodic_offset(f[a], b.ref[a], n[a]);
        m[a] = active ? o[a] : INT_MAX;
        m[3 + a] = active ? o[a] : INT_MIN;
    }
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            m[a] = min(m[a], __shfl_xor(m[a], sh, 64));
            m[3 + a] = max(m[3 + a], __shfl_xor(m[3 + a], sh, 64));
        }
    if (lane == 0)
        for (int a = 0; a < 6; a++)
            sred[wave][a] = m[a];
    __syncthreads();
    for (int a = 0; a < 3; a++) {
        int lo = sred[0][a], hi = sred[0][3 + a];
        for (int w = 1; w < NWAVE; w++) {
            lo = min(lo, sred[w][a]);
            hi = max(hi, sred[w][3 + a]);
        }
        const bool used = D3 || a == 2;
        b.lo[a] = used ? lo : 0;
        b.s[a] = used ? hi - lo + SW : 1;
        if (!used)
            o[a] = 0;
    }
    b.cells = (int64_t)b.s[0] * b.s[1] * b.s[2];
    return b;
}

// ---- redistribution: counting sort by cell ----------------------------
// Sort key: the cell whose centre is the nearest one at or below the
// particle along each axis (the linear stencil's first cell) at the start
// of the current step; cells numbered x fastest.
__device__ __forceinline__ int sort_key(const PDesc &S, int64_t i, double t)
{
    double w[3];
    int cx = 0, cy = 0, cz;
    axis_stencil<1>(gld(S.pos + 2 * S.np + i), gld(S.v + 2 * S.np + i), t, S.dx[2], S.n[2], &cz, w);
    if (S.n[0] > 1 || S.n[1] > 1) {  // 3D boxes (1D boxes hold z positions only)
        axis_stencil<1>(gld(S.pos + i), gld(S.v + i), t, S.dx[0], S.n[0], &cx, w);
        axis_stencil<1>(gld(S.pos + S.np + i), gld(S.v + S.np + i), t, S.dx[1], S.n[1], &cy, w);
    }
    return (cz * S.n[1] + cy) * S.n[0] + cx;
}

// The keys of a workgroup's particles (nearly sorted) fall in a short range
// of the periodic cell numbering: a histogram of that range in LDS takes the
// per-particle atomics, and the workgroup adds one count per cell to the
// global counters.  A workgroup whose range exceeds HIST_MAX cells uses
// global atomics per particle.
constexpr int HIST_MAX = 8192;

struct KeyRange {
    int ref, lo, len, off;
};

__device__ __forceinline__ KeyRange key_range(int key, bool active, int nc, int (*sred)[2], int *sref)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        *sref = key;
    __syncthreads();
    KeyRange r;
    r.ref = *sref;
    r.off = periodic_offset(key, r.ref, nc);
    int lo = active ? r.off : INT_MAX, hi = active ? r.off : INT_MIN;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        lo = min(lo, __shfl_xor(lo, sh, 64));
        hi = max(hi, __shfl_xor(hi, sh, 64));
    }
    if (lane == 0) {
        sred[wave][0] = lo;
        sred[wave][1] = hi;
    }
    __syncthreads();
    lo = sred[0][0];
    hi = sred[0][1];
    for (int w = 1; w < NWAVE; w++) {
        lo = min(lo, sred[w][0]);
        hi = max(hi, sred[w][1]);
    }
    r.lo = lo;
    r.len = hi - lo + 1;
    return r;
}

// MODE 1..4: Runge-Kutta stages; PM_S4_SORT: stage 4 that also moves every
// particle to its place in the cell order of the next step (the counts and
// offsets come from sort_count_kernel and sort_scan_kernel beforehand), so a
// sort needs no pass of its own; PM_DEPOSIT: deposit the current state at
// the current time into the buffer stage 1 reads; PM_MOM_NU / PM_MOM_NUBAR:
// deposit N rho or Nbar rhobar alone into outG (moment diagnostics).
// EXACT: deposits summed exactly in the limbs (finalize_kernel then writes
// the grid); otherwise with floating-point atomics straight into the grid.
//
// Two waves per SIMD for every shape.  With the quadratic shape that costs
// registers (the 3D kernels spill 130-330 bytes per lane to scratch memory)
// but against one wave per SIMD it is still faster: exact sums on the random
// 2048-cell box 0.737 -> 0.613 ms per step, on the random 32^3 box 21.2 ->
// 14.6 ms.
template <int MODE, int SH, bool D3, bool EXACT>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2)))
pstage_kernel(const PDesc *__restrict__ dp, double *outG)
{
    constexpr int SW = SH + 1;  // stencil cells per axis
    constexpr bool RK = MODE <= 4 || MODE == PM_S4_SORT;
    // The stage grids hold traceless moments: the interpolated Hamiltonian
    // is needed only up to a multiple of the identity (it commutes with rho
    // and rhobar), so each source matrix is deposited as x11 - x00,
    // x22 - x00 and its six off-diagonal reals (NXT = 8), 32 components per
    // cell.  The moment diagnostics deposit all nine.
    constexpr bool FULL = MODE == PM_MOM_NU || MODE == PM_MOM_NUBAR;
    constexpr int NCS = FULL ? 9 : NXT, NGC = 4 * NCS;
    constexpr int STG = MODE == PM_S4_SORT ? 4 : MODE;  // Runge-Kutta stage
    constexpr int ACC_DOUBLES = acc_words<EXACT>();
    __shared__ double acc[ACC_DOUBLES];
    __shared__ int sred[NWAVE][6];
    __shared__ int sref[3];
    const PDesc S = *dp;
    const int64_t np = S.np;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const bool active = i < np;
    const int64_t ip = active ? i : 0;
    const int64_t n = *S.step;
    const double dt = S.dt;
    const int lane = threadIdx.x & 63;

    double t_cur = 0.0, t_nxt;
    if (MODE == 1) {
        t_cur = stage_time(n, dt, 0.0);
        t_nxt = stage_time(n, dt, 0.5);
    } else if (MODE == 2) {
        t_cur = stage_time(n, dt, 0.5);
        t_nxt = stage_time(n, dt, 0.5);
    } else if (MODE == 3) {
        t_cur = stage_time(n, dt, 0.5);
        t_nxt = stage_time(n, dt, 1.0);
    } else if (STG == 4) {
        t_cur = stage_time(n, dt, 1.0);
        t_nxt = stage_time(n + 1, dt, 0.0);
    } else {
        t_nxt = stage_time(n, dt, 0.0);
    }

    // grid buffers (selects, no indexing into the descriptor copy): the one
    // this stage interpolates from; exact sums deposit into the limbs S.GL,
    // floating-point atomics into Gout, clearing Gclr for the next stage
    double *Gin = nullptr, *Gout = nullptr, *Gclr = nullptr;
    if (RK) {
        const int r = (int)((4 * n + STG - 1) % 3);
        Gin = r == 0 ? S.G0 : (r == 1 ? S.G1 : S.G2);
        Gout = r == 0 ? S.G1 : (r == 1 ? S.G2 : S.G0);
        Gclr = r == 0 ? S.G2 : (r == 1 ? S.G0 : S.G1);
    } else if (MODE == PM_DEPOSIT) {
        const int r = (int)((4 * n) % 3);
        Gout = r == 0 ? S.G0 : (r == 1 ? S.G1 : S.G2);
    } else {
        Gout = outG;
    }
    if (RK && !EXACT) {
        // nothing reads or writes Gclr during this launch
        const int64_t len = (int64_t)NGC * S.ncell;
        for (int64_t q = i; q < len; q += (int64_t)gridDim.x * BLK)
            gst(Gclr + q, 0.0);
    }
    const int64_t plane = (int64_t)NG * S.ncell;  // hi plane -> lo plane
    const double qs = S.qs;

    const double vx = gld(S.v + ip), vy = gld(S.v + np + ip), vz = gld(S.v + 2 * np + ip);
    const double px = D3 ? gld(S.pos + ip) : 0.0;
    const double py = D3 ? gld(S.pos + np + ip) : 0.0;
    const double pz = gld(S.pos + 2 * np + ip);
    const double wN = gld(S.wN + ip), wNb = gld(S.wNb + ip);
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int64_t nc = S.ncell;

    const int nn[3] = {nx, ny, nz};

    // stencil at the current position.  The grid cells a workgroup's
    // particles interpolate from are staged in LDS when they fit, except in
    // stage 4 of a 1D box, which streams the most particle data and reads
    // its two cells per particle through the caches (there the staging
    // barrier held its streams back).  In 3D the 256 reads per particle
    // from memory keep only a few loads in flight: staging them took the
    // random 32^3 box from 6.20 to 5.93 ms per step.
    int gf[3] = {0, 0, 0}, go[3] = {0, 0, 0};
    double gw[3][3] = {{1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}};
    Box gb = {};
    bool g_lds = false;
    if (RK) {
        axis_stencil<SH>(pz, vz, t_cur, S.dx[2], nz, &gf[2], gw[2]);
        if (D3) {
            axis_stencil<SH>(px, vx, t_cur, S.dx[0], nx, &gf[0], gw[0]);
            axis_stencil<SH>(py, vy, t_cur, S.dx[1], ny, &gf[1], gw[1]);
        }
    }
    if (MODE <= 3 || (D3 && RK)) {
        gb = block_box<SW, D3>(gf, active, nn, sred, sref, go);
        g_lds = gb.cells * NGC <= ACC_DOUBLES && gb.cells <= BLK;
        if (g_lds) {
            const int cells = (int)gb.cells;
            if (D3) {
                // thread l stages cell l of the box: one cell index
                // decomposition, all its components' loads in flight at once
                // (a 3D box has tens of cells; element by element, each
                // thread's loads waited one after another)
                const int l = threadIdx.x;
                if (l < cells) {
                    const int lx = l % gb.s[0], ly = (l / gb.s[0]) % gb.s[1], lz = l / (gb.s[0] * gb.s[1]);
                    const int cz = wrap_int(gb.ref[2] + gb.lo[2] + lz, nz);
                    const int cy = wrap_int(gb.ref[1] + gb.lo[1] + ly, ny);
                    const int cx = wrap_int(gb.ref[0] + gb.lo[0] + lx, nx);
                    const double *src = Gin + ((int64_t)cz * ny + cy) * nx + cx;
                    double v[NGC];
#pragma unroll
                    for (int comp = 0; comp < NGC; comp++)
                        v[comp] = gld(src + (int64_t)comp * nc);
#pragma unroll
                    for (int comp = 0; comp < NGC; comp++)
                        acc[comp * cells + l] = v[comp];
                }
            } else {
                // a 1D box has a few cells: one element per thread
                for (int q = threadIdx.x; q < NGC * cells; q += BLK) {
                    const int comp = q / cells, l = q - comp * cells;
                    const int cz = wrap_int(gb.ref[2] + gb.lo[2] + l, nz);
                    acc[q] = gld(Gin + (int64_t)comp * nc + cz);
                }
            }
            __syncthreads();
        }
    }

    double X[9], Ynew[18];
#pragma unroll
    for (int k = 0; k < 9; k++)
        X[k] = 0.0;
    if (active) {
        double Y[18];
#pragma unroll
        for (int k = 0; k < 18; k++)
            Y[k] = D3 ? fpic::gld_nt(S.Y + k * np + i) : gld(S.Y + k * np + i);
        if (MODE == PM_DEPOSIT) {
#pragma unroll
            for (int k = 0; k < 9; k++)
                X[k] = source_comp(k, wN, Y[k], wNb, Y[9 + k]);
        } else if (MODE == PM_MOM_NU) {
#pragma unroll
            for (int k = 0; k < 9; k++)
                X[k] = wN * Y[k];
        } else if (MODE == PM_MOM_NUBAR) {
#pragma unroll
            for (int k = 0; k < 9; k++)
                X[k] = wNb * Y[9 + k];
        } else {
            // interpolate the grid at the current position: from the LDS
            // box when it was staged, else from the grid in memory
            double A[NXT], Bx[NXT], By[NXT], Bz[NXT];  // traceless
#pragma unroll
            for (int k = 0; k < NXT; k++)
                A[k] = Bx[k] = By[k] = Bz[k] = 0.0;
            if (g_lds) {
                const int cells = (int)gb.cells;
#pragma unroll
                for (int bz = 0; bz < SW; bz++)
#pragma unroll
                    for (int by = 0; by < (D3 ? SW : 1); by++)
#pragma unroll
                        for (int bx = 0; bx < (D3 ? SW : 1); bx++) {
                            const double w = D3 ? (gw[0][bx] * gw[1][by]) * gw[2][bz] : gw[2][bz];
                            const double *g = acc + ((go[2] - gb.lo[2] + bz) * gb.s[1] +
                                                     (go[1] - gb.lo[1] + by)) * gb.s[0] +
                                              (go[0] - gb.lo[0] + bx);
#pragma unroll
                            for (int k = 0; k < NXT; k++) {
                                A[k] += w * g[k * cells];
                                Bx[k] += w * g[(NXT + k) * cells];
                                By[k] += w * g[(2 * NXT + k) * cells];
                                Bz[k] += w * g[(3 * NXT + k) * cells];
                            }
                        }
            } else {
#pragma unroll
                for (int bz = 0; bz < SW; bz++)
#pragma unroll
                    for (int by = 0; by < (D3 ? SW : 1); by++)
#pragma unroll
                        for (int bx = 0; bx < (D3 ? SW : 1); bx++) {
                            const double w = D3 ? (gw[0][bx] * gw[1][by]) * gw[2][bz] : gw[2][bz];
                            const int cz = wrap_int(gf[2] + bz, nz);
                            const int cy = D3 ? wrap_int(gf[1] + by, ny) : 0;
                            const int cx = D3 ? wrap_int(gf[0] + bx, nx) : 0;
                            const double *g = Gin + ((int64_t)cz * ny + cy) * nx + cx;
#pragma unroll
                            for (int k = 0; k < NXT; k++) {
                                A[k] += w * gld(g + (int64_t)k * nc);
                                Bx[k] += w * gld(g + (int64_t)(NXT + k) * nc);
                                By[k] += w * gld(g + (int64_t)(2 * NXT + k) * nc);
                                Bz[k] += w * gld(g + (int64_t)(3 * NXT + k) * nc);
                            }
                        }
            }
            // traceless Hnn: its ee entry is 0
            double Hnn[9];
            Hnn[0] = 0.0;
#pragma unroll
            for (int k = 0; k < NXT; k++)
                Hnn[k + 1] = A[k] - (vx * Bx[k] + vy * By[k] + vz * Bz[k]);
            // stage state y and the base of the next state (Y for stages
            // 1-3, Y + dt/6 (k1 + 2 k2 + 2 k3) for stage 4)
            double y[18], base[18];
            if (MODE == 1) {
#pragma unroll
                for (int k = 0; k < 18; k++)
                    y[k] = base[k] = Y[k];
            } else if (STG == 4) {
                const double h6 = dt / 6.0;
                double k1[18], k2[18], k3[18];
                load_slope<true>(S.K1, np, i, k1);
                load_slope<true>(S.K2, np, i, k2);
                load_slope<true>(S.K3, np, i, k3);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    y[k] = Y[k] + dt * k3[k];
                    const double ks = (k1[k] + 2.0 * k2[k]) + 2.0 * k3[k];
                    base[k] = Y[k] + h6 * ks;
                }
            } else {
                const double a = 0.5 * dt;
                double kp[18];
                load_slope<D3>(MODE == 2 ? S.K1 : S.K2, np, i, kp);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    y[k] = Y[k] + a * kp[k];
                    base[k] = Y[k];
                }
            }
            double H[9], Hb[9], kk[18];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                H[k] = S.hvac[k] + Hnn[k];
                const double hb = S.hvacb[k] - Hnn[k];
                Hb[k] = (k == 4 || k == 6 || k == 8) ? -hb : hb;
            }
            commutator(H, y, kk);
            commutator(Hb, y + 9, kk + 9);
            double yn[18];
            if (STG == 4) {
                const double h6 = dt / 6.0;
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yn[k] = base[k] + h6 * kk[k];
                    if (MODE == 4)
                        fpic::gst_nt(S.Y + k * np + i, yn[k]);
                    Ynew[k] = yn[k];
                }
            } else {
                double *Ko = MODE == 1 ? S.K1 : (MODE == 2 ? S.K2 : S.K3);
                const double an = MODE == 3 ? dt : 0.5 * dt;
                // k2 streams; k1 and k3 stay cached in 1D, where the next
                // kernel finds part of them in the Infinity Cache; a 3D box
                // streams every particle array (its 3 million particles'
                // arrays dwarf that cache: 6.35 -> 6.19 ms per step)
                if (MODE == 2 || D3)
                    store_slope<true>(Ko, np, i, kk);
                else
                    store_slope<false>(Ko, np, i, kk);
#pragma unroll
                for (int k = 0; k < 18; k++)
                    yn[k] = base[k] + an * kk[k];
            }
#pragma unroll
            for (int k = 0; k < 9; k++)
                X[k] = source_comp(k, wN, yn[k], wNb, yn[9 + k]);
        }
    }

    // ---- deposit with the next-stage weights ---------------------------
    // deposit sources: the traceless part of X for the stage grids
    double Xd[NCS];
    if (FULL) {
#pragma unroll
        for (int k = 0; k < NCS; k++)
            Xd[k] = X[k];
    } else {
        Xd[0] = X[1] - X[0];
        Xd[1] = X[2] - X[0];
#pragma unroll
        for (int k = 2; k < NCS; k++)
            Xd[k] = X[k + 1];
    }
    int df[3] = {0, 0, 0}, o[3];
    double dw[3][3] = {{1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}};
    axis_stencil<SH>(pz, vz, t_nxt, S.dx[2], nz, &df[2], dw[2]);
    if (D3) {
        axis_stencil<SH>(px, vx, t_nxt, S.dx[0], nx, &df[0], dw[0]);
        axis_stencil<SH>(py, vy, t_nxt, S.dx[1], ny, &df[1], dw[1]);
    }
    const Box db = block_box<SW, D3>(df, active, nn, sred, sref, o);
    const int sx = db.s[0], sy = db.s[1];
    const int64_t box = db.cells;
    constexpr int NCORNER = D3 ? SW * SW * SW : SW;
    // each lane walks its stencil corners starting at its own offset, so one
    // instruction's lanes target different corners
    const int rot = lane % NCORNER;

    if (EXACT) {
        // Limb accumulators of the box in LDS: some of the four groups
        // (A, B_x, B_y, B_z) per pass, R copies of them (lane l adding into
        // copy (l / NCORNER) % R: lanes of a dense workgroup target the same
        // few cells, and the copies and the corner rotation spread their
        // atomics over distinct addresses; a copy holds an odd number of
        // 8-byte words, so the copies start in different banks).  Every
        // contribution is the same whatever the passes, and its limbs add
        // exactly.
        // Fewer groups per pass buy more copies: passes are taken until a
        // pass holds at least four copies (or one group).
        // (workgroup-uniform integer arithmetic; box <= ACC_DOUBLES here)
        const int cells = (int)min(box, (int64_t)ACC_DOUBLES);
        int gpp = 4, R = 0;
        for (;;) {
            const int st = 2 * NCS * gpp * cells + 1;
            R = ACC_DOUBLES / st;   // copies that fit, then a power of two
            R = R >= MAX_COPIES ? MAX_COPIES : (R >= 16 ? 16 : (R >= 8 ? 8 : (R >= 4 ? 4 : (R >= 2 ? 2 : R))));
            if (R >= 4 || gpp == 1)
                break;
            gpp >>= 1;
        }
        if (R > 0 && box <= ACC_DOUBLES) {
            const int half = NCS * gpp * cells;
            const int cstride = 2 * half + 1;
            long long *lacc = reinterpret_cast<long long *>(acc);
            for (int g0 = 0; g0 < 4; g0 += gpp) {
                for (int q = threadIdx.x; q < R * cstride; q += BLK)
                    lacc[q] = 0;
                __syncthreads();
                if (active) {
                    // copy by lane / NCORNER, independent of the lane's
                    // first corner (lane % NCORNER)
                    long long *mine = lacc + ((lane / NCORNER) & (R - 1)) * cstride;
#pragma unroll 1
                    for (int g = 0; g < gpp; g++) {
                        const int gg = g0 + g;
                        const double m = gg == 0 ? 1.0 : (gg == 1 ? vx : (gg == 2 ? vy : vz));
                        long long *mg = mine + g * NCS * cells;
                        // (a rolled corner loop: unrolled, the limb
                        // conversions of all corners would spill)
#pragma unroll 1
                        for (int j = 0; j < NCORNER; j++) {
                            int c = j + rot;
                            c = c >= NCORNER ? c - NCORNER : c;
                            const int bx = D3 ? c % SW : 0;
                            const int by = D3 ? (c / SW) % SW : 0;
                            const int bz = D3 ? c / (SW * SW) : c;
                            const double w = D3 ? (pick(dw[0], bx) * pick(dw[1], by)) * pick(dw[2], bz)
                                                : pick(dw[2], bz);
                            const int idx = ((o[2] - db.lo[2] + bz) * sy + (o[1] - db.lo[1] + by)) * sx +
                                            (o[0] - db.lo[0] + bx);
#pragma unroll
                            for (int k = 0; k < NCS; k++) {
                                // m * (w X_k): the product the floating-point
                                // path forms (1 * x is x)
                                const double xc = w * Xd[k];
                                long long *a = mg + idx + k * cells;
                                lds_add_limbs(a, a + half, m * xc, qs);
                            }
                        }
                    }
                }
                __syncthreads();
                // flush; integer sums, so the order in which the atomics land
                // does not matter
                if (D3) {
                    // BLK / cells threads per box cell (each forms the cell's
                    // grid index once) share the pass's components
                    const int per = cells < BLK ? BLK / cells : 1;
                    for (int t = threadIdx.x; t < per * cells; t += BLK) {
                        const int l = t % cells, c0 = t / cells;
                        const int lx = l % sx, ly = (l / sx) % sy, lz = l / (sx * sy);
                        const int cz = wrap_int(db.ref[2] + db.lo[2] + lz, nz);
                        const int cy = wrap_int(db.ref[1] + db.lo[1] + ly, ny);
                        const int cx = wrap_int(db.ref[0] + db.lo[0] + lx, nx);
                        const int64_t cell = ((int64_t)cz * ny + cy) * nx + cx;
                        for (int c = c0; c < NCS * gpp; c += per)
                            flush_limbs(lacc, R, cstride, half, c * cells + l, S.GL,
                                        (int64_t)(g0 * NCS + c) * nc + cell, plane);
                    }
                } else {
                    // a 1D box has a few cells: one entry per thread
                    for (int q = threadIdx.x; q < half; q += BLK) {
                        const int c = q / cells, l = q - c * cells;
                        const int cz = wrap_int(db.ref[2] + db.lo[2] + l, nz);
                        flush_limbs(lacc, R, cstride, half, q, S.GL, (int64_t)(g0 * NCS + c) * nc + cz, plane);
                    }
                }
                __syncthreads();  // the next pass clears the accumulators
            }
        } else if (active) {
            // spread-out workgroup: straight to the grid limbs (a rolled
            // corner loop: unrolled, the conversions would spill)
#pragma unroll 1
            for (int c = 0; c < NCORNER; c++) {
                const int bx = D3 ? c % SW : 0;
                const int by = D3 ? (c / SW) % SW : 0;
                const int bz = D3 ? c / (SW * SW) : c;
                const double w = D3 ? (pick(dw[0], bx) * pick(dw[1], by)) * pick(dw[2], bz) : pick(dw[2], bz);
                const int cz = wrap_int(df[2] + bz, nz);
                const int cy = D3 ? wrap_int(df[1] + by, ny) : 0;
                const int cx = D3 ? wrap_int(df[0] + bx, nx) : 0;
                const int64_t g = ((int64_t)cz * ny + cy) * nx + cx;
#pragma unroll 1
                for (int k = 0; k < NCS; k++) {
                    const double xc = w * Xd[k];
                    global_add_limbs(S.GL, plane, g + (int64_t)k * nc, xc, qs);
                    global_add_limbs(S.GL, plane, g + (int64_t)(NCS + k) * nc, vx * xc, qs);
                    global_add_limbs(S.GL, plane, g + (int64_t)(2 * NCS + k) * nc, vy * xc, qs);
                    global_add_limbs(S.GL, plane, g + (int64_t)(3 * NCS + k) * nc, vz * xc, qs);
                }
            }
        }
    } else if (box * NGC <= ACC_DOUBLES) {
        // floating-point atomics (not reproducible bit for bit): R copies of
        // the box accumulator as above, flushed with global FP64 atomics
        const int cells = (int)box;
        const int cstride = NGC * cells + 1;
        int R = MAX_COPIES;
        while (R > 1 && R * cstride > ACC_DOUBLES)
            R >>= 1;
        for (int q = threadIdx.x; q < R * cstride; q += BLK)
            acc[q] = 0.0;
        __syncthreads();
        if (active) {
            double *mine = acc + ((lane / NCORNER) & (R - 1)) * cstride;
#pragma unroll
            for (int j = 0; j < NCORNER; j++) {
                int c = j + rot;
                c = c >= NCORNER ? c - NCORNER : c;
                const int bx = D3 ? c % SW : 0;
                const int by = D3 ? (c / SW) % SW : 0;
                const int bz = D3 ? c / (SW * SW) : c;
                const double w = D3 ? (pick(dw[0], bx) * pick(dw[1], by)) * pick(dw[2], bz) : pick(dw[2], bz);
                const int idx = ((o[2] - db.lo[2] + bz) * sy + (o[1] - db.lo[1] + by)) * sx + (o[0] - db.lo[0] + bx);
#pragma unroll
                for (int k = 0; k < NCS; k++) {
                    const double xc = w * Xd[k];
                    atomicAdd(&mine[k * cells + idx], xc);
                    atomicAdd(&mine[(NCS + k) * cells + idx], vx * xc);
                    atomicAdd(&mine[(2 * NCS + k) * cells + idx], vy * xc);
                    atomicAdd(&mine[(3 * NCS + k) * cells + idx], vz * xc);
                }
            }
        }
        __syncthreads();
        if (D3) {
            const int per = cells < BLK ? BLK / cells : 1;  // threads per box cell
            for (int t = threadIdx.x; t < per * cells; t += BLK) {
                const int l = t % cells, c0 = t / cells;
                const int lx = l % sx, ly = (l / sx) % sy, lz = l / (sx * sy);
                const int cz = wrap_int(db.ref[2] + db.lo[2] + lz, nz);
                const int cy = wrap_int(db.ref[1] + db.lo[1] + ly, ny);
                const int cx = wrap_int(db.ref[0] + db.lo[0] + lx, nx);
                double *gcell = Gout + ((int64_t)cz * ny + cy) * nx + cx;
                for (int comp = c0; comp < NGC; comp += per) {
                    const int q = comp * cells + l;
                    double val = 0.0;
                    for (int r = 0; r < R; r++)
                        val += acc[r * cstride + q];
                    if (val != 0.0)
                        gatomic_add(gcell + (int64_t)comp * nc, val);
                }
            }
        } else {
            for (int q = threadIdx.x; q < NGC * cells; q += BLK) {
                const int comp = q / cells, l = q - comp * cells;
                double val = 0.0;
                for (int r = 0; r < R; r++)
                    val += acc[r * cstride + q];
                if (val != 0.0)
                    gatomic_add(Gout + (int64_t)comp * nc + wrap_int(db.ref[2] + db.lo[2] + l, nz), val);
            }
        }
    } else if (active) {
#pragma unroll
        for (int bz = 0; bz < SW; bz++)
#pragma unroll
            for (int by = 0; by < (D3 ? SW : 1); by++)
#pragma unroll
                for (int bx = 0; bx < (D3 ? SW : 1); bx++) {
                    const double w = D3 ? (dw[0][bx] * dw[1][by]) * dw[2][bz] : dw[2][bz];
                    const int cz = wrap_int(df[2] + bz, nz);
                    const int cy = D3 ? wrap_int(df[1] + by, ny) : 0;
                    const int cx = D3 ? wrap_int(df[0] + bx, nx) : 0;
                    double *g = Gout + ((int64_t)cz * ny + cy) * nx + cx;
#pragma unroll
                    for (int k = 0; k < NCS; k++) {
                        const double xc = w * Xd[k];
                        gatomic_add(g + (int64_t)k * nc, xc);
                        gatomic_add(g + (int64_t)(NCS + k) * nc, vx * xc);
                        gatomic_add(g + (int64_t)(2 * NCS + k) * nc, vy * xc);
                        gatomic_add(g + (int64_t)(3 * NCS + k) * nc, vz * xc);
                    }
                }
    }

    if (MODE == PM_S4_SORT) {
        // move the particle to its place in the next step's cell order:
        // rank within the workgroup's particles of the same cell (LDS
        // histogram in the deposit buffer), one reservation per cell
        __shared__ int ksred[NWAVE][2];
        __shared__ int ksref;
        const int ncl = (int)nc;
        const int key = active ? sort_key(S, i, t_nxt) : 0;
        __syncthreads();  // the deposit box is no longer read
        const KeyRange kr = key_range(key, active, ncl, ksred, &ksref);
        int *hist = reinterpret_cast<int *>(acc);
        int64_t j;
        if (kr.len <= 2 * ACC_DOUBLES) {
            for (int q = threadIdx.x; q < kr.len; q += BLK)
                hist[q] = 0;
            __syncthreads();
            const int rank = active ? atomicAdd(&hist[kr.off - kr.lo], 1) : 0;
            __syncthreads();
            for (int q = threadIdx.x; q < kr.len; q += BLK)
                if (hist[q])
                    hist[q] = gatomic_add(S.cur + wrap_int(kr.ref + kr.lo + q, ncl), hist[q]);
            __syncthreads();
            j = active ? hist[kr.off - kr.lo] + rank : 0;
        } else {
            j = active ? gatomic_add(S.cur + key, 1) : 0;
        }
        // j < np whenever the counts were taken from the same keys (they are:
        // same inputs, same arithmetic); the guard keeps any mismatch in bounds
        if (active && j >= 0 && j < np) {
#pragma unroll
            for (int k = 0; k < 18; k++)
                gst(S.Y2 + k * np + j, Ynew[k]);
            if (D3) {
                gst(S.pos2 + j, px);
                gst(S.pos2 + np + j, py);
            }
            gst(S.pos2 + 2 * np + j, pz);
            gst(S.v2 + j, vx);
            gst(S.v2 + np + j, vy);
            gst(S.v2 + 2 * np + j, vz);
            gst(S.wN2 + j, wN);
            gst(S.wNb2 + j, wNb);
            S.pid2[j] = S.pid[i];
        }
    }
}

// After a deposit: the limb sums as doubles in the grid the next stage
// reads (Runge-Kutta stage STG of step n: G[(4n + STG) % 3]; PM_DEPOSIT:
// G[(4n) % 3], the grid stage 1 reads; moments: outG), and the limbs
// cleared for the next deposit.  Runs before the step counter moves on.
template <int MODE>
__global__ void __launch_bounds__(256) finalize_kernel(const PDesc *__restrict__ dp, double *outG)
{
    constexpr bool FULL = MODE == PM_MOM_NU || MODE == PM_MOM_NUBAR;
    constexpr int NGC = FULL ? NG : 4 * NXT;
    constexpr int STG = MODE == PM_S4_SORT ? 4 : MODE;
    const PDesc &S = *dp;
    double *G = outG;
    if (!FULL) {
        const int64_t n = *S.step;
        const int r = (int)((MODE == PM_DEPOSIT ? 4 * n : 4 * n + STG) % 3);
        G = r == 0 ? S.G0 : (r == 1 ? S.G1 : S.G2);
    }
    const int64_t len = (int64_t)NGC * S.ncell, plane = (int64_t)NG * S.ncell;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len;
         q += (int64_t)gridDim.x * blockDim.x) {
        const long long hi = S.GL[q], lo = S.GL[plane + q];
        gst(G + q, from_limbs(hi, lo, S.qi));
        S.GL[q] = 0;
        S.GL[plane + q] = 0;
    }
}

// the largest |N/dV| + |Nbar/dV| of a particle, for the scale of the exact
// deposit sums (a maximum: the same whatever the particles' order)
__global__ void __launch_bounds__(256) weight_max_kernel(const PDesc *__restrict__ dp, double *partial)
{
    const PDesc &S = *dp;
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.np;
         i += (int64_t)gridDim.x * blockDim.x)
        a = fmax(a, fabs(S.wN[i]) + fabs(S.wNb[i]));
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = sh[0];
}

__global__ void tick_kernel(const PDesc *dp)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dp->step += 1;
}

__global__ void set_step_kernel(const PDesc *dp, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dp->step = v;
}

__global__ void fill_f64(double *p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

__global__ void fill_i32(int32_t *p, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0;
}

// dstep = 1 counts the cells of the next step's start (before the stage 4
// that moves the particles), 0 those of the current step.
__global__ void __launch_bounds__(BLK) sort_count_kernel(const PDesc *__restrict__ dp, int dstep)
{
    __shared__ int hist[HIST_MAX];
    __shared__ int sred[NWAVE][2];
    __shared__ int sref;
    const PDesc &S = *dp;
    const int nc = (int)S.ncell;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const bool active = i < S.np;
    const double t = stage_time(*S.step + dstep, S.dt, 0.0);
    const int key = active ? sort_key(S, i, t) : 0;
    const KeyRange r = key_range(key, active, nc, sred, &sref);
    if (r.len <= HIST_MAX) {
        for (int j = threadIdx.x; j < r.len; j += BLK)
            hist[j] = 0;
        __syncthreads();
        if (active)
            atomicAdd(&hist[r.off - r.lo], 1);
        __syncthreads();
        for (int j = threadIdx.x; j < r.len; j += BLK)
            if (hist[j])
                gatomic_add(S.cnt + wrap_int(r.ref + r.lo + j, nc), hist[j]);
    } else if (active) {
        gatomic_add(S.cnt + key, 1);
    }
}

// exclusive scan of cnt into cur (one workgroup of 1024 threads)
__global__ void __launch_bounds__(1024) sort_scan_kernel(const PDesc *__restrict__ dp)
{
    const PDesc &S = *dp;
    __shared__ int64_t part[1024];
    const int64_t nc = S.ncell;
    const int64_t per = (nc + 1023) / 1024;
    const int64_t b = threadIdx.x * per, e = min(nc, b + per);
    int64_t s = 0;
    for (int64_t c = b; c < e; c++)
        s += S.cnt[c];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t c = b; c < e; c++) {
        const int32_t k = S.cnt[c];
        S.cur[c] = (int32_t)run;
        run += k;
    }
}

template <bool D3>
__global__ void __launch_bounds__(BLK) sort_scatter_kernel(const PDesc *__restrict__ dp)
{
    __shared__ int hist[HIST_MAX];
    __shared__ int sred[NWAVE][2];
    __shared__ int sref;
    const PDesc &S = *dp;
    const int64_t np = S.np;
    const int nc = (int)S.ncell;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const bool active = i < np;
    const double t = stage_time(*S.step, S.dt, 0.0);
    const int key = active ? sort_key(S, i, t) : 0;
    const KeyRange r = key_range(key, active, nc, sred, &sref);
    int base;
    if (r.len <= HIST_MAX) {
        // rank within the workgroup's particles of the same cell, then one
        // reservation per cell in the global cursor
        for (int jj = threadIdx.x; jj < r.len; jj += BLK)
            hist[jj] = 0;
        __syncthreads();
        const int rank = active ? atomicAdd(&hist[r.off - r.lo], 1) : 0;
        __syncthreads();
        for (int jj = threadIdx.x; jj < r.len; jj += BLK)
            if (hist[jj])
                hist[jj] = gatomic_add(S.cur + wrap_int(r.ref + r.lo + jj, nc), hist[jj]);
        __syncthreads();
        base = active ? hist[r.off - r.lo] + rank : 0;
    } else {
        base = active ? gatomic_add(S.cur + key, 1) : 0;
    }
    if (!active || base < 0 || base >= np)
        return;
    const int64_t j = base;
#pragma unroll
    for (int k = 0; k < 18; k++)
        gst(S.Y2 + k * np + j, gld(S.Y + k * np + i));
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (D3 || a == 2)
            gst(S.pos2 + a * np + j, gld(S.pos + a * np + i));
        gst(S.v2 + a * np + j, gld(S.v + a * np + i));
    }
    gst(S.wN2 + j, gld(S.wN + i));
    gst(S.wNb2 + j, gld(S.wNb + i));
    S.pid2[j] = S.pid[i];
}

// ---- loading, unloading, diagnostics ---------------------------------
__global__ void load_kernel(const PDesc *__restrict__ dp, const double *pos0, const double *dirs,
                            const double *N, const double *Nb, const double *state, double inv_dV,
                            int *bad)
{
    const PDesc &S = *dp;
    const int64_t np = S.np;
    int nbad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v2 = 0.0;
        for (int a = 0; a < 3; a++) {
            const double x = pos0[a * np + i], v = dirs[a * np + i];
            if (!isfinite(x))
                nbad++;
            v2 += v * v;
            S.pos[a * np + i] = x;
            S.v[a * np + i] = v;
        }
        if (!isfinite(v2) || fabs(v2 - 1.0) > 1e-9)
            nbad++;
        if (!isfinite(N[i]) || !isfinite(Nb[i]))
            nbad++;
        S.wN[i] = N[i] * inv_dV;
        S.wNb[i] = Nb[i] * inv_dV;
        S.pid[i] = (int32_t)i;
        for (int k = 0; k < 18; k++)
            S.Y[k * np + i] = state[k * np + i];
    }
    if (nbad)
        atomicAdd(bad, nbad);
}

__global__ void unload_kernel(const PDesc *__restrict__ dp, double *out)
{
    const PDesc &S = *dp;
    const int64_t np = S.np;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = S.pid[i];
        for (int k = 0; k < 18; k++)
            out[k * np + j] = S.Y[k * np + i];
    }
}

// Flavor totals, summed exactly in limbs like the deposits (the particle
// order within a cell is not fixed): per block the 18 (hi, lo) limb sums.
__global__ void __launch_bounds__(256) totals_kernel(const PDesc *__restrict__ dp, long long *partial)
{
    const PDesc &S = *dp;
    __shared__ long long sh[4][36];
    long long hs[18], ls[18];
    for (int k = 0; k < 18; k++)
        hs[k] = ls[k] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double wN = S.wN[i], wNb = S.wNb[i];
        for (int k = 0; k < 18; k++) {
            long long h, l;
            to_limbs((k < 9 ? wN : wNb) * S.Y[k * S.np + i], S.qs, h, l);
            hs[k] += h;
            ls[k] += l;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 18; k++) {
        for (int m = 32; m >= 1; m >>= 1) {
            hs[k] += __shfl_xor(hs[k], m, 64);
            ls[k] += __shfl_xor(ls[k], m, 64);
        }
        if (lane == 0) {
            sh[wave][2 * k] = hs[k];
            sh[wave][2 * k + 1] = ls[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 36)
        partial[blockIdx.x * 36 + threadIdx.x] =
            sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

__global__ void totals_finish_kernel(const PDesc *__restrict__ dp, const long long *partial, int nblk,
                                     double *out)
{
    const int k = threadIdx.x;
    if (k >= 18)
        return;
    long long h = 0, l = 0;
    for (int b = 0; b < nblk; b++) {
        h += partial[(size_t)b * 36 + 2 * k];
        l += partial[(size_t)b * 36 + 2 * k + 1];
    }
    out[k] = from_limbs(h, l, dp->qi);
}

__global__ void __launch_bounds__(256) check_kernel(const PDesc *__restrict__ dp, double *partial)
{
    const PDesc &S = *dp;
    __shared__ double sh[3][256];
    double e0 = 0.0, e1 = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.np;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v[18];
        for (int k = 0; k < 18; k++) {
            v[k] = S.Y[k * S.np + i];
            if (!isfinite(v[k]))
                bad += 1.0;
        }
        e0 = fmax(e0, fabs(v[0] + v[1] + v[2] - 1.0));
        e1 = fmax(e1, fabs(v[9] + v[10] + v[11] - 1.0));
    }
    sh[0][threadIdx.x] = e0;
    sh[1][threadIdx.x] = e1;
    sh[2][threadIdx.x] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + h]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + h]);
            sh[2][threadIdx.x] += sh[2][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; q++)
            partial[blockIdx.x * 3 + q] = sh[q][0];
}

__global__ void finish_kernel(const double *partial, int nblk, int width, int is_check, double *out)
{
    const int k = threadIdx.x;
    if (k >= width)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) {
        const double v = partial[(size_t)b * width + k];
        s = (is_check && k < 2) ? fmax(s, v) : s + v;
    }
    out[k] = s;
}

// ------------------------------------------------------------------ host
#define HIPCHECK(x)                                                                     \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess)                                                           \
            return fail(FPIC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));    \
    } while (0)

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t set[2][6];  // Y, pos, v, wN, wNb, pid of sets A and B
    size_t K1, K2, K3, G[3], GL, cnt, cur, step, desc, scratch, flag, total;
};

static int validate(const fpic_pconfig &c)
{
    if (c.ncell[0] < 1 || c.ncell[1] < 1 || c.ncell[2] < 1)
        return fail(FPIC_EINVAL, "cell counts must be >= 1");
    if ((int64_t)c.ncell[0] * c.ncell[1] * c.ncell[2] > ((int64_t)1 << 30))
        return fail(FPIC_EINVAL, "too many cells");
    if (c.npart < 1 || c.npart > INT32_MAX)
        return fail(FPIC_EINVAL, "npart must be in 1 .. 2^31 - 1");
    if (c.shape_order != 1 && c.shape_order != 2)
        return fail(FPIC_EUNSUPPORTED, "shape_order must be 1 (linear) or 2 (quadratic)");
    if (c.sort_every < 0 || c.sort_every > 1024)
        return fail(FPIC_EINVAL, "sort_every must be in 0 .. 1024");
    if (c.flags & ~FPIC_PFLOAT_ATOMICS)
        return fail(FPIC_EINVAL, "unknown flags");
    if (!(c.dt > 0.0) || !std::isfinite(c.dt))
        return fail(FPIC_EINVAL, "dt must be positive and finite");
    for (int a = 0; a < 3; ++a)
        if (!(c.dx[a] > 0.0) || !std::isfinite(c.dx[a]))
            return fail(FPIC_EINVAL, "cell widths must be positive and finite");
    double hmax = 0.0;
    for (int i = 0; i < 18; ++i) {
        if (!std::isfinite(c.hvac[i]))
            return fail(FPIC_EINVAL, "hvac has a non-finite entry");
        hmax = std::max(hmax, std::fabs(c.hvac[i]));
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c.vmat[a]))
            return fail(FPIC_EINVAL, "vmat has a non-finite entry");
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double re = c.hvac[2 * (3 * i + j)], im = c.hvac[2 * (3 * i + j) + 1];
            const double rt = c.hvac[2 * (3 * j + i)], it = c.hvac[2 * (3 * j + i) + 1];
            if (std::fabs(re - rt) + std::fabs(im + it) > 1e-12 * (1.0 + hmax))
                return fail(FPIC_EINVAL, "hvac is not Hermitian");
        }
    return FPIC_OK;
}

static int layout(const fpic_pconfig &c, Layout &L)
{
    int rc = validate(c);
    if (rc)
        return rc;
    const size_t np = (size_t)c.npart;
    const size_t nc = (size_t)c.ncell[0] * c.ncell[1] * c.ncell[2];
    size_t off = 0;
    auto take = [&](size_t b) {
        off = al(off);
        const size_t o = off;
        off += b;
        return o;
    };
    const size_t d = sizeof(double);
    for (int s = 0; s < 2; ++s) {
        L.set[s][0] = take(d * 18 * np);
        L.set[s][1] = take(d * 3 * np);
        L.set[s][2] = take(d * 3 * np);
        L.set[s][3] = take(d * np);
        L.set[s][4] = take(d * np);
        L.set[s][5] = take(sizeof(int32_t) * np);
    }
    L.K1 = take(d * fpic::NK * np);
    L.K2 = take(d * fpic::NK * np);
    L.K3 = take(d * fpic::NK * np);
    for (int g = 0; g < 3; ++g)
        L.G[g] = take(d * NG * nc);
    L.GL = take(sizeof(long long) * 2 * NG * nc);
    L.cnt = take(sizeof(int32_t) * nc);
    L.cur = take(sizeof(int32_t) * nc);
    L.step = take(sizeof(int64_t));
    L.desc = take(2 * sizeof(PDesc));
    L.scratch = take(d * (kScratch3 + kRedBlk));
    L.flag = take(sizeof(int32_t) * 4);
    L.total = al(off);
    return FPIC_OK;
}

}  // namespace fpicp

using namespace fpicp;

struct fpic_pctx {
    PDesc h[2];          // parity p: current set p, the sort writes set 1 - p
    PDesc *d[2] = {nullptr, nullptr};
    char *ws = nullptr;
    hipStream_t stream = nullptr, cap = nullptr;
    int spg = 4;         // steps between sorts (= steps per graph)
    int par = 0;         // set holding the particles after the enqueued work
    int sh = 1;
    bool d3 = false;
    bool exact = true;   // exact (limb) deposit sums; false: floating-point atomics
    unsigned nblk = 1;   // stage workgroups
    double dV = 1.0;
    double *scratch = nullptr, *hbuf = nullptr;
    int32_t *flag = nullptr;
    hipGraphExec_t g[2] = {nullptr, nullptr};
    bool state_set = false;
};

namespace fpicp {

template <int SH, bool D3, bool EX>
static void launch_mode_t(const fpic_pctx *c, int mode, const PDesc *dd, double *out, hipStream_t s)
{
    const dim3 grid(c->nblk), blk(BLK);
    switch (mode) {
    case 1: pstage_kernel<1, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case 2: pstage_kernel<2, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case 3: pstage_kernel<3, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case 4: pstage_kernel<4, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_S4_SORT: pstage_kernel<PM_S4_SORT, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_DEPOSIT: pstage_kernel<PM_DEPOSIT, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_MOM_NU: pstage_kernel<PM_MOM_NU, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    default: pstage_kernel<PM_MOM_NUBAR, SH, D3, EX><<<grid, blk, 0, s>>>(dd, out); break;
    }
}

// the limb sums of a deposit (mode as above) into their grid
static void launch_finalize(const fpic_pctx *c, int mode, const PDesc *dd, double *out, hipStream_t s)
{
    const bool full = mode == PM_MOM_NU || mode == PM_MOM_NUBAR;
    const int64_t len = (int64_t)(full ? NG : 4 * NXT) * c->h[0].ncell;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (len + 255) / 256))), blk(256);
    switch (mode) {
    case 1: finalize_kernel<1><<<grid, blk, 0, s>>>(dd, out); break;
    case 2: finalize_kernel<2><<<grid, blk, 0, s>>>(dd, out); break;
    case 3: finalize_kernel<3><<<grid, blk, 0, s>>>(dd, out); break;
    case 4: finalize_kernel<4><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_S4_SORT: finalize_kernel<PM_S4_SORT><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_DEPOSIT: finalize_kernel<PM_DEPOSIT><<<grid, blk, 0, s>>>(dd, out); break;
    case PM_MOM_NU: finalize_kernel<PM_MOM_NU><<<grid, blk, 0, s>>>(dd, out); break;
    default: finalize_kernel<PM_MOM_NUBAR><<<grid, blk, 0, s>>>(dd, out); break;
    }
}

template <bool EX>
static void launch_mode_e(const fpic_pctx *c, int mode, const PDesc *dd, double *out, hipStream_t s)
{
    if (c->sh == 2) {
        if (c->d3) launch_mode_t<2, true, EX>(c, mode, dd, out, s);
        else launch_mode_t<2, false, EX>(c, mode, dd, out, s);
    } else {
        if (c->d3) launch_mode_t<1, true, EX>(c, mode, dd, out, s);
        else launch_mode_t<1, false, EX>(c, mode, dd, out, s);
    }
}

// a stage or deposit launch, and with exact sums the finalize of its limbs
static void launch_mode(const fpic_pctx *c, int mode, const PDesc *dd, double *out, hipStream_t s)
{
    if (c->exact) {
        launch_mode_e<true>(c, mode, dd, out, s);
        launch_finalize(c, mode, dd, out, s);
    } else {
        launch_mode_e<false>(c, mode, dd, out, s);
    }
}

// cell counts and offsets of set par (dstep = 1: at the next step's start)
static void launch_count_scan(const fpic_pctx *c, int par, int dstep, hipStream_t s)
{
    const PDesc &H = c->h[par];
    const PDesc *dd = c->d[par];
    fill_i32<<<std::max<int64_t>(1, std::min<int64_t>(1024, (H.ncell + 255) / 256)), 256, 0, s>>>(H.cnt, H.ncell);
    sort_count_kernel<<<c->nblk, BLK, 0, s>>>(dd, dstep);
    sort_scan_kernel<<<1, 1024, 0, s>>>(dd);
}

// Stages 1-4 of one step on set par and the step counter; with sort_after,
// stage 4 writes the particles into set 1 - par in the next step's cell
// order (the caller flips the parity).
static void launch_step(const fpic_pctx *c, int par, bool sort_after, hipStream_t s)
{
    for (int m = 1; m <= 3; ++m)
        launch_mode(c, m, c->d[par], nullptr, s);
    if (sort_after) {
        launch_count_scan(c, par, 1, s);
        launch_mode(c, PM_S4_SORT, c->d[par], nullptr, s);
    } else {
        launch_mode(c, 4, c->d[par], nullptr, s);
    }
    tick_kernel<<<1, 64, 0, s>>>(c->d[par]);
}

// counting sort of the particles in set par into set 1 - par, in a pass of
// its own (after loading)
static void launch_sort(const fpic_pctx *c, int par, hipStream_t s)
{
    const PDesc *dd = c->d[par];
    launch_count_scan(c, par, 0, s);
    if (c->d3)
        sort_scatter_kernel<true><<<c->nblk, BLK, 0, s>>>(dd);
    else
        sort_scatter_kernel<false><<<c->nblk, BLK, 0, s>>>(dd);
}

static int capture(fpic_pctx *c, int par, hipGraphExec_t *exec)
{
    HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < c->spg; ++k)
        launch_step(c, par, k == c->spg - 1, c->cap);
    hipError_t err = hipGetLastError();
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &gr);
    if (err != hipSuccess) {
        if (gr)
            (void)hipGraphDestroy(gr);
        return fail(FPIC_EHIP, std::string("launch during capture: ") + hipGetErrorString(err));
    }
    HIPCHECK(e2);
    hipError_t e3 = hipGraphInstantiate(exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIPCHECK(e3);
    return FPIC_OK;
}

}  // namespace fpicp

extern "C" {

int fpic_particles_workspace_bytes(const fpic_pconfig *cfg, size_t *bytes)
{
    if (!cfg || !bytes)
        return fail(FPIC_EINVAL, "null argument");
    Layout L;
    int rc = layout(*cfg, L);
    if (rc)
        return rc;
    *bytes = L.total;
    return FPIC_OK;
}

int fpic_particles_create(const fpic_pconfig *cfg, void *workspace, size_t bytes, fpic_stream stream,
                          fpic_pctx **out)
{
    if (!cfg || !out)
        return fail(FPIC_EINVAL, "null argument");
    *out = nullptr;
    Layout L;
    int rc = layout(*cfg, L);
    if (rc)
        return rc;
    if (!workspace || bytes < L.total || reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(FPIC_EINVAL, "workspace missing, too small or misaligned");
    fpic_pctx *c = new fpic_pctx();
    c->ws = static_cast<char *>(workspace);
    c->stream = static_cast<hipStream_t>(stream);
    c->spg = cfg->sort_every ? cfg->sort_every : 4;
    c->sh = cfg->shape_order;
    c->d3 = !(cfg->ncell[0] == 1 && cfg->ncell[1] == 1);
    c->exact = !(cfg->flags & FPIC_PFLOAT_ATOMICS);
    c->nblk = (unsigned)((cfg->npart + BLK - 1) / BLK);
    c->dV = cfg->dx[0] * cfg->dx[1] * cfg->dx[2];
    auto P = [&](size_t o) { return reinterpret_cast<double *>(c->ws + o); };
    auto I = [&](size_t o) { return reinterpret_cast<int32_t *>(c->ws + o); };
    for (int p = 0; p < 2; ++p) {
        PDesc &D = c->h[p];
        std::memset(&D, 0, sizeof D);
        for (int a = 0; a < 3; ++a) {
            D.n[a] = cfg->ncell[a];
            D.dx[a] = cfg->dx[a];
        }
        D.shape = cfg->shape_order;
        D.ncell = (int64_t)cfg->ncell[0] * cfg->ncell[1] * cfg->ncell[2];
        D.np = cfg->npart;
        D.dt = cfg->dt;
        const double *h = cfg->hvac;
        const double hv[9] = {h[0], h[8], h[16], h[2], h[3], h[4], h[5], h[10], h[11]};
        for (int k = 0; k < 9; ++k) {
            D.hvac[k] = hv[k] + (k < 3 ? cfg->vmat[k] : 0.0);
            D.hvacb[k] = hv[k] - (k < 3 ? cfg->vmat[k] : 0.0);
        }
        const int s = p, t = 1 - p;
        D.Y = P(L.set[s][0]);
        D.pos = P(L.set[s][1]);
        D.v = P(L.set[s][2]);
        D.wN = P(L.set[s][3]);
        D.wNb = P(L.set[s][4]);
        D.pid = I(L.set[s][5]);
        D.Y2 = P(L.set[t][0]);
        D.pos2 = P(L.set[t][1]);
        D.v2 = P(L.set[t][2]);
        D.wN2 = P(L.set[t][3]);
        D.wNb2 = P(L.set[t][4]);
        D.pid2 = I(L.set[t][5]);
        D.K1 = P(L.K1);
        D.K2 = P(L.K2);
        D.K3 = P(L.K3);
        D.G0 = P(L.G[0]);
        D.G1 = P(L.G[1]);
        D.G2 = P(L.G[2]);
        D.cnt = I(L.cnt);
        D.cur = I(L.cur);
        D.GL = reinterpret_cast<long long *>(c->ws + L.GL);
        D.qs = D.qi = 1.0;
        D.step = reinterpret_cast<int64_t *>(c->ws + L.step);
        c->d[p] = reinterpret_cast<PDesc *>(c->ws + L.desc) + p;
    }
    c->scratch = P(L.scratch);
    c->flag = I(L.flag);
    hipError_t e = hipMemcpy(c->d[0], c->h, sizeof(PDesc) * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&c->hbuf), sizeof(double) * 64, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        fpic_particles_destroy(c);
        return fail(FPIC_EHIP, std::string("create: ") + hipGetErrorString(e));
    }
    rc = capture(c, 0, &c->g[0]);
    if (!rc)
        rc = capture(c, 1, &c->g[1]);
    if (rc) {
        fpic_particles_destroy(c);
        return rc;
    }
    *out = c;
    return FPIC_OK;
}

int fpic_particles_set(fpic_pctx *c, const double *pos0, const double *dirs, const double *N,
                       const double *Nbar, const double *state, int64_t step0)
{
    if (!c || !pos0 || !dirs || !N || !Nbar || !state)
        return fail(FPIC_EINVAL, "set: null argument");
    if (step0 < 0)
        return fail(FPIC_EINVAL, "set: step0 must be >= 0");
    hipStream_t s = c->stream;
    c->par = 0;
    const PDesc &H = c->h[0];
    fill_i32<<<1, 64, 0, s>>>(c->flag, 4);
    const unsigned nb = (unsigned)std::min<int64_t>(2048, (H.np + 255) / 256);
    load_kernel<<<nb, 256, 0, s>>>(c->d[0], pos0, dirs, N, Nbar, state, 1.0 / c->dV, c->flag);
    set_step_kernel<<<1, 64, 0, s>>>(c->d[0], step0);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    int32_t bad = 0;
    std::memcpy(&bad, c->hbuf, sizeof bad);
    if (bad) {
        c->state_set = false;
        return fail(FPIC_EINVAL, "set: non-finite position or weight, or a direction that is "
                                 "not a unit vector");
    }
    // the fixed-point scale of the exact deposit sums: 2^S with
    // 16 np max_p (|N_p| + |Nbar_p|)/dV <= 2^84.  A contribution is at most
    // 2 max_p (|N_p| + |Nbar_p|)/dV and a cell's moment component at most
    // 2 sum_p (|N_p| + |Nbar_p|)/dV (density-matrix entries and differences
    // of two diagonal entries are at most 1, velocity components and shape
    // weights at most 1): both stay below 2^81 after scaling, a factor 4
    // inside the 2^83 that the limb split needs (room for states whose
    // entries drift past 1), and no limb sum can overflow.
    // The bound uses a maximum, not a sum, so that S does not depend on the
    // order of the particles.
    double *wmax = c->scratch + kScratch3;
    weight_max_kernel<<<kRedBlk, 256, 0, s>>>(c->d[0], wmax);
    finish_kernel<<<1, 64, 0, s>>>(wmax, kRedBlk, 1, 1, c->scratch);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->scratch, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double wtot = 16.0 * (double)H.np * c->hbuf[0];
    int S2 = 0;
    if (wtot > 0.0 && std::isfinite(wtot)) {
        int e = 0;
        (void)std::frexp(wtot, &e);  // wtot < 2^e
        S2 = 84 - e;
    }
    if (c->exact && (S2 < -900 || S2 > 900)) {
        // 2^S and 2^-S must stay normal doubles with room for the scaled
        // contributions; weights this extreme take the floating-point path
        c->state_set = false;
        return fail(FPIC_EUNSUPPORTED, "set: weights outside the range of the exact deposit sums "
                                       "(16 npart max(|N| + |Nbar|)/dV outside about 2^-816 .. 2^984); use FPIC_PFLOAT_ATOMICS");
    }
    S2 = std::max(-1000, std::min(1000, S2));  // (the totals' scale with floating-point atomics)
    for (int p = 0; p < 2; ++p) {
        c->h[p].qs = std::ldexp(1.0, S2);
        c->h[p].qi = std::ldexp(1.0, -S2);
    }
    HIPCHECK(hipMemcpy(c->d[0], c->h, sizeof(PDesc) * 2, hipMemcpyHostToDevice));
    launch_sort(c, 0, s);
    c->par = 1;
    const int64_t glen = (int64_t)NG * H.ncell;
    const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (glen + 255) / 256));
    fill_f64<<<gb, 256, 0, s>>>(H.G0, glen);
    fill_f64<<<gb, 256, 0, s>>>(H.G1, glen);
    fill_f64<<<gb, 256, 0, s>>>(H.G2, glen);
    fill_f64<<<gb, 256, 0, s>>>(reinterpret_cast<double *>(H.GL), 2 * glen);
    launch_mode(c, PM_DEPOSIT, c->d[c->par], nullptr, s);
    HIPCHECK(hipGetLastError());
    c->state_set = true;
    return FPIC_OK;
}

int fpic_particles_get_state(fpic_pctx *c, double *state)
{
    if (!c || !state)
        return fail(FPIC_EINVAL, "get_state: null argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "get_state before set");
    const unsigned nb = (unsigned)std::min<int64_t>(2048, (c->h[0].np + 255) / 256);
    unload_kernel<<<nb, 256, 0, c->stream>>>(c->d[c->par], state);
    HIPCHECK(hipGetLastError());
    return FPIC_OK;
}

int fpic_particles_step(fpic_pctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0)
        return fail(FPIC_EINVAL, "step: bad argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "step before set");
    int64_t left = nsteps;
    while (left >= c->spg) {
        HIPCHECK(hipGraphLaunch(c->g[c->par], c->stream));
        c->par ^= 1;
        left -= c->spg;
    }
    if (left > 0) {
        for (int64_t k = 0; k < left; ++k)
            launch_step(c, c->par, k == left - 1, c->stream);
        HIPCHECK(hipGetLastError());
        c->par ^= 1;
    }
    return FPIC_OK;
}

int fpic_particles_moments(fpic_pctx *c, double *out)
{
    if (!c || !out)
        return fail(FPIC_EINVAL, "moments: null argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "moments before set");
    if (!c->exact) {  // the atomics add into out
        const int64_t len = (int64_t)2 * NG * c->h[0].ncell;
        const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (len + 255) / 256));
        fill_f64<<<gb, 256, 0, c->stream>>>(out, len);
    }
    launch_mode(c, PM_MOM_NU, c->d[c->par], out, c->stream);
    launch_mode(c, PM_MOM_NUBAR, c->d[c->par], out + (size_t)NG * c->h[0].ncell, c->stream);
    HIPCHECK(hipGetLastError());
    return FPIC_OK;
}

int fpic_particles_flavor_totals(fpic_pctx *c, double *out)
{
    if (!c || !out)
        return fail(FPIC_EINVAL, "flavor_totals: null argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "flavor_totals before set");
    long long *part = reinterpret_cast<long long *>(c->scratch + kScratch1);
    totals_kernel<<<kRedBlk, 256, 0, c->stream>>>(c->d[c->par], part);
    totals_finish_kernel<<<1, 64, 0, c->stream>>>(c->d[c->par], part, kRedBlk, c->scratch);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->scratch, sizeof(double) * 18, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < 18; ++k)
        out[k] = c->hbuf[k] * c->dV;
    return FPIC_OK;
}

int fpic_particles_check(fpic_pctx *c, double tol, double *max_trace_err)
{
    if (!c)
        return fail(FPIC_EINVAL, "null context");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "check before set");
    double *part = c->scratch + kScratch2;
    check_kernel<<<kRedBlk, 256, 0, c->stream>>>(c->d[c->par], part);
    finish_kernel<<<1, 64, 0, c->stream>>>(part, kRedBlk, 3, 1, c->scratch);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->scratch, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    const double e = std::max(c->hbuf[0], c->hbuf[1]);
    if (max_trace_err)
        *max_trace_err = e;
    if (c->hbuf[2] > 0.0)
        return fail(FPIC_ENUMERIC, "state holds NaN or Inf entries");
    if (!(e <= tol))
        return fail(FPIC_ENUMERIC, "trace drift exceeds the tolerance");
    return FPIC_OK;
}

int fpic_particles_get_step(fpic_pctx *c, int64_t *step)
{
    if (!c || !step)
        return fail(FPIC_EINVAL, "null argument");
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->h[0].step, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    std::memcpy(step, c->hbuf, sizeof(int64_t));
    return FPIC_OK;
}

int fpic_particles_sync(fpic_pctx *c)
{
    if (!c)
        return fail(FPIC_EINVAL, "null context");
    HIPCHECK(hipStreamSynchronize(c->stream));
    return FPIC_OK;
}

int fpic_particles_profile(fpic_pctx *c, int32_t nsteps, double *ms)
{
    if (!c || !ms || nsteps < 1)
        return fail(FPIC_EINVAL, "profile: bad argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "profile before set");
    hipEvent_t ev[6];
    for (auto &e : ev)
        HIPCHECK(hipEventCreate(&e));
    double acc[6] = {0, 0, 0, 0, 0, 0};
    hipStream_t s = c->stream;
    int rc = FPIC_OK;
    for (int n = 0; n < nsteps && !rc; ++n) {
        const int p = c->par;
        (void)hipEventRecord(ev[0], s);
        for (int m = 1; m <= 3; ++m) {
            launch_mode(c, m, c->d[p], nullptr, s);
            (void)hipEventRecord(ev[m], s);
        }
        launch_count_scan(c, p, 1, s);
        (void)hipEventRecord(ev[4], s);
        launch_mode(c, PM_S4_SORT, c->d[p], nullptr, s);
        tick_kernel<<<1, 64, 0, s>>>(c->d[p]);
        (void)hipEventRecord(ev[5], s);
        c->par ^= 1;
        hipError_t err = hipGetLastError();
        if (err == hipSuccess)
            err = hipEventSynchronize(ev[5]);
        // intervals: stages 1-3, count and scan, stage 4 (with the move)
        const int slot[5] = {0, 1, 2, 4, 3};
        for (int k = 0; k < 5 && err == hipSuccess; ++k) {
            float t = 0.f;
            err = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[slot[k]] += t;
        }
        float tt = 0.f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&tt, ev[0], ev[5]);
        acc[5] += tt;
        if (err != hipSuccess)
            rc = fail(FPIC_EHIP, std::string("profile: ") + hipGetErrorString(err));
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    for (int k = 0; k < 6; ++k)
        ms[k] = acc[k] / nsteps;
    return rc;
}

void fpic_particles_destroy(fpic_pctx *c)
{
    if (!c)
        return;
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->g)
        if (g)
            (void)hipGraphExecDestroy(g);
    if (c->cap)
        (void)hipStreamDestroy(c->cap);
    if (c->hbuf)
        (void)hipHostFree(c->hbuf);
    delete c;
}

}  // extern "C"
