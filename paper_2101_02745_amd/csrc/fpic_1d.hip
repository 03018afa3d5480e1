// HIP kernels of the 1D hot path (gfx950, FP64, wave64).
//
// One launch per Runge-Kutta stage covers every tile of every simulation of
// a batch.  A workgroup owns one tile of TILE = 64 consecutive cells and one
// group of directions; each of its waves sweeps `dpw` directions.  For
// direction d, lane l handles the particle whose *next-stage* left cell is
// m = tile*64 + l (positions are implicit, see below).  Per particle the
// lane
//   1. forms the stage state y_s from Y and the previous slope,
//   2. interpolates the staged grid tile (LDS) at the particle's current
//      position with the linear shape function (eq. pic_interpolation),
//   3. builds H and Hbar (eq. potentials, antineutrino conventions of
//      Sec. II.A) and the slopes -i[H, rho], -i[Hbar, rhobar] (eq. eom),
//   4. writes the slope (or the finished step) and forms the next-stage
//      state; with RK1 stage 1 writes no slope, and stages 2 and 4 form k1
//      again from the state and the stage-1 grid,
//   5. deposits that state with the next-stage weights (eq. pic_deposition):
//      its left weight goes to cell m, its right weight to cell m+1, which
//      lane l+1 picks up with a one-lane shuffle; the last lane's right part
//      goes to an edge partial.
// The deposit therefore needs no atomics: each lane accumulates the 36
// combined moments of its own cell over its directions in registers, the
// waves of a workgroup are summed in LDS in a fixed order, and a small
// reduction kernel sums the direction groups (and the edge partials) in a
// fixed order.  Results are bitwise reproducible run to run.
//
// Positions.  Every particle starts at the centre of its cell and moves with
// constant Omega (eq. eom), so at stage time t its displacement along z in
// cells is u = (Omega_z t) / dz, the same for every particle of a direction:
// floor(u) is the integer shift, u - floor(u) the CIC fraction.  Stage times
// are t = n dt + c_s dt (c_s = 0, 1/2, 1/2, 1), each operation rounded once,
// exactly as the CPU reference forms them.
#include "fpic_device.h"
#include "fpic_internal.h"

namespace fpic {

struct Shift {
    int64_t i;
    double phi;
};

__device__ __forceinline__ Shift shift_of(double v, double t, double dx)
{
#pragma clang fp contract(off)
    const double u = (v * t) / dx;
    const double fl = floor(u);
    Shift s;
    s.i = (int64_t)fl;
    s.phi = u - fl;
    return s;
}

// Value of the lane one below (lane 0 receives 0): DPP wave_shr:1 on the two
// 32-bit halves, no LDS traffic.
__device__ __forceinline__ double lane_below(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Value of the lane one above (lane 63 receives 0): DPP wave_shl:1.
__device__ __forceinline__ double lane_above(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int pmod_i64(int64_t a, int n)
{
    int64_t r = a % n;
    return (int)(r < 0 ? r + n : r);
}

// r = i mod n for an integer-valued double i (|i| < 2^52), without 64-bit
// integer division.
__device__ __forceinline__ int pmod_dbl(double i, int n)
{
    const double nd = (double)n;
    double r = i - nd * floor(i / nd);
    if (r < 0.0)
        r += nd;
    if (r >= nd)
        r -= nd;
    return (int)r;
}

// The slope path of the 1D stages (gather, Hamiltonians, commutators) is
// written with explicit fused multiply-adds and no other contraction, so a
// slope formed again in a later stage rounds exactly as where it was first
// formed, whatever the surrounding code lets the compiler fuse.

// Neutrino self-interaction part of H at a particle (eq. potentials,
// interpolated with eq. pic_interpolation): the four staged moment groups
// n - nbar^*, f_x, f_y, f_z - fbar^* of the tile Gt (stride gts per
// component) at column kl and fraction phi, combined as n - v.f.
template <int SH>
__device__ __forceinline__ void gather_hnn(const double *Gt, int gts, int kl, double phi, double vx,
                                           double vy, double vz, double Hnn[9])
{
#pragma clang fp contract(off)
    if (SH == 2) {
        const Quad q = quad_weights(phi);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double *g = Gt + k * gts + kl - 1 + q.up;
            double B[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const double *h = g + 9 * c * gts;
                B[c] = __builtin_fma(q.w2, h[2], __builtin_fma(q.w1, h[1], q.w0 * h[0]));
            }
            Hnn[k] = __builtin_fma(-vz, B[3], __builtin_fma(-vy, B[2], __builtin_fma(-vx, B[1], B[0])));
        }
    } else {
        const double omp = 1.0 - phi;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double *g = Gt + k * gts + kl;
            double B[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const double *h = g + 9 * c * gts;
                B[c] = __builtin_fma(phi, h[1], omp * h[0]);
            }
            Hnn[k] = __builtin_fma(-vz, B[3], __builtin_fma(-vy, B[2], __builtin_fma(-vx, B[1], B[0])));
        }
    }
}

// -i [H, rho] for Hermitian H and rho packed as 9 reals (diagonal, then
// Re/Im of the (0,1), (0,2), (1,2) entries), the same packing and slope as
// commutator() of the shared helpers, each sum of products written as one
// chain of fused multiply-adds.
__device__ __forceinline__ void commutator_fma(const double h[9], const double r[9], double k[9])
{
#pragma clang fp contract(off)
    const double h0 = h[0], h1 = h[1], h2 = h[2];
    const double ar = h[3], ai = h[4], br = h[5], bi = h[6], cr = h[7], ci = h[8];
    const double p0 = r[0], p1 = r[1], p2 = r[2];
    const double xr = r[3], xi = r[4], yr = r[5], yi = r[6], zr = r[7], zi = r[8];
    const double k1 = 2.0 * (__builtin_fma(ar, xi, -(ai * xr)) + __builtin_fma(ci, zr, -(cr * zi)));
    const double k2 = 2.0 * (__builtin_fma(br, yi, -(bi * yr)) + __builtin_fma(cr, zi, -(ci * zr)));
    k[1] = k1;
    k[2] = k2;
    k[0] = -(k1 + k2);
    // C01 = h0 x + a p1 + b z^*,  C10 = a^* p0 + h1 x^* + c y^*
    const double c01r = __builtin_fma(h0, xr, __builtin_fma(ar, p1, __builtin_fma(br, zr, bi * zi)));
    const double c01i = __builtin_fma(h0, xi, __builtin_fma(ai, p1, __builtin_fma(bi, zr, -(br * zi))));
    const double c10r = __builtin_fma(ar, p0, __builtin_fma(h1, xr, __builtin_fma(cr, yr, ci * yi)));
    const double c10i = __builtin_fma(-ai, p0, __builtin_fma(-h1, xi, __builtin_fma(ci, yr, -(cr * yi))));
    k[3] = c01i + c10i;
    k[4] = c10r - c01r;
    // C02 = h0 y + a z + b p2,  C20 = b^* p0 + c^* x^* + h2 y^*
    const double c02r = __builtin_fma(h0, yr, __builtin_fma(ar, zr, __builtin_fma(-ai, zi, br * p2)));
    const double c02i = __builtin_fma(h0, yi, __builtin_fma(ar, zi, __builtin_fma(ai, zr, bi * p2)));
    const double c20r = __builtin_fma(br, p0, __builtin_fma(cr, xr, __builtin_fma(-ci, xi, h2 * yr)));
    const double c20i = __builtin_fma(-bi, p0, __builtin_fma(-cr, xi, __builtin_fma(-ci, xr, -(h2 * yi))));
    k[5] = c02i + c20i;
    k[6] = c20r - c02r;
    // C12 = a^* y + h1 z + c p2,  C21 = b^* x + c^* p1 + h2 z^*
    const double c12r = __builtin_fma(ar, yr, __builtin_fma(ai, yi, __builtin_fma(h1, zr, cr * p2)));
    const double c12i = __builtin_fma(ar, yi, __builtin_fma(-ai, yr, __builtin_fma(h1, zi, ci * p2)));
    const double c21r = __builtin_fma(br, xr, __builtin_fma(bi, xi, __builtin_fma(cr, p1, h2 * zr)));
    const double c21i = __builtin_fma(br, xi, __builtin_fma(-bi, xr, __builtin_fma(-ci, p1, -(h2 * zi))));
    k[7] = c12i + c21i;
    k[8] = c21r - c12r;
}

// Slopes of rho and rhobar (eq. eom): H = Hvac + Hmat + Hnn and
// Hbar = (Hvac - Hmat - Hnn)^*, hv and hvb holding Hvac + Hmat and
// Hvac - Hmat packed.
__device__ __forceinline__ void slope_of(const double hv[9], const double hvb[9], const double Hnn[9],
                                         const double y[18], double kk[18])
{
#pragma clang fp contract(off)
    double H[9], Hb[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        H[k] = hv[k] + Hnn[k];
        const double hb = hvb[k] - Hnn[k];
        Hb[k] = (k == 4 || k == 6 || k == 8) ? -hb : hb;
    }
    commutator_fma(H, y, kk);
    commutator_fma(Hb, y + 9, kk + 9);
}

// NT: streaming (nontemporal) cache policy for the data a stage does not
// read again soon (the last reads of the slopes in stage 4, and k2); the
// default policy keeps everything cacheable.  Streaming pays when
// the arrays overflow the Infinity Cache (a large single box), not for
// smaller working sets (chosen per context, see fpic_tuning.cache_policy).
// SH: shape-function order, 1 (linear) or 2 (quadratic).  The staged grid
// tile holds cells tile*64 - SH .. tile*64 + 64 + SH; the quadratic deposit
// reaches one cell left of the tile and two right of it (edge partials).
// RK: slopes formed again instead of stored.  RK >= 1: stage 1 stores no k1;
// stages 2 and 4 form it again from the state and the stage-1 grid, which
// stays in HBM until stage 4 ends (the grid is tiny in 1D, so 128 B per
// particle are neither written in stage 1 nor read in stages 2 and 4).
// RK = 2: stage 2 stores no k2 either; stages 3 and 4 form k1 and then k2
// from the stage-2 grid.  The same operations on the same operands give the
// same slopes, bit for bit.
template <int MODE, int SH, bool NT, int RK>
__global__ void __launch_bounds__(MAX_WAVES * TILE)
stage1d_kernel(const WorkItem *__restrict__ work, const SimDesc *__restrict__ sims, int max_dpw)
{
    constexpr int GTC = gt_cells(SH), GTS = gt_stride(SH), NE = n_edges(SH);
    // stage-1 grid tile of the recomputing stages: one more cell on each
    // side, since a particle moves up to two cells between the stage-1
    // position and the next step's (dt/2 max|v| < dz)
    constexpr bool G1 = (RK >= 1 && (MODE == M_S2 || MODE == M_S4)) || (RK >= 2 && MODE == M_S3);
    constexpr bool G2 = RK >= 2 && (MODE == M_S3 || MODE == M_S4);
    constexpr int GTC1 = gt_cells(SH + 1), GTS1 = gt_stride(SH + 1);
    extern __shared__ double smem[];
    const WorkItem wi = work[blockIdx.x];
    // private copy: the kernel's stores cannot alias the descriptor
    const SimDesc S = sims[wi.sim];
    const int lane = threadIdx.x & (TILE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / TILE);
    const int nwaves = blockDim.x / TILE;
    const int nc = S.ncell;
    const int64_t np = S.np;
    const int tile0 = wi.tile * TILE;
    const int m = tile0 + lane;
    const bool active = m < nc;
    const int nact = min(TILE, nc - tile0);
    const int64_t n = *S.step;
    const double dt = S.dt, dz = S.dz;

    // stage times of the current (gathered) and next (deposited) positions
    double t_cur = 0.0, t_nxt;
    if (MODE == M_S1) {
        t_cur = stage_time(n, dt, 0.0);
        t_nxt = stage_time(n, dt, 0.5);
    } else if (MODE == M_S2) {
        t_cur = stage_time(n, dt, 0.5);
        t_nxt = stage_time(n, dt, 0.5);
    } else if (MODE == M_S3) {
        t_cur = stage_time(n, dt, 0.5);
        t_nxt = stage_time(n, dt, 1.0);
    } else if (MODE == M_S4) {
        t_cur = stage_time(n, dt, 1.0);
        t_nxt = stage_time(n + 1, dt, 0.0);
    } else {
        t_nxt = stage_time(n, dt, 0.0);
    }

    // LDS: [grid tile | reduction] [edge buffers] [per-direction shifts]
    const int gslot = max(NG * GTS, NG * TILE + nwaves * NG * NE);
    double *Gt = smem;                                        // [NG][GTS]
    double *eb = smem + gslot + wave * max_dpw * 9 * NE;      // [dpw][NE][9] of this wave
    double *tphi = smem + gslot + nwaves * max_dpw * 9 * NE;  // [dpg][2]: phi_cur, phi_nxt
    int *tint = (int *)(tphi + 2 * nwaves * max_dpw);         // [dpg][2]: r, delta
    double *G1t = (double *)(tint + 2 * nwaves * max_dpw);    // [NG][GTS1], G1 only
    double *G2t = G1t + (G1 ? NG * GTS1 : 0);                 // [NG][GTS1], G2 only
    const double t1 = stage_time(n, dt, 0.0);                 // stage-1 time
    const double t2 = stage_time(n, dt, 0.5);                 // stage-2 time

    const int dgrp0 = wi.group * S.dpg;
    // shifts of the workgroup's directions, one thread per direction
    for (int j = threadIdx.x; j < S.dpg; j += blockDim.x) {
        const int d = dgrp0 + j;
        if (d < S.ndir) {
            const double vz = tld(S.vz, d);
            const Shift sn = shift_of(vz, t_nxt, dz);
            const Shift sc = shift_of(vz, t_cur, dz);
            tphi[2 * j + 0] = sc.phi;
            tphi[2 * j + 1] = sn.phi;
            tint[2 * j + 0] = pmod_dbl((double)sn.i, nc);
            tint[2 * j + 1] = max(-1, min(1, (int)(sn.i - sc.i)));
        }
    }
    if (MODE <= M_S4) {
        const double *Gin = S.G[MODE - 1];
        for (int idx = threadIdx.x; idx < NG * GTC; idx += blockDim.x) {
            const int comp = idx / GTC;
            const int k = idx - comp * GTC;
            int cell = tile0 - SH + k;
            if (nc < GTC) {
                cell %= nc;
                cell = (cell < 0) ? cell + nc : cell;
            } else {
                cell = (cell < 0) ? cell + nc : (cell >= nc ? cell - nc : cell);
            }
            Gt[comp * GTS + k] = gld(Gin + (size_t)comp * nc + cell);
        }
    }
    // earlier stages' grid tiles, one more cell on each side
    auto stage_tile = [&](const double *Gin, double *Gdst) {
        for (int idx = threadIdx.x; idx < NG * GTC1; idx += blockDim.x) {
            const int comp = idx / GTC1;
            const int k = idx - comp * GTC1;
            int cell = tile0 - SH - 1 + k;
            if (nc < GTC1) {
                cell %= nc;
                cell = (cell < 0) ? cell + nc : cell;
            } else {
                cell = (cell < 0) ? cell + nc : (cell >= nc ? cell - nc : cell);
            }
            Gdst[comp * GTS1 + k] = gld(Gin + (size_t)comp * nc + cell);
        }
    };
    if (G1)
        stage_tile(S.G[0], G1t);
    if (G2)
        stage_tile(S.G[1], G2t);
    __syncthreads();

    double hv[9], hvb[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        hv[k] = S.hvac[k];
        hvb[k] = S.hvacb[k];
    }

    double acc[NG];
#pragma unroll
    for (int k = 0; k < NG; k++)
        acc[k] = 0.0;

    const int dbeg = dgrp0 + wave * S.dpw;
    const int dend = min(dbeg + S.dpw, S.ndir);

    for (int d = dbeg; d < dend; ++d) {
        const int j = d - dgrp0;
        const double vx = tld(S.vx, d), vy = tld(S.vy, d), vz = tld(S.vz, d);
        const double wN = tld(S.wN, d), wNb = tld(S.wNb, d);
        const double ph = tphi[2 * j + 1];
        const int r = tint[2 * j + 0];
        int c = m - r;
        if (c < 0)
            c += nc;
        const int64_t p = (int64_t)d * nc + c;

        double X[9];
        if (active) {
            double Y[18];
#pragma unroll
            for (int k = 0; k < 18; k++)
                Y[k] = gld(S.Y + k * np + p);
            if (MODE == M_DEPOSIT) {
#pragma unroll
                for (int k = 0; k < 9; k++)
                    X[k] = source_comp(k, wN, Y[k], wNb, Y[9 + k]);
            } else if (MODE == M_MOM_NU) {
#pragma unroll
                for (int k = 0; k < 9; k++)
                    X[k] = wN * Y[k];
            } else if (MODE == M_MOM_NUBAR) {
#pragma unroll
                for (int k = 0; k < 9; k++)
                    X[k] = wNb * Y[9 + k];
            } else {
                // interpolate the staged grid at the current position
                const int kl = lane - tint[2 * j + 1] + SH;  // LDS column of cell m - delta
                const double phi = tphi[2 * j + 0];
                // (where k2 is formed again, after it: fewer live registers)
                double Hnn[9];
                if (!G2)
                    gather_hnn<SH>(Gt, GTS, kl, phi, vx, vy, vz, Hnn);
                // k1 of the RK stages, from the stage-1 grid at the stage-1
                // position (the same gather and commutators as stage 1)
                auto stage1_slope = [&](double k1[18]) {
                    const Shift s1 = shift_of(vz, t1, dz);
                    const Shift sn = shift_of(vz, t_nxt, dz);
                    const int dl = max(-2, min(2, (int)(sn.i - s1.i)));
                    double H1[9];
                    gather_hnn<SH>(G1t, GTS1, lane - dl + SH + 1, s1.phi, vx, vy, vz, H1);
                    slope_of(hv, hvb, H1, Y, k1);
                };
                // k2 of the RK = 2 stages, from k1, the stage-2 grid and the
                // stage-2 position (the same stage state and gather as stage 2)
                auto stage2_slope = [&](const double k1[18], double k2[18]) {
                    const Shift s2 = shift_of(vz, t2, dz);
                    const Shift sn = shift_of(vz, t_nxt, dz);
                    const int dl = max(-2, min(2, (int)(sn.i - s2.i)));
                    const double a = 0.5 * dt;
                    double y2[18];
#pragma unroll
                    for (int k = 0; k < 18; k++)
                        y2[k] = __builtin_fma(a, k1[k], Y[k]);
                    double H2[9];
                    gather_hnn<SH>(G2t, GTS1, lane - dl + SH + 1, s2.phi, vx, vy, vz, H2);
                    slope_of(hv, hvb, H2, y2, k2);
                };
                // stage state y, and the base the next state is built on:
                // Y for stages 1-3, Y + dt/6 (k1 + 2 k2 + 2 k3) for stage 4
                // (the slopes are consumed before the commutators)
                double y[18], base[18];
                if (MODE == M_S1) {
#pragma unroll
                    for (int k = 0; k < 18; k++)
                        y[k] = base[k] = Y[k];
                } else if (MODE == M_S4) {
                    // last reads of the three slopes
                    const double h6 = dt / 6.0;
                    if (G2) {
                        // k1 + 2 k2 as soon as k2 exists (the same sums)
                        double k12[18], k3[18];
                        {
                            double k1[18], k2[18];
                            stage1_slope(k1);
                            stage2_slope(k1, k2);
#pragma unroll
                            for (int k = 0; k < 18; k++)
                                k12[k] = k1[k] + 2.0 * k2[k];
                        }
                        load_slope<NT>(S.K3, np, p, k3);
#pragma unroll
                        for (int k = 0; k < 18; k++) {
                            y[k] = __builtin_fma(dt, k3[k], Y[k]);
                            const double ks = k12[k] + 2.0 * k3[k];
                            base[k] = __builtin_fma(h6, ks, Y[k]);
                        }
                    } else {
                        double k1[18], k2[18], k3[18];
                        if (G1)
                            stage1_slope(k1);
                        else
                            load_slope<NT>(S.K1, np, p, k1);
                        load_slope<NT>(S.K2, np, p, k2);
                        load_slope<NT>(S.K3, np, p, k3);
#pragma unroll
                        for (int k = 0; k < 18; k++) {
                            y[k] = __builtin_fma(dt, k3[k], Y[k]);
                            const double ks = (k1[k] + 2.0 * k2[k]) + 2.0 * k3[k];
                            base[k] = __builtin_fma(h6, ks, Y[k]);
                        }
                    }
                } else {
                    const double a = 0.5 * dt;
                    double kp[18];
                    if (MODE == M_S2 && G1) {
                        stage1_slope(kp);
                    } else if (MODE == M_S3 && G2) {
                        double k1[18];
                        stage1_slope(k1);
                        stage2_slope(k1, kp);
                    } else {
                        load_slope((MODE == M_S2) ? S.K1 : S.K2, np, p, kp);
                    }
                    // one fused multiply-add, as where k2 is formed again
#pragma unroll
                    for (int k = 0; k < 18; k++) {
                        y[k] = __builtin_fma(a, kp[k], Y[k]);
                        base[k] = Y[k];
                    }
                }
                if (G2)
                    gather_hnn<SH>(Gt, GTS, kl, phi, vx, vy, vz, Hnn);
                // Hamiltonians and slopes, through the same helper as the
                // k1 and k2 of the RK stages (one code path, one rounding)
                double kk[18];
                slope_of(hv, hvb, Hnn, y, kk);
                double yn[18];
                if (MODE == M_S4) {
                    const double h6 = dt / 6.0;
                    // (the new state keeps the default policy: the next
                    // step's first stage reads it straight back)
#pragma unroll
                    for (int k = 0; k < 18; k++) {
                        yn[k] = __builtin_fma(h6, kk[k], base[k]);
                        gst(S.Yout + k * np + p, yn[k]);
                    }
                } else {
                    double *Ko = (MODE == M_S1) ? S.K1 : (MODE == M_S2) ? S.K2 : S.K3;
                    const double an = (MODE == M_S3) ? dt : 0.5 * dt;
                    // with streaming, k2 streams; k1 and k3, read again by
                    // the very next kernel, stay cached (measured on the
                    // 2048-cell, 378-direction box)
                    if (!(RK >= 1 && MODE == M_S1) && !(RK >= 2 && MODE == M_S2))
                        store_slope<NT && MODE == M_S2>(Ko, np, p, kk);
#pragma unroll
                    for (int k = 0; k < 18; k++)
                        yn[k] = __builtin_fma(an, kk[k], base[k]);
                }
#pragma unroll
                for (int k = 0; k < 9; k++)
                    X[k] = source_comp(k, wN, yn[k], wNb, yn[9 + k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 9; k++)
                X[k] = 0.0;
        }

        if (SH == 2) {
            // quadratic deposit with the next-stage weights: the particle at
            // anchor m feeds cells m - 1 + up' .. m + 1 + up', so cell m
            // takes w0' w1' w2' of lanes (m + 1, m, m - 1) when up' = 0 and
            // of lanes (m, m - 1, m - 2) when up' = 1 (one-lane DPP moves);
            // what leaves the tile goes to the edge partials: one cell on
            // the left (lane 0), two on the right (the last active lanes)
            const Quad q = quad_weights(ph);
#pragma unroll
            for (int k = 0; k < 9; k++) {
                const double x = X[k];
                double s1 = lane_below(x);
                s1 = (lane == 0) ? 0.0 : s1;
                double a, b, c;
                if (q.up) {
                    double s2 = lane_below(s1);
                    s2 = (lane == 0) ? 0.0 : s2;
                    a = x;
                    b = s1;
                    c = s2;
                } else {
                    double xa = lane_above(x);
                    xa = (lane == TILE - 1) ? 0.0 : xa;
                    a = xa;
                    b = x;
                    c = s1;
                }
                const double xc = wsum3(q.w0, a, q.w1, b, q.w2, c);
                acc[k] += xc;
                acc[9 + k] += vx * xc;
                acc[18 + k] += vy * xc;
                acc[27 + k] += vz * xc;
                if (lane == nact - 1) {
                    eb[((d - dbeg) * NE + 0) * 9 + k] = q.up ? wsum2(q.w1, x, q.w2, s1) : q.w2 * x;
                    eb[((d - dbeg) * NE + 1) * 9 + k] = q.up ? q.w2 * x : 0.0;
                }
                if (lane == 0)
                    eb[((d - dbeg) * NE + 2) * 9 + k] = q.up ? 0.0 : q.w0 * x;
            }
        } else {
            // deposit with the next-stage weights: cell m gets (1 - phi') of
            // its own particle and phi' of the particle one lane to the left
            const double omph = 1.0 - ph;
#pragma unroll
            for (int k = 0; k < 9; k++) {
                double xl = lane_below(X[k]);
                xl = (lane == 0) ? 0.0 : xl;
                const double xc = wsum2(omph, X[k], ph, xl);
                acc[k] += xc;
                acc[9 + k] += vx * xc;
                acc[18 + k] += vy * xc;
                acc[27 + k] += vz * xc;
            }
            if (lane == nact - 1) {
#pragma unroll
                for (int k = 0; k < 9; k++)
                    eb[(d - dbeg) * 9 + k] = ph * X[k];
            }
        }
    }

    // ---- workgroup reduction (fixed order over waves) -----------------
    __syncthreads();  // the grid tile is no longer needed: reuse it
    double *redb = smem;  // [NG][TILE]
    for (int w = 0; w < nwaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < NG; k++)
                redb[k * TILE + lane] = (w == 0) ? acc[k] : redb[k * TILE + lane] + acc[k];
        }
        __syncthreads();
    }
    // edge partials of each wave: one lane per (edge, moment component)
    // sums over the wave's directions
    double *esum = smem + NG * TILE;  // [nwaves][NE][NG]
    for (int q = lane; q < NE * NG; q += TILE) {
        const int e = q / NG, r = q - e * NG;
        const int comp = r % 9, grp = r / 9;
        double s = 0.0;
        for (int d = dbeg; d < dend; ++d) {
            const double coef = (grp == 0) ? 1.0 : (grp == 1) ? tld(S.vx, d) : (grp == 2) ? tld(S.vy, d) : tld(S.vz, d);
            s += coef * eb[((d - dbeg) * NE + e) * 9 + comp];
        }
        esum[(wave * NE + e) * NG + r] = s;
    }
    __syncthreads();

    const int ntc = S.ntile * TILE;
    double *part = S.part + (size_t)wi.group * NG * ntc;
    for (int idx = threadIdx.x; idx < NG * TILE; idx += blockDim.x) {
        const int k = idx / TILE, l = idx - k * TILE;
        gst(part + (size_t)k * ntc + tile0 + l, redb[idx]);
    }
    for (int q = threadIdx.x; q < NE * NG; q += blockDim.x) {
        const int e = q / NG, r = q - e * NG;
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w)
            s += esum[(w * NE + e) * NG + r];
        gst(S.edge + (((size_t)wi.group * NG + r) * NE + e) * S.ntile + wi.tile, s);
    }
}

// ---------------------------------------------------------------------------
// Reverse mode of one Runge-Kutta stage (hand-written adjoint).
//
// For stage s with slope k_s = F(t_s, y_s), given g_s = dL/dk_s, the stage
// adjoint dL/dy_s = F_y^T g_s and the weight gradients F_w^T g_s are
//   per particle:   G = g with halved off-diagonals (packed cotangent ->
//                   Hermitian matrix), direct part D = -i[G, H] (off-
//                   diagonals doubled back), dH = -i[rho, G];
//                   the same with (Hbar, rhobar); the source
//                   S = dH - conj-sign * dHbar (cotangent of H_nunu),
//   deposit:        Gamma_A = sum_p w S_p, Gamma_B = -sum_p w Omega_p S_p
//                   (the transpose of the interpolation, same weights),
//   gather:         dX = Gamma_A + Omega . Gamma_B (the transpose of the
//                   deposition), dL/drho = D + (N/dV) dX,
//                   dL/drhobar = Dbar - conj-sign (Nbar/dV) dX,
//                   dL/d(N/dV) += rho . dX, dL/d(Nbar/dV) -= rhobar . dX.
// Phase 0 forms g_s from the step's lambda and the previous stage's lambda,
// writes D and deposits S; phase 1 gathers Gamma, writes the stage lambda
// and accumulates the step's lambda and the weight gradients.  Both phases
// place particles at t_s (the same weights as the forward pass).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, TILE);
    return v;
}

// One launch covers the second half of stage SB's adjoint (DO_B: gather the
// deposited sources, stage lambda, step lambda and weight gradients) and the
// first half of stage SA = SB - 1 (DO_A: g_SA from the step lambda and the
// stage lambda just formed, direct part, sources and their deposit), for the
// same particle in the same lane.  Lanes are anchored at the deposit time
// t_SA (at t_SB when only DO_B); the sources of stage SB are gathered at
// t_SB, which lies at most one cell away (offset delta), as in the forward
// stage kernels.
__device__ __forceinline__ double stage_c(int s) { return s == 1 ? 0.0 : (s == 4 ? 1.0 : 0.5); }

template <bool DO_B, bool DO_A, int SB, int SA, int SH>
__global__ void __launch_bounds__(MAX_WAVES * TILE)
adj1d_kernel(const WorkItem *__restrict__ work, const SimDesc *__restrict__ sims, int max_dpw)
{
    constexpr int GTC = gt_cells(SH), GTS = gt_stride(SH), NE = n_edges(SH);
    extern __shared__ double smem[];
    const WorkItem wi = work[blockIdx.x];
    const SimDesc S = sims[wi.sim];
    const int lane = threadIdx.x & (TILE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / TILE);
    const int nwaves = blockDim.x / TILE;
    const int nc = S.ncell;
    const int64_t np = S.np;
    const int tile0 = wi.tile * TILE;
    const int m = tile0 + lane;
    const bool active = m < nc;
    const int nact = min(TILE, nc - tile0);
    const int64_t n = *S.step;
    const double dt = S.dt, dz = S.dz;
    const double tA = DO_A ? stage_time(n, dt, stage_c(SA)) : 0.0;
    const double tB = DO_B ? stage_time(n, dt, stage_c(SB)) : 0.0;
    const double tanc = DO_A ? tA : tB;

    // LDS: [Gamma tile | reduction] [stage-SA grid tile] [edge buffers]
    //      [phi_anchor, phi_B per direction] [r, delta per direction]
    const int gslot = max(NG * GTS, NG * TILE + nwaves * NG * NE);
    double *GtB = smem;
    double *GtA = smem + gslot;
    double *eb = smem + 2 * gslot + wave * max_dpw * 9 * NE;
    double *tphi = smem + 2 * gslot + nwaves * max_dpw * 9 * NE;
    int *tint = (int *)(tphi + 2 * nwaves * max_dpw);

    const int dgrp0 = wi.group * S.dpg;
    for (int j = threadIdx.x; j < S.dpg; j += blockDim.x) {
        const int d = dgrp0 + j;
        if (d < S.ndir) {
            const Shift sa = shift_of(tld(S.vz, d), tanc, dz);
            tphi[2 * j + 0] = sa.phi;
            tint[2 * j + 0] = pmod_dbl((double)sa.i, nc);
            if (DO_A && DO_B) {
                const Shift sb = shift_of(tld(S.vz, d), tB, dz);
                tphi[2 * j + 1] = sb.phi;
                tint[2 * j + 1] = max(-1, min(1, (int)(sa.i - sb.i)));
            } else {
                tphi[2 * j + 1] = sa.phi;
                tint[2 * j + 1] = 0;
            }
        }
    }
    for (int idx = threadIdx.x; idx < NG * GTC; idx += blockDim.x) {
        const int comp = idx / GTC;
        const int k = idx - comp * GTC;
        int cell = tile0 - SH + k;
        if (nc < GTC) {
            cell %= nc;
            cell = (cell < 0) ? cell + nc : cell;
        } else {
            cell = (cell < 0) ? cell + nc : (cell >= nc ? cell - nc : cell);
        }
        const size_t at = (size_t)comp * nc + cell;
        if (DO_B)
            GtB[comp * GTS + k] = gld(S.GA + at);
        if (DO_A)
            GtA[comp * GTS + k] = gld(S.G[SA - 1] + at);
    }
    __syncthreads();

    double hv[9], hvb[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        hv[k] = S.hvac[k];
        hvb[k] = S.hvacb[k];
    }
    double acc[NG];
#pragma unroll
    for (int k = 0; k < NG; k++)
        acc[k] = 0.0;

    // (selects, not a run-time index into the descriptor copy, which would
    // put the whole copy in scratch memory)
    const double *lam_in = (n & 1) ? S.lam[0] : S.lam[1];
    double *lam_out = (n & 1) ? S.lam[1] : S.lam[0];
    const double *KB = (SB == 2) ? S.K1 : (SB == 3) ? S.K2 : S.K3;
    const double aB = (SB == 4) ? dt : 0.5 * dt;
    const double *KA = (SA == 2) ? S.K1 : (SA == 3) ? S.K2 : S.K3;
    const double aA = (SA == 4) ? dt : 0.5 * dt;

    const int dbeg = dgrp0 + wave * S.dpw;
    const int dend = min(dbeg + S.dpw, S.ndir);
    for (int d = dbeg; d < dend; ++d) {
        const int j = d - dgrp0;
        const double vx = tld(S.vx, d), vy = tld(S.vy, d), vz = tld(S.vz, d);
        const double wN = tld(S.wN, d), wNb = tld(S.wNb, d);
        const double phA = tphi[2 * j + 0], omA = 1.0 - phA;
        int c = m - tint[2 * j + 0];
        if (c < 0)
            c += nc;
        const int64_t p = (int64_t)d * nc + c;

        double Yv[18];
#pragma unroll
        for (int k = 0; k < 18; k++)
            Yv[k] = active ? gld(S.Y + k * np + p) : 0.0;

        double lam_s[18];
        double sN = 0.0, sNb = 0.0;
        if (DO_B) {
            // gather the deposited sources at t_SB: dX = Gamma_A + Omega.Gamma_B
            const int kl = lane - tint[2 * j + 1] + SH;
            const double phB = tphi[2 * j + 1], omB = 1.0 - phB;
            double dX[9];
            if (SH == 2) {
                const Quad q = quad_weights(phB);
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double *g = GtB + k * GTS + kl - 1 + q.up;
                    const double A = (q.w0 * g[0] + q.w1 * g[1]) + q.w2 * g[2];
                    const double Bx = (q.w0 * g[9 * GTS] + q.w1 * g[9 * GTS + 1]) + q.w2 * g[9 * GTS + 2];
                    const double By = (q.w0 * g[18 * GTS] + q.w1 * g[18 * GTS + 1]) + q.w2 * g[18 * GTS + 2];
                    const double Bz = (q.w0 * g[27 * GTS] + q.w1 * g[27 * GTS + 1]) + q.w2 * g[27 * GTS + 2];
                    dX[k] = A + (vx * Bx + vy * By + vz * Bz);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double *g = GtB + k * GTS + kl;
                    const double A = omB * g[0] + phB * g[1];
                    const double Bx = omB * g[9 * GTS] + phB * g[9 * GTS + 1];
                    const double By = omB * g[18 * GTS] + phB * g[18 * GTS + 1];
                    const double Bz = omB * g[27 * GTS] + phB * g[27 * GTS + 1];
                    dX[k] = A + (vx * Bx + vy * By + vz * Bz);
                }
            }
            if (active) {
                double kb1 = 0.0, kb2 = 0.0, kb10 = 0.0, kb11 = 0.0;
                if (SB != 1) {
                    kb1 = gld(KB + kslot(1) * np + p);
                    kb2 = gld(KB + kslot(2) * np + p);
                    kb10 = gld(KB + kslot(10) * np + p);
                    kb11 = gld(KB + kslot(11) * np + p);
                }
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double sgn = (k == 4 || k == 6 || k == 8) ? -1.0 : 1.0;
                    double kbn = 0.0, kbb = 0.0;
                    if (SB != 1) {
                        kbn = (k == 0) ? -(kb1 + kb2) : (k == 1) ? kb1 : (k == 2) ? kb2 : gld(KB + kslot(k) * np + p);
                        kbb = (k == 0) ? -(kb10 + kb11) : (k == 1) ? kb10 : (k == 2) ? kb11
                                                                         : gld(KB + kslot(9 + k) * np + p);
                    }
                    const double yb = (SB == 1) ? Yv[k] : Yv[k] + aB * kbn;
                    const double ybb = (SB == 1) ? Yv[9 + k] : Yv[9 + k] + aB * kbb;
                    lam_s[k] = gld(S.dres + k * np + p) + wN * dX[k];
                    lam_s[9 + k] = gld(S.dres + (9 + k) * np + p) - sgn * wNb * dX[k];
                    const double base_n = (SB == 4) ? gld(lam_in + k * np + p) : gld(lam_out + k * np + p);
                    const double base_b = (SB == 4) ? gld(lam_in + (9 + k) * np + p)
                                                    : gld(lam_out + (9 + k) * np + p);
                    gst(lam_out + k * np + p, base_n + lam_s[k]);
                    gst(lam_out + (9 + k) * np + p, base_b + lam_s[9 + k]);
                    sN += yb * dX[k];
                    sNb -= sgn * ybb * dX[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 18; k++)
                    lam_s[k] = 0.0;
            }
            sN = wave_sum(sN);
            sNb = wave_sum(sNb);
            if (lane == 0) {
                const size_t at = (size_t)d * S.ntile + wi.tile;
                gst(S.dwN + at, gld(S.dwN + at) + sN);
                gst(S.dwNb + at, gld(S.dwNb + at) + sNb);
            }
        }

        if (DO_A) {
            double X[9];
            // interpolate the stage-SA grid at t_SA (the anchor time)
            double Hnn[9];
            if (SH == 2) {
                const Quad q = quad_weights(phA);
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double *g = GtA + k * GTS + lane + 1 + q.up;
                    const double A = (q.w0 * g[0] + q.w1 * g[1]) + q.w2 * g[2];
                    const double Bx = (q.w0 * g[9 * GTS] + q.w1 * g[9 * GTS + 1]) + q.w2 * g[9 * GTS + 2];
                    const double By = (q.w0 * g[18 * GTS] + q.w1 * g[18 * GTS + 1]) + q.w2 * g[18 * GTS + 2];
                    const double Bz = (q.w0 * g[27 * GTS] + q.w1 * g[27 * GTS + 1]) + q.w2 * g[27 * GTS + 2];
                    Hnn[k] = A - (vx * Bx + vy * By + vz * Bz);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double *g = GtA + k * GTS + lane + 1;
                    const double A = omA * g[0] + phA * g[1];
                    const double Bx = omA * g[9 * GTS] + phA * g[9 * GTS + 1];
                    const double By = omA * g[18 * GTS] + phA * g[18 * GTS + 1];
                    const double Bz = omA * g[27 * GTS] + phA * g[27 * GTS + 1];
                    Hnn[k] = A - (vx * Bx + vy * By + vz * Bz);
                }
            }
            if (active) {
                const double c1 = (SA == 1 || SA == 4) ? dt / 6.0 : dt / 3.0;
                const double c2 = (SA == 3) ? dt : 0.5 * dt;
                // neutrinos, then antineutrinos
#pragma unroll
                for (int part = 0; part < 2; part++) {
                    const int o = 9 * part;
                    double G[9], y[9], H[9];
                    double ka1 = 0.0, ka2 = 0.0;
                    if (SA != 1) {
                        ka1 = gld(KA + kslot(o + 1) * np + p);
                        ka2 = gld(KA + kslot(o + 2) * np + p);
                    }
#pragma unroll
                    for (int k = 0; k < 9; k++) {
                        double gk = c1 * gld(lam_in + (o + k) * np + p);
                        if (DO_B)
                            gk += c2 * lam_s[o + k];
                        G[k] = (k >= 3) ? 0.5 * gk : gk;
                        double ka = 0.0;
                        if (SA != 1)
                            ka = (k == 0) ? -(ka1 + ka2) : (k == 1) ? ka1 : (k == 2) ? ka2
                                                                     : gld(KA + kslot(o + k) * np + p);
                        y[k] = (SA == 1) ? Yv[o + k] : Yv[o + k] + aA * ka;
                        const double hk = part == 0 ? hv[k] + Hnn[k] : hvb[k] - Hnn[k];
                        H[k] = (part == 1 && (k == 4 || k == 6 || k == 8)) ? -hk : hk;
                    }
                    double Dk[9], dH[9];
                    commutator(G, H, Dk);
                    commutator(y, G, dH);
#pragma unroll
                    for (int k = 0; k < 9; k++) {
                        const double f = (k >= 3) ? 2.0 : 1.0;
                        gst(S.dres + (o + k) * np + p, f * Dk[k]);
                        const double sgn = (k == 4 || k == 6 || k == 8) ? -1.0 : 1.0;
                        // source: dH for neutrinos minus conj-sign * dHbar
                        X[k] = (part == 0) ? f * dH[k] : X[k] - sgn * f * dH[k];
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 9; k++)
                    X[k] = 0.0;
            }
            if (SH == 2) {
                // quadratic deposit at t_SA, as in the stage kernels
                const Quad q = quad_weights(phA);
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const double x = X[k];
                    double s1 = lane_below(x);
                    s1 = (lane == 0) ? 0.0 : s1;
                    double a, b, cc;
                    if (q.up) {
                        double s2 = lane_below(s1);
                        s2 = (lane == 0) ? 0.0 : s2;
                        a = x;
                        b = s1;
                        cc = s2;
                    } else {
                        double xa = lane_above(x);
                        xa = (lane == TILE - 1) ? 0.0 : xa;
                        a = xa;
                        b = x;
                        cc = s1;
                    }
                    const double xc = (q.w0 * a + q.w1 * b) + q.w2 * cc;
                    acc[k] += xc;
                    acc[9 + k] -= vx * xc;
                    acc[18 + k] -= vy * xc;
                    acc[27 + k] -= vz * xc;
                    if (lane == nact - 1) {
                        eb[((d - dbeg) * NE + 0) * 9 + k] = q.up ? q.w1 * x + q.w2 * s1 : q.w2 * x;
                        eb[((d - dbeg) * NE + 1) * 9 + k] = q.up ? q.w2 * x : 0.0;
                    }
                    if (lane == 0)
                        eb[((d - dbeg) * NE + 2) * 9 + k] = q.up ? 0.0 : q.w0 * x;
                }
            } else {
                // deposit the sources at t_SA: cell m gets (1 - phi) of its
                // own particle and phi of the particle one lane to the left
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    double xl = lane_below(X[k]);
                    xl = (lane == 0) ? 0.0 : xl;
                    const double xc = omA * X[k] + phA * xl;
                    acc[k] += xc;
                    acc[9 + k] -= vx * xc;
                    acc[18 + k] -= vy * xc;
                    acc[27 + k] -= vz * xc;
                }
                if (lane == nact - 1) {
#pragma unroll
                    for (int k = 0; k < 9; k++)
                        eb[(d - dbeg) * 9 + k] = phA * X[k];
                }
            }
        }
    }
    if (!DO_A)
        return;

    // ---- workgroup reduction of the deposited sources (as in the stages)
    __syncthreads();
    double *redb = smem;
    for (int w = 0; w < nwaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < NG; k++)
                redb[k * TILE + lane] = (w == 0) ? acc[k] : redb[k * TILE + lane] + acc[k];
        }
        __syncthreads();
    }
    double *esum = smem + NG * TILE;  // [nwaves][NE][NG]
    for (int q = lane; q < NE * NG; q += TILE) {
        const int e = q / NG, r = q - e * NG;
        const int comp = r % 9, grp = r / 9;
        double sacc = 0.0;
        for (int d = dbeg; d < dend; ++d) {
            const double coef = (grp == 0) ? 1.0 : (grp == 1) ? -tld(S.vx, d) : (grp == 2) ? -tld(S.vy, d) : -tld(S.vz, d);
            sacc += coef * eb[((d - dbeg) * NE + e) * 9 + comp];
        }
        esum[(wave * NE + e) * NG + r] = sacc;
    }
    __syncthreads();
    const int ntc = S.ntile * TILE;
    double *part = S.part + (size_t)wi.group * NG * ntc;
    for (int idx = threadIdx.x; idx < NG * TILE; idx += blockDim.x) {
        const int k = idx / TILE, l = idx - k * TILE;
        gst(part + (size_t)k * ntc + tile0 + l, redb[idx]);
    }
    for (int q = threadIdx.x; q < NE * NG; q += blockDim.x) {
        const int e = q / NG, r = q - e * NG;
        double sacc = 0.0;
        for (int w = 0; w < nwaves; ++w)
            sacc += esum[(w * NE + e) * NG + r];
        gst(S.edge + (((size_t)wi.group * NG + r) * NE + e) * S.ntile + wi.tile, sacc);
    }
}

__global__ void fill_kernel(double *p, size_t n, double v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

// Sum the direction-group partials of one tile in a fixed order and close
// the periodic box: cell tile*64 also receives the right-edge partial of
// the previous tile (cell 0 that of the last tile).  Block (item, q) handles
// components 4q .. 4q+3 of the item's 64 cells, one thread per value.
__global__ void __launch_bounds__(256)
reduce1d_kernel(const RedItem *__restrict__ items, const SimDesc *__restrict__ sims, int which,
                double *override_out, int tick)
{
    const RedItem it = items[blockIdx.x];
    const SimDesc &S = sims[it.sim];
    const int nc = S.ncell, ntile = S.ntile, ntc = ntile * TILE;
    const int tile0 = it.tile * TILE;
    const int nact = min(TILE, nc - tile0);
    double *out = (which <= 4) ? S.G[which] : (which == RED_GA) ? S.GA : override_out;
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & (TILE - 1);
    if (l < nact) {
        const int ng = S.ngroup;
        const double *pp = S.part + (size_t)k * ntc + tile0 + l;
        const size_t gstride = (size_t)NG * ntc;
        // loads in flight together, sums in group order
        double s = 0.0;
        int g = 0;
        for (; g + 8 <= ng; g += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = gld(pp + (size_t)(g + q) * gstride);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                s += v[q];
        }
        for (; g < ng; ++g)
            s += gld(pp + (size_t)g * gstride);
        if (S.shape == 2) {
            // quadratic: a tile's right-edge cells are the first two after
            // it (the second lies two tiles on when the next tile has one
            // cell), its left-edge cell the last before it; with one tile
            // or very few cells they fold onto the tile itself.  Candidate
            // sources in a fixed order: tiles T-2, T-1, T, T+1 (each once).
            const int j = tile0 + l;
            int cand[4] = {(it.tile + 2 * ntile - 2) % ntile, (it.tile + ntile - 1) % ntile, it.tile,
                           (it.tile + 1) % ntile};
            for (int ci = 0; ci < 4; ++ci) {
                const int src = cand[ci];
                bool seen = false;
                for (int cj = 0; cj < ci; ++cj)
                    seen = seen || (cand[cj] == src);
                if (seen)
                    continue;
                const int t0s = src * TILE, nas = min(TILE, nc - t0s);
                for (int e = 0; e < 3; ++e) {
                    const int target = (e < 2) ? (t0s + nas + e) % nc : (t0s + nc - 1) % nc;
                    if (target != j)
                        continue;
                    const double *ep = S.edge + ((size_t)k * 3 + e) * ntile + src;
                    const size_t estride = (size_t)NG * 3 * ntile;
                    int g2 = 0;
                    for (; g2 + 8 <= ng; g2 += 8) {
                        double v[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            v[q] = gld(ep + (size_t)(g2 + q) * estride);
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            s += v[q];
                    }
                    for (; g2 < ng; ++g2)
                        s += gld(ep + (size_t)g2 * estride);
                }
            }
        } else if (l == 0) {
            const int tprev = (it.tile + ntile - 1) % ntile;
            const double *ep = S.edge + (size_t)k * ntile + tprev;
            const size_t estride = (size_t)NG * ntile;
            int g2 = 0;
            for (; g2 + 8 <= ng; g2 += 8) {
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    v[q] = gld(ep + (size_t)(g2 + q) * estride);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    s += v[q];
            }
            for (; g2 < ng; ++g2)
                s += gld(ep + (size_t)g2 * estride);
        }
        out[(size_t)k * nc + tile0 + l] = s;
    }
    if (tick && it.tile == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        *S.step += tick;
}

__global__ void tick_kernel(const SimDesc *sims, int64_t delta)
{
    if (threadIdx.x == 0)
        *sims[0].step += delta;
}

// dst[d] = scale * sum_t src[d * ntile + t], fixed order over tiles
__global__ void tile_sum_kernel(const double *src, int ndir, int ntile, double scale, double *dst)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= ndir)
        return;
    double s = 0.0;
    for (int t = 0; t < ntile; ++t)
        s += src[(size_t)d * ntile + t];
    dst[d] = scale * s;
}

__global__ void set_step_kernel(const SimDesc *sims, int lo, int hi, int64_t value)
{
    const int i = lo + (int)threadIdx.x;
    if (i < hi)
        *sims[i].step = value;
}

// Deterministic two-level sums for diagnostics: block b sums particles
// b, b + nblk*256, ... per thread, then a fixed LDS tree.
__global__ void __launch_bounds__(256)
totals_kernel(const SimDesc *sims, int sim, double *partial)
{
    const SimDesc &S = sims[sim];
    __shared__ double sh[256];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < 18; ++k) {
        double s = 0.0;
        for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += stride) {
            const int d = (int)(p / S.ncell);
            const double w = (k < 9) ? tld(S.Nw, d) : tld(S.Nbw, d);
            s += w * S.Y[k * S.np + p];
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h)
                sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            partial[(size_t)blockIdx.x * 18 + k] = sh[0];
        __syncthreads();
    }
}

__global__ void sum_blocks_kernel(const double *partial, int nblk, int width, double *out)
{
    const int k = threadIdx.x;
    if (k >= width)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b)
        s += partial[(size_t)b * width + k];
    out[k] = s;
}

// max |Tr rho - 1|, max |Tr rhobar - 1|, count of non-finite entries
__global__ void __launch_bounds__(256)
check_kernel(const SimDesc *sims, int sim, double *partial)
{
    const SimDesc &S = sims[sim];
    __shared__ double sh[3][256];
    double e0 = 0.0, e1 = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += stride) {
        double v[18];
        for (int k = 0; k < 18; ++k) {
            v[k] = S.Y[k * S.np + p];
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
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 3 + 0] = sh[0][0];
        partial[blockIdx.x * 3 + 1] = sh[1][0];
        partial[blockIdx.x * 3 + 2] = sh[2][0];
    }
}

__global__ void check_final_kernel(const double *partial, int nblk, double *out)
{
    if (threadIdx.x != 0)
        return;
    double e0 = 0.0, e1 = 0.0, bad = 0.0;
    for (int b = 0; b < nblk; ++b) {
        e0 = fmax(e0, partial[b * 3 + 0]);
        e1 = fmax(e1, partial[b * 3 + 1]);
        bad += partial[b * 3 + 2];
    }
    out[0] = e0;
    out[1] = e1;
    out[2] = bad;
}

// Electron-flavor state rho = rhobar = diag(1, 0, 0) (autotuning input).
__global__ void fill_state_kernel(const SimDesc *sims, int sim)
{
    const SimDesc &S = sims[sim];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += stride)
        for (int k = 0; k < 18; ++k)
            S.Y[k * S.np + p] = (k == 0 || k == 9) ? 1.0 : 0.0;
}

size_t stage1d_smem_bytes(int waves, int max_dpw, int shape)
{
    const size_t ne = n_edges(shape);
    size_t tile = (size_t)NG * gt_stride(shape);
    size_t red = (size_t)NG * TILE + (size_t)waves * NG * ne;
    size_t gslot = tile > red ? tile : red;
    const size_t dpg = (size_t)waves * max_dpw;
    // grid slot, edge buffers, phi table, (r, delta) table
    return (gslot + dpg * 9 * ne + dpg * 2) * sizeof(double) + dpg * 2 * sizeof(int);
}

template <int SH, bool NT, int RK>
static hipError_t launch_stage1d_sh(int mode, const WorkItem *work, int nwork, const SimDesc *sims,
                                    int waves, int max_dpw, hipStream_t s)
{
    const dim3 grid(nwork), block(waves * TILE);
    size_t smem = stage1d_smem_bytes(waves, max_dpw, SH);
    // staged tiles of earlier stages' grids (k1: stages 2 and 4, and 3 when
    // k2 is formed too; k2: stages 3 and 4)
    const int ntiles = ((RK >= 1 && (mode == M_S2 || mode == M_S4)) || (RK >= 2 && mode == M_S3) ? 1 : 0) +
                       (RK >= 2 && (mode == M_S3 || mode == M_S4) ? 1 : 0);
    smem += sizeof(double) * NG * gt_stride(SH + 1) * ntiles;
    switch (mode) {
    case M_S1: stage1d_kernel<M_S1, SH, NT, RK><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_S2: stage1d_kernel<M_S2, SH, NT, RK><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_S3: stage1d_kernel<M_S3, SH, NT, RK><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_S4: stage1d_kernel<M_S4, SH, NT, RK><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_DEPOSIT: stage1d_kernel<M_DEPOSIT, SH, false, 0><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_MOM_NU: stage1d_kernel<M_MOM_NU, SH, false, 0><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case M_MOM_NUBAR: stage1d_kernel<M_MOM_NUBAR, SH, false, 0><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SH, bool NT>
static hipError_t launch_stage1d_nt(int mode, const WorkItem *work, int nwork, const SimDesc *sims,
                                    int waves, int max_dpw, int rk, hipStream_t s)
{
    if (rk == 2)
        return launch_stage1d_sh<SH, NT, 2>(mode, work, nwork, sims, waves, max_dpw, s);
    if (rk == 1)
        return launch_stage1d_sh<SH, NT, 1>(mode, work, nwork, sims, waves, max_dpw, s);
    return launch_stage1d_sh<SH, NT, 0>(mode, work, nwork, sims, waves, max_dpw, s);
}

hipError_t launch_stage1d(int mode, const WorkItem *work, int nwork, const SimDesc *sims,
                          int waves, int max_dpw, int shape, bool stream_policy, int reform,
                          hipStream_t s)
{
    if (reform < 0 || reform > 2)
        return hipErrorInvalidValue;
    if (shape == 2)
        return stream_policy ? launch_stage1d_nt<2, true>(mode, work, nwork, sims, waves, max_dpw, reform, s)
                             : launch_stage1d_nt<2, false>(mode, work, nwork, sims, waves, max_dpw, reform, s);
    if (shape == 1)
        return stream_policy ? launch_stage1d_nt<1, true>(mode, work, nwork, sims, waves, max_dpw, reform, s)
                             : launch_stage1d_nt<1, false>(mode, work, nwork, sims, waves, max_dpw, reform, s);
    return hipErrorInvalidValue;
}

hipError_t launch_reduce1d(const RedItem *items, int nitems, const SimDesc *sims, int which,
                           double *override_out, int tick, hipStream_t s)
{
    reduce1d_kernel<<<dim3(nitems, NG / 4), dim3(256), 0, s>>>(items, sims, which, override_out, tick);
    return hipGetLastError();
}

size_t adj1d_smem_bytes(int waves, int max_dpw, int shape)
{
    const size_t ne = n_edges(shape);
    size_t tile = (size_t)NG * gt_stride(shape);
    size_t red = (size_t)NG * TILE + (size_t)waves * NG * ne;
    size_t gslot = tile > red ? tile : red;
    const size_t dpg = (size_t)waves * max_dpw;
    return (2 * gslot + dpg * 9 * ne + dpg * 2) * sizeof(double) + dpg * 2 * sizeof(int);
}

// kind 4: stage 4 sources; 3, 2, 1: gather of stage kind+1 fused with the
// sources of stage kind; 0: gather of stage 1
template <int SH>
static hipError_t launch_adj1d_sh(int kind, const WorkItem *work, int nwork, const SimDesc *sims,
                                  int waves, int max_dpw, hipStream_t s)
{
    const dim3 grid(nwork), block(waves * TILE);
    const size_t smem = adj1d_smem_bytes(waves, max_dpw, SH);
    switch (kind) {
    case 4: adj1d_kernel<false, true, 5, 4, SH><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case 3: adj1d_kernel<true, true, 4, 3, SH><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case 2: adj1d_kernel<true, true, 3, 2, SH><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case 1: adj1d_kernel<true, true, 2, 1, SH><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    case 0: adj1d_kernel<true, false, 1, 0, SH><<<grid, block, smem, s>>>(work, sims, max_dpw); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj1d(int kind, const WorkItem *work, int nwork, const SimDesc *sims, int waves,
                        int max_dpw, int shape, hipStream_t s)
{
    if (shape == 2)
        return launch_adj1d_sh<2>(kind, work, nwork, sims, waves, max_dpw, s);
    if (shape == 1)
        return launch_adj1d_sh<1>(kind, work, nwork, sims, waves, max_dpw, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tick(const SimDesc *sims, int64_t delta, hipStream_t s)
{
    tick_kernel<<<1, 64, 0, s>>>(sims, delta);
    return hipGetLastError();
}

hipError_t launch_tile_sum(const double *src, int ndir, int ntile, double scale, double *dst,
                           hipStream_t s)
{
    tile_sum_kernel<<<(ndir + 255) / 256, 256, 0, s>>>(src, ndir, ntile, scale, dst);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s)
{
    fill_kernel<<<512, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_step(const SimDesc *sims, int lo, int hi, int64_t value, hipStream_t s)
{
    const int n = hi - lo;
    set_step_kernel<<<1, n < 1 ? 1 : n, 0, s>>>(sims, lo, hi, value);
    return hipGetLastError();
}

hipError_t launch_totals(const SimDesc *sims, int sim, int nblk, double *out18, hipStream_t s)
{
    // partials live after the 18 outputs in the same scratch area
    double *partial = out18 + 18;
    totals_kernel<<<nblk, 256, 0, s>>>(sims, sim, partial);
    sum_blocks_kernel<<<1, 64, 0, s>>>(partial, nblk, 18, out18);
    return hipGetLastError();
}

hipError_t launch_check(const SimDesc *sims, int sim, int nblk, double *out3, hipStream_t s)
{
    double *partial = out3 + 3;
    check_kernel<<<nblk, 256, 0, s>>>(sims, sim, partial);
    check_final_kernel<<<1, 64, 0, s>>>(partial, nblk, out3);
    return hipGetLastError();
}

hipError_t launch_fill_state(const SimDesc *sims, int sim, hipStream_t s)
{
    fill_state_kernel<<<1024, 256, 0, s>>>(sims, sim);
    return hipGetLastError();
}

}  // namespace fpic
