// 3D periodic boxes: two kernels per Runge-Kutta stage.
//
// particle kernel (a workgroup = one x-row of current cells and a group of
// directions, lane = x): forms the stage state, interpolates the combined
// moments at the particle's current position with the trilinear
// cloud-in-cell weights (y and z first, from the four neighbouring grid rows
// staged in LDS, then x from the lane one to the right), builds H and Hbar,
// the commutator slopes and the next stage state, and writes that state's
// deposit source X = (N/dV) rho - (Nbar/dV) rhobar^* (its traceless part: 8
// reals per particle, see NXT below).
//
// deposit kernel (one wave = one x-row of destination cells, all directions
// in a fixed order; a workgroup holds a small patch of neighbouring rows):
// every cell pulls X from the eight particles whose next-stage positions
// straddle it (four rows in y and z, then the lane one to the left in x)
// with the same weights, and accumulates the combined moments (32 traceless
// components; 36 for the moments diagnostic) in registers.  Each cell is
// written once: no atomics, no partial sums, bitwise reproducible.
//
// Positions are implicit as in 1D: particle (d, c) is at cell c shifted by
// floor(Omega_a t / dx_a) along each axis with fraction Omega_a t / dx_a minus
// that, t = n dt + c_s dt.  Along an axis with one cell the particle stays in
// cell 0 with weight 1.  The x axis of a box must fit one wave (nx <= 64).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fpic_3d.h"
#include "fpic_device.h"
#include "fpic_internal.h"

namespace fpic3d {

using fpic::commutator;
using fpic::fail;
using fpic::gld;
using fpic::gst;
using fpic::stage_time;
using fpic::tld;

constexpr int NG = 36;
constexpr int W = 64;

struct Desc3 {
    int32_t n[3];    // nx, ny, nz
    int32_t ndir;
    int64_t ncell, np;
    double dt, dx[3];
    double hvac[9];         // constant part of H (vacuum + matter), packed
    double hvacb[9];        // of Hbar before conjugation (vacuum - matter)
    const double *v[3];     // [ndir] direction components
    const double *wN, *wNb; // [ndir] N/dV, Nbar/dV
    const double *Nw, *Nbw; // [ndir] N, Nbar
    double *Y, *K1, *K2, *K3;
    double *X;              // [9][ndir][ncell] deposit sources (stages: 8 traceless)
    double *G[2];           // [36][ncell] (stages: 32 traceless): stage s reads G[(s-1)&1]
    int64_t *step;
    int32_t shape;          // shape-function order: 1 linear, 2 quadratic
    int32_t pad_;
};

// integer shift (mod n) and fraction along one axis; one-cell axes: (0, 0)
__device__ __forceinline__ void axis_shift(double v, double t, double dx, int n, int *r, double *phi)
{
#pragma clang fp contract(off)
    if (n == 1) {
        *r = 0;
        *phi = 0.0;
        return;
    }
    const double u = (v * t) / dx;
    const double fl = floor(u);
    *phi = u - fl;
    const double nd = (double)n;
    double q = fl - nd * floor(fl / nd);
    if (q < 0.0)
        q += nd;
    if (q >= nd)
        q -= nd;
    *r = (int)q;
}

// Slopes in memory: fpic::NK reals per particle (components 0 and 9 are
// the negated sums of the next two and are not stored).
__device__ __forceinline__ int kslot(int c) { return c < 9 ? c - 1 : c - 2; }

// NT: streaming (nontemporal) loads, for the last read of a slope
template <bool NT = false>
__device__ __forceinline__ void load_slope(const double *K, int64_t np, int64_t p, bool active, double k[18])
{
#pragma unroll
    for (int c = 1; c < 18; c++)
        if (c != 9)
            k[c] = active ? (NT ? fpic::gld_nt(K + kslot(c) * np + p) : gld(K + kslot(c) * np + p)) : 0.0;
    k[0] = -(k[1] + k[2]);
    k[9] = -(k[10] + k[11]);
}

__device__ __forceinline__ double lane_get(double v, int src)
{
    return __shfl(v, src, W);
}

// Stage deposits carry the traceless part of each 3x3 source matrix: the
// interpolated Hamiltonian is needed only up to a multiple of the identity,
// which commutes with every state and leaves both commutators unchanged.
// Per particle the source X = (N/dV) rho - (Nbar/dV) rhobar^* is stored as
// NXT = 8 reals (x11 - x00, x22 - x00 and the six off-diagonal reals), and
// the stage grids hold NGT = 32 components (A, B_x, B_y, B_z, eight each);
// the moments diagnostic deposits all nine components of its sources.
constexpr int NXT = 8, NGT = 4 * NXT;

__device__ __forceinline__ void store_source(const Desc3 &S, int64_t p, double wN, double wNb,
                                             const double yn[18])
{
    double x[9];
#pragma unroll
    for (int k = 0; k < 9; k++)
        x[k] = (k == 4 || k == 6 || k == 8) ? wN * yn[k] + wNb * yn[9 + k] : wN * yn[k] - wNb * yn[9 + k];
    gst(S.X + p, x[1] - x[0]);
    gst(S.X + S.np + p, x[2] - x[0]);
#pragma unroll
    for (int k = 3; k < 9; k++)
        gst(S.X + (k - 1) * S.np + p, x[k]);
}

// MODE 1..4: Runge-Kutta stages; 5: deposit sources of the current state.
//
// A workgroup owns one row (y, z) of *current* lower cells and a group of
// directions (waves x dpw); for direction d, lane x takes the particle whose
// lower cell at the stage time is (x, y, z), i.e. the one stored at cell
// (x, y, z) minus the direction's integer shift.  Every particle of the
// workgroup then interpolates from the same four grid rows (y or y + 1,
// z or z + 1), which are staged in LDS once per workgroup; the particle data
// of each direction is one contiguous row, rotated in x.  MODE 5 has no
// interpolation and takes the particles in storage order.
constexpr int MAX_WAVES3 = 8;

template <int MODE>
__global__ void __launch_bounds__(MAX_WAVES3 * W)
particle3d_kernel(const Desc3 *__restrict__ dp, int dpw, int nitems)
{
    __shared__ double Gt[MODE == 5 ? 1 : 4 * NGT * W];  // [row q = 2 cz + cy][comp][x]
    const Desc3 S = *dp;
    const int lane = threadIdx.x & (W - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
    const int nwaves = blockDim.x / W;
    const int item = blockIdx.x;
    if (item >= nitems)
        return;  // whole workgroup: uniform
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int nrows = ny * nz;
    const int row = item % nrows, grp = item / nrows;
    const int y0 = row % ny, z0 = row / ny;
    const bool active = lane < nx;
    const int64_t n = *S.step;
    const double dt = S.dt;
    double t_cur = 0.0;
    if (MODE == 2 || MODE == 3)
        t_cur = stage_time(n, dt, 0.5);
    else if (MODE == 4)
        t_cur = stage_time(n, dt, 1.0);
    else
        t_cur = stage_time(n, dt, 0.0);
    const double *Gin = S.G[(MODE - 1) & 1];
    const double *Kp = (MODE == 2) ? S.K1 : (MODE == 3) ? S.K2 : S.K3;
    const int dbeg = (grp * nwaves + wave) * dpw, dend = min(dbeg + dpw, S.ndir);
    const int right = (lane + 1) % (nx < 1 ? 1 : nx);

    if (MODE != 5) {
        for (int idx = threadIdx.x; idx < 4 * NGT * nx; idx += blockDim.x) {
            const int x = idx % nx, t = idx / nx;
            const int comp = t % NGT, q = t / NGT;
            int yy = y0 + (q & 1), zz = z0 + (q >> 1);
            yy = (yy >= ny) ? yy - ny : yy;
            zz = (zz >= nz) ? zz - nz : zz;
            Gt[(q * NGT + comp) * W + x] = gld(Gin + (int64_t)comp * S.ncell + ((int64_t)zz * ny + yy) * nx + x);
        }
        __syncthreads();
    }

    for (int d = dbeg; d < dend; ++d) {
        const double vx = tld(S.v[0], d), vy = tld(S.v[1], d), vz = tld(S.v[2], d);
        const double wN = tld(S.wN, d), wNb = tld(S.wNb, d);
        int rx = 0, ry = 0, rz = 0;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        int64_t c;
        if (MODE == 5) {
            c = (int64_t)row * nx + (active ? lane : 0);
        } else {
            axis_shift(vx, t_cur, S.dx[0], nx, &rx, &fx);
            axis_shift(vy, t_cur, S.dx[1], ny, &ry, &fy);
            axis_shift(vz, t_cur, S.dx[2], nz, &rz, &fz);
            int cx = lane - rx, cy = y0 - ry, cz = z0 - rz;
            cx = (cx < 0) ? cx + nx : cx;
            cy = (cy < 0) ? cy + ny : cy;
            cz = (cz < 0) ? cz + nz : cz;
            c = ((int64_t)cz * ny + cy) * nx + (active ? cx : 0);
        }
        const int64_t p = (int64_t)d * S.ncell + c;
        double Y[18];
#pragma unroll
        for (int k = 0; k < 18; k++)
            Y[k] = active ? gld(S.Y + k * S.np + p) : 0.0;
        double yn[18];
        if (MODE == 5) {
#pragma unroll
            for (int k = 0; k < 18; k++)
                yn[k] = Y[k];
        } else {
            // y/z interpolation from the four staged rows, then x with the
            // lane to the right (periodic in x); one group of 8 traceless
            // components (A, B_x, B_y, B_z) at a time:
            // Hnn = A - (vx B_x + vy B_y + vz B_z), its ee entry 0
            double wyz[4];
#pragma unroll
            for (int cz = 0; cz < 2; cz++)
#pragma unroll
                for (int cy = 0; cy < 2; cy++)
                    wyz[2 * cz + cy] = (cy ? fy : 1.0 - fy) * (cz ? fz : 1.0 - fz);
            double Hnn[9];
#pragma unroll
            for (int k = 0; k < 9; k++)
                Hnn[k] = 0.0;
#pragma unroll 1
            for (int grp4 = 0; grp4 < 4; grp4++) {
                const double coef = (grp4 == 0) ? 1.0 : (grp4 == 1) ? -vx : (grp4 == 2) ? -vy : -vz;
#pragma unroll
                for (int k = 0; k < NXT; k++) {
                    const double *g = Gt + (NXT * grp4 + k) * W + lane;
                    double r = 0.0;
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        r += wyz[q] * (active ? g[q * NGT * W] : 0.0);
                    const double nb = lane_get(r, right);
                    const double val = (1.0 - fx) * r + fx * nb;
                    Hnn[k + 1] += coef * val;
                }
            }
            const double a = (MODE == 4) ? dt : 0.5 * dt;
            double yv[18], base[18];
            if (MODE == 1) {
#pragma unroll
                for (int k = 0; k < 18; k++)
                    yv[k] = base[k] = Y[k];
            } else if (MODE == 4) {
                const double h6 = dt / 6.0;
                double k1[18], k2[18], k3[18];
                load_slope<true>(S.K1, S.np, p, active, k1);
                load_slope<true>(S.K2, S.np, p, active, k2);
                load_slope<true>(S.K3, S.np, p, active, k3);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yv[k] = Y[k] + dt * k3[k];
                    const double ks = (k1[k] + 2.0 * k2[k]) + 2.0 * k3[k];
                    base[k] = Y[k] + h6 * ks;
                }
            } else {
                double kp[18];
                load_slope(Kp, S.np, p, active, kp);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yv[k] = Y[k] + a * kp[k];
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
            commutator(H, yv, kk);
            commutator(Hb, yv + 9, kk + 9);
            if (MODE == 4) {
                const double h6 = dt / 6.0;
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yn[k] = base[k] + h6 * kk[k];
                    if (active)
                        fpic::gst_nt(S.Y + k * S.np + p, yn[k]);
                }
            } else {
                double *Ko = (MODE == 1) ? S.K1 : (MODE == 2) ? S.K2 : S.K3;
                const double an = (MODE == 3) ? dt : 0.5 * dt;
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    if (active && k != 0 && k != 9) {
                        if (MODE == 2)  // k2 streams; k1 and k3 stay cached (as in 1D)
                            fpic::gst_nt(Ko + kslot(k) * S.np + p, kk[k]);
                        else
                            gst(Ko + kslot(k) * S.np + p, kk[k]);
                    }
                    yn[k] = base[k] + an * kk[k];
                }
            }
        }
        if (active)
            store_source(S, p, wN, wNb, yn);
    }
}

// Deposit of the sources at the positions of time t = (n + cnext) dt
// (cnext_num / 2 steps after step n's start; 2 means the next step).
// Each wave owns one x-row of destination cells and sweeps every direction
// in ascending order; per direction it interpolates the sources of the four
// rows in y and z, then in x with the lane to the left (accumulate).  The
// loop is software-pipelined: the 4 NC source values of direction d + 1
// (four rows, NC components) are loaded while direction d is summed.  NC is
// NXT (traceless stage sources, grid of NGT components) or 9 (moments, grid
// of 36).
template <int NC>
struct Pull {
    double X[NC];      // sources interpolated in y and z at the lane's x
    double fx, vx, vy, vz;
};

// One direction's components and interpolation fractions, and its 4 NC raw
// source values for the wave's row.  Lanes past the row (lane >= nx) load
// cell 0 of the row (never used).
template <int NC>
struct DepDir {
    double vx, vy, vz, fx, fy, fz;
    double raw[4 * NC];  // [2 cz + cy][NC]
};

template <int NC>
__device__ __forceinline__ void dep_load(const Desc3 &S, int d, double t, int y, int z, int lane,
                                         DepDir<NC> &o)
{
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    o.vx = tld(S.v[0], d);
    o.vy = tld(S.v[1], d);
    o.vz = tld(S.v[2], d);
    int rx, ry, rz;
    axis_shift(o.vx, t, S.dx[0], nx, &rx, &o.fx);
    axis_shift(o.vy, t, S.dx[1], ny, &ry, &o.fy);
    axis_shift(o.vz, t, S.dx[2], nz, &rz, &o.fz);
    // the same for the whole wave: row addresses in scalar registers
    rx = __builtin_amdgcn_readfirstlane(rx);
    ry = __builtin_amdgcn_readfirstlane(ry);
    rz = __builtin_amdgcn_readfirstlane(rz);
    int xs = lane - rx;
    xs = (xs < 0) ? xs + nx : xs;
    xs = (lane < nx) ? xs : 0;
#pragma unroll
    for (int cz = 0; cz < 2; cz++)
#pragma unroll
        for (int cy = 0; cy < 2; cy++) {
            int yy = y - ry - cy, zz = z - rz - cz;
            yy = (yy < 0) ? yy + ny : yy;
            yy = (yy < 0) ? yy + ny : yy;
            zz = (zz < 0) ? zz + nz : zz;
            zz = (zz < 0) ? zz + nz : zz;
            const double *xp = S.X + (int64_t)d * S.ncell + ((int64_t)zz * ny + yy) * nx;
#pragma unroll
            for (int k = 0; k < NC; k++)
                o.raw[(cz * 2 + cy) * NC + k] = gld(xp + (int64_t)k * S.np + xs);
        }
}

// y/z interpolation of one direction's raw sources (rows in the order
// cz, cy; inactive lanes take 0)
template <int NC>
__device__ __forceinline__ void pull_dir(const DepDir<NC> &c, bool active, Pull<NC> &o)
{
    o.vx = c.vx;
    o.vy = c.vy;
    o.vz = c.vz;
    o.fx = c.fx;
#pragma unroll
    for (int k = 0; k < NC; k++)
        o.X[k] = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; cz++)
#pragma unroll
        for (int cy = 0; cy < 2; cy++) {
            const double w = (cy ? c.fy : 1.0 - c.fy) * (cz ? c.fz : 1.0 - c.fz);
#pragma unroll
            for (int k = 0; k < NC; k++)
                o.X[k] += w * (active ? c.raw[(cz * 2 + cy) * NC + k] : 0.0);
        }
}

template <int NC>
__device__ __forceinline__ void accumulate(const Pull<NC> &o, int left, double acc[4 * NC])
{
#pragma unroll
    for (int k = 0; k < NC; k++) {
        const double xl = lane_get(o.X[k], left);
        const double xc = (1.0 - o.fx) * o.X[k] + o.fx * xl;
        acc[k] += xc;
        acc[NC + k] += o.vx * xc;
        acc[2 * NC + k] += o.vy * xc;
        acc[3 * NC + k] += o.vz * xc;
    }
}

// A deposit workgroup covers a patch of DEP_PY x DEP_PZ destination rows,
// one wave per row; its waves sweep the directions in the same order, so
// the source rows they share (a patch of (DEP_PY + 1) x (DEP_PZ + 1) rows
// per direction) are mostly read from memory once.
constexpr int DEP_PY = 2, DEP_PZ = 2;
constexpr int DEP_WAVES = DEP_PY * DEP_PZ;

template <int NC>
__global__ void __launch_bounds__(DEP_WAVES * W)
deposit3d_kernel(const Desc3 *__restrict__ dp, int half_steps, int out_buf)
{
    const Desc3 S = *dp;
    const int lane = threadIdx.x & (W - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int npy = (ny + DEP_PY - 1) / DEP_PY;
    const int y = (blockIdx.x % npy) * DEP_PY + wave % DEP_PY;
    const int z = (blockIdx.x / npy) * DEP_PZ + wave / DEP_PY;
    if (y >= ny || z >= nz)
        return;  // no workgroup barrier in this kernel
    const bool active = lane < nx;
    const int64_t n0 = *S.step;
    // half_steps: 0 -> t_n, 1 -> t_n + dt/2, 2 -> t_n + dt (stage 4 of step
    // n), 3 -> first stage of step n + 1
    double t;
    if (half_steps == 3)
        t = stage_time(n0 + 1, S.dt, 0.0);
    else
        t = stage_time(n0, S.dt, 0.5 * half_steps);
    const int left = (lane + nx - 1) % (nx < 1 ? 1 : nx);
    double acc[4 * NC];
#pragma unroll
    for (int q = 0; q < 4 * NC; q++)
        acc[q] = 0.0;
    DepDir<NC> nxt;
    if (S.ndir > 0)
        dep_load<NC>(S, 0, t, y, z, lane, nxt);
    for (int d = 0; d < S.ndir; ++d) {
        const DepDir<NC> cur = nxt;
        if (d + 1 < S.ndir)
            dep_load<NC>(S, d + 1, t, y, z, lane, nxt);
        Pull<NC> a;
        pull_dir<NC>(cur, active, a);
        accumulate<NC>(a, left, acc);
    }
    if (active) {
        double *G = out_buf ? S.G[1] : S.G[0];  // (no dynamic index into the descriptor)
        const int64_t cell = ((int64_t)z * ny + y) * nx + lane;
#pragma unroll
        for (int q = 0; q < 4 * NC; q++)
            gst(G + (int64_t)q * S.ncell + cell, acc[q]);
    }
}

static unsigned deposit_blocks(const Desc3 &h)
{
    return (unsigned)(((h.n[1] + DEP_PY - 1) / DEP_PY) * ((h.n[2] + DEP_PZ - 1) / DEP_PZ));
}

// ---------------------------------------------------------------------------
// Quadratic (triangular-shaped cloud) shape function, Sec. II.B.1.  Along
// each axis a particle spreads over its nearest cell centre and the two
// neighbours with weights (1/2 - xi)^2 / 2, 3/4 - xi^2, (1/2 + xi)^2 / 2,
// xi = x - x_nearest in [-1/2, 1/2) (each operation rounded once, as the CPU
// reference forms them); a one-cell axis gives (0, 1, 0).  The particle
// kernel's workgroup owns one row of *nearest* cells and stages the nine grid
// rows it interpolates from in LDS, as the 32 traceless moment components
// (nine rows of all 36 would not fit the 160 KB at 64 cells per row).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void axis_quad(double v, double t, double dx, int n, int *r, double w[3])
{
#pragma clang fp contract(off)
    if (n == 1) {
        *r = 0;
        w[0] = 0.0;
        w[1] = 1.0;
        w[2] = 0.0;
        return;
    }
    const double u = (v * t) / dx;
    const double fl = floor(u);
    const double phi = u - fl;
    const int up = phi < 0.5 ? 0 : 1;
    const double xi = up ? phi - 1.0 : phi;
    w[0] = 0.5 * ((0.5 - xi) * (0.5 - xi));
    w[1] = 0.75 - xi * xi;
    w[2] = 0.5 * ((0.5 + xi) * (0.5 + xi));
    const double nd = (double)n;
    const double near = fl + (double)up;
    double q = near - nd * floor(near / nd);
    if (q < 0.0)
        q += nd;
    if (q >= nd)
        q -= nd;
    *r = (int)q;
}

__device__ __forceinline__ int wrap(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// w[b] for a run-time b in 0..2, without indexing a private array
__device__ __forceinline__ double pick3(const double w[3], int b)
{
    return b == 0 ? w[0] : (b == 1 ? w[1] : w[2]);
}

// Directions per gather block: each LDS read of a grid row serves the
// block's directions.  Two for stages 1-3; stage 4 holds three slopes and
// keeps one (more would spill).
template <int MODE>
constexpr int qdb() { return MODE == 4 ? 1 : 2; }

template <int MODE>
__global__ void __launch_bounds__(MAX_WAVES3 * W)
particle3q_kernel(const Desc3 *__restrict__ dp, int dpw, int nitems)
{
    __shared__ double Gq[9 * NGT * W];   // [row q][component][x], 144 KiB
    const Desc3 S = *dp;
    const int lane = threadIdx.x & (W - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
    const int nwaves = blockDim.x / W;
    const int item = blockIdx.x;
    if (item >= nitems)
        return;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int nrows = ny * nz;
    const int row = item % nrows, grp = item / nrows;
    const int y0 = row % ny, z0 = row / ny;
    const bool active = lane < nx;
    const int64_t n = *S.step;
    const double dt = S.dt;
    double t_cur = 0.0;
    if (MODE == 2 || MODE == 3)
        t_cur = stage_time(n, dt, 0.5);
    else if (MODE == 4)
        t_cur = stage_time(n, dt, 1.0);
    else
        t_cur = stage_time(n, dt, 0.0);
    const double *Gin = S.G[(MODE - 1) & 1];
    const double *Kp = (MODE == 2) ? S.K1 : (MODE == 3) ? S.K2 : S.K3;
    const int dbeg = (grp * nwaves + wave) * dpw, dend = min(dbeg + dpw, S.ndir);
    const int xl = (lane + nx - 1) % (nx < 1 ? 1 : nx), xr = (lane + 1) % (nx < 1 ? 1 : nx);
    // Stage the nine grid rows around the nearest row (y0, z0) in LDS, row
    // q = 3 c + b being (y0 + b - 1, z0 + c - 1): the 32 traceless moment
    // components of the stage grid (36 would not fit at 64 cells per row).
    // Columns past the row (x >= nx) hold 0.
    for (int idx = threadIdx.x; idx < 9 * 4 * W; idx += blockDim.x) {
        const int x = idx % W, t = idx / W;
        const int g4 = t % 4, q = t / 4;  // eight components of one matrix per task
        const int b = q % 3, cc = q / 3;
        double v[NXT];
#pragma unroll
        for (int k = 0; k < NXT; k++)
            v[k] = 0.0;
        if (x < nx) {
            const int64_t cell = ((int64_t)wrap(z0 + cc - 1, nz) * ny + wrap(y0 + b - 1, ny)) * nx + x;
#pragma unroll
            for (int k = 0; k < NXT; k++)
                v[k] = gld(Gin + (int64_t)(NXT * g4 + k) * S.ncell + cell);
        }
#pragma unroll
        for (int k = 0; k < NXT; k++)
            Gq[(q * NGT + NXT * g4 + k) * W + x] = v[k];
    }
    __syncthreads();

    constexpr int QDB = qdb<MODE>();
    for (int d0 = dbeg; d0 < dend; d0 += QDB) {
        // weights of the block's directions (past the end: the last one
        // again, not stored)
        double vb[QDB][3], wxb[QDB][3], wyb[QDB][3], wzb[QDB][3];
        int rxb[QDB], ryb[QDB], rzb[QDB];
#pragma unroll
        for (int j = 0; j < QDB; j++) {
            const int d = min(d0 + j, dend - 1);
            vb[j][0] = tld(S.v[0], d);
            vb[j][1] = tld(S.v[1], d);
            vb[j][2] = tld(S.v[2], d);
            axis_quad(vb[j][0], t_cur, S.dx[0], nx, &rxb[j], wxb[j]);
            axis_quad(vb[j][1], t_cur, S.dx[1], ny, &ryb[j], wyb[j]);
            axis_quad(vb[j][2], t_cur, S.dx[2], nz, &rzb[j], wzb[j]);
        }
        // traceless Hnn: components 1..8 of the packed nine (component 0,
        // the ee entry, is 0)
        double Hb4[QDB][NXT];
#pragma unroll
        for (int j = 0; j < QDB; j++)
#pragma unroll
            for (int k = 0; k < NXT; k++)
                Hb4[j][k] = 0.0;
#pragma unroll 1
        for (int grp4 = 0; grp4 < 4; grp4++) {
            // y/z interpolation row by row from LDS, each read used by every
            // direction of the block
            double r[QDB][NXT];
#pragma unroll
            for (int j = 0; j < QDB; j++)
#pragma unroll
                for (int k = 0; k < NXT; k++)
                    r[j][k] = 0.0;
#pragma unroll 3
            for (int q = 0; q < 9; q++) {
                const int b = q % 3, cc = q / 3;
                const double *gp = Gq + (q * NGT + NXT * grp4) * W + lane;
                double gv[NXT];
#pragma unroll
                for (int k = 0; k < NXT; k++)
                    gv[k] = gp[k * W];
#pragma unroll
                for (int j = 0; j < QDB; j++) {
                    const double wq = pick3(wyb[j], b) * pick3(wzb[j], cc);
#pragma unroll
                    for (int k = 0; k < NXT; k++)
                        r[j][k] += wq * gv[k];
                }
            }
#pragma unroll
            for (int j = 0; j < QDB; j++) {
                const double coef = (grp4 == 0) ? 1.0 : -pick3(vb[j], grp4 - 1);
#pragma unroll
                for (int k = 0; k < NXT; k++) {
                    const double nl = lane_get(r[j][k], xl), nr = lane_get(r[j][k], xr);
                    Hb4[j][k] += coef * ((wxb[j][0] * nl + wxb[j][1] * r[j][k]) + wxb[j][2] * nr);
                }
            }
        }

#pragma unroll 1
        for (int j = 0; j < QDB; j++) {
            const int d = d0 + j;
            if (d >= dend)
                break;
            const double wN = tld(S.wN, d), wNb = tld(S.wNb, d);
            int rx = rxb[0], ry = ryb[0], rz = rzb[0];
            double Hnn[9];
            Hnn[0] = 0.0;
#pragma unroll
            for (int k = 1; k < 9; k++)
                Hnn[k] = Hb4[0][k - 1];
#pragma unroll
            for (int jj = 1; jj < QDB; jj++) {
                const bool m = j == jj;
                rx = m ? rxb[jj] : rx;
                ry = m ? ryb[jj] : ry;
                rz = m ? rzb[jj] : rz;
#pragma unroll
                for (int k = 1; k < 9; k++)
                    Hnn[k] = m ? Hb4[jj][k - 1] : Hnn[k];
            }
            const int cx = wrap(lane - rx, nx), cy = wrap(y0 - ry, ny), cz = wrap(z0 - rz, nz);
            const int64_t c = ((int64_t)cz * ny + cy) * nx + (active ? cx : 0);
            const int64_t p = (int64_t)d * S.ncell + c;
            double Y[18];
#pragma unroll
            for (int k = 0; k < 18; k++)
                Y[k] = active ? gld(S.Y + k * S.np + p) : 0.0;
            double yv[18], base[18], yn[18];
            if (MODE == 1) {
#pragma unroll
                for (int k = 0; k < 18; k++)
                    yv[k] = base[k] = Y[k];
            } else if (MODE == 4) {
                // slopes one at a time into (k1 + 2 k2) + 2 k3 (fewer live
                // registers than holding all three)
                const double h6 = dt / 6.0;
                double ks[18], kt[18];
                load_slope<true>(S.K1, S.np, p, active, ks);
                load_slope<true>(S.K2, S.np, p, active, kt);
#pragma unroll
                for (int k = 0; k < 18; k++)
                    ks[k] = ks[k] + 2.0 * kt[k];
                load_slope<true>(S.K3, S.np, p, active, kt);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yv[k] = Y[k] + dt * kt[k];
                    base[k] = Y[k] + h6 * (ks[k] + 2.0 * kt[k]);
                }
            } else {
                double kp[18];
                load_slope(Kp, S.np, p, active, kp);
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yv[k] = Y[k] + 0.5 * dt * kp[k];
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
            commutator(H, yv, kk);
            commutator(Hb, yv + 9, kk + 9);
            if (MODE == 4) {
                const double h6 = dt / 6.0;
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    yn[k] = base[k] + h6 * kk[k];
                    if (active)
                        fpic::gst_nt(S.Y + k * S.np + p, yn[k]);
                }
            } else {
                double *Ko = (MODE == 1) ? S.K1 : (MODE == 2) ? S.K2 : S.K3;
                const double an = (MODE == 3) ? dt : 0.5 * dt;
#pragma unroll
                for (int k = 0; k < 18; k++) {
                    if (active && k != 0 && k != 9) {
                        if (MODE == 2)  // k2 streams; k1 and k3 stay cached (as in 1D)
                            fpic::gst_nt(Ko + kslot(k) * S.np + p, kk[k]);
                        else
                            gst(Ko + kslot(k) * S.np + p, kk[k]);
                    }
                    yn[k] = base[k] + an * kk[k];
                }
            }
            if (active)
                store_source(S, p, wN, wNb, yn);
        }
    }
}

// Quadratic deposit: destination cell (x, y, z) takes weight
// wx[i] wy[j] wz[k] from the particle whose nearest cell is
// (x - i + 1, y - j + 1, z - k + 1), i, j, k = 0..2: nine source rows in y
// and z, then the lanes one right and one left in x.
template <int NC>
__global__ void __launch_bounds__(DEP_WAVES * W)
deposit3q_kernel(const Desc3 *__restrict__ dp, int half_steps, int out_buf)
{
    const Desc3 S = *dp;
    const int lane = threadIdx.x & (W - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int npy = (ny + DEP_PY - 1) / DEP_PY;
    const int y = (blockIdx.x % npy) * DEP_PY + wave % DEP_PY;
    const int z = (blockIdx.x / npy) * DEP_PZ + wave / DEP_PY;
    if (y >= ny || z >= nz)
        return;  // no workgroup barrier in this kernel
    const bool active = lane < nx;
    const int64_t n0 = *S.step;
    double t;
    if (half_steps == 3)
        t = stage_time(n0 + 1, S.dt, 0.0);
    else
        t = stage_time(n0, S.dt, 0.5 * half_steps);
    const int xl = (lane + nx - 1) % (nx < 1 ? 1 : nx), xr = (lane + 1) % (nx < 1 ? 1 : nx);
    double acc[4 * NC];
#pragma unroll
    for (int q = 0; q < 4 * NC; q++)
        acc[q] = 0.0;
    for (int d = 0; d < S.ndir; ++d) {
        const double vx = tld(S.v[0], d), vy = tld(S.v[1], d), vz = tld(S.v[2], d);
        int rx, ry, rz;
        double wx[3], wy[3], wz[3];
        axis_quad(vx, t, S.dx[0], nx, &rx, wx);
        axis_quad(vy, t, S.dx[1], ny, &ry, wy);
        axis_quad(vz, t, S.dx[2], nz, &rz, wz);
        const int xs = active ? wrap(lane - rx, nx) : 0;
        double Xyz[NC];
#pragma unroll
        for (int k = 0; k < NC; k++)
            Xyz[k] = 0.0;
#pragma unroll 1
        for (int kk = 0; kk < 3; kk++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const int yy = wrap(y - j + 1 - ry, ny), zz = wrap(z - kk + 1 - rz, nz);
                const double w = wy[j] * wz[kk];
                const double *xp = S.X + (int64_t)d * S.ncell + ((int64_t)zz * ny + yy) * nx + xs;
#pragma unroll
                for (int k = 0; k < NC; k++)
                    Xyz[k] += w * (active ? gld(xp + (int64_t)k * S.np) : 0.0);
            }
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const double right = lane_get(Xyz[k], xr), left = lane_get(Xyz[k], xl);
            const double xc = (wx[0] * right + wx[1] * Xyz[k]) + wx[2] * left;
            acc[k] += xc;
            acc[NC + k] += vx * xc;
            acc[2 * NC + k] += vy * xc;
            acc[3 * NC + k] += vz * xc;
        }
    }
    if (active) {
        double *G = out_buf ? S.G[1] : S.G[0];
        const int64_t cell = ((int64_t)z * ny + y) * nx + lane;
#pragma unroll
        for (int q = 0; q < 4 * NC; q++)
            gst(G + (int64_t)q * S.ncell + cell, acc[q]);
    }
}

// moments of neutrinos (which = 0) or antineutrinos (1) at the current step
// time, written to out[36][ncell] (deposits N rho or Nbar rhobar alone)
__global__ void __launch_bounds__(256)
momsrc3d_kernel(const Desc3 *__restrict__ dp, int which)
{
    const Desc3 S = *dp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += stride) {
        const int d = (int)(p / S.ncell);
        const double w = which ? tld(S.wNb, d) : tld(S.wN, d);
        for (int k = 0; k < 9; k++)
            gst(S.X + k * S.np + p, w * gld(S.Y + (which * 9 + k) * S.np + p));
    }
}

__global__ void set_step3d(const Desc3 *dp, int64_t v)
{
    if (threadIdx.x == 0)
        *dp->step = v;
}

__global__ void tick3d(const Desc3 *dp)
{
    if (threadIdx.x == 0)
        *dp->step += 1;
}

__global__ void __launch_bounds__(256) totals3d(const Desc3 *dp, double *partial)
{
    const Desc3 &S = *dp;
    __shared__ double sh[256];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < 18; ++k) {
        double s = 0.0;
        for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S.np; p += stride) {
            const int d = (int)(p / S.ncell);
            s += ((k < 9) ? tld(S.Nw, d) : tld(S.Nbw, d)) * S.Y[k * S.np + p];
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

__global__ void __launch_bounds__(256) check3d(const Desc3 *dp, double *partial)
{
    const Desc3 &S = *dp;
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
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q)
            partial[blockIdx.x * 3 + q] = sh[q][0];
}

__global__ void finish_sums(const double *partial, int nblk, int width, int is_check, double *out)
{
    const int k = threadIdx.x;
    if (k >= width)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) {
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

constexpr int kBlk = 256;  // blocks of the diagnostic reductions

struct Ctx3D {
    Desc3 h;
    Desc3 *d = nullptr;
    char *ws = nullptr;
    hipStream_t stream = nullptr, cap = nullptr;
    int waves = 8, dpw = 0, ngroup = 0, spg = 8, nitems = 0;
    double *scratch = nullptr, *hbuf = nullptr;
    hipGraphExec_t g1 = nullptr, gK = nullptr;
    bool state_set = false;
};

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t tab, Y, K1, K2, K3, X, G0, G1, step, desc, scratch, total;
    int waves, dpw, ngroup, spg;
};

static int validate(const fpic_config &c)
{
    if (c.ncell[0] < 1 || c.ncell[1] < 1 || c.ncell[2] < 1 || c.ndir < 1)
        return fail(FPIC_EINVAL, "cell and direction counts must be >= 1");
    if (c.ncell[0] > W)
        return fail(FPIC_EUNSUPPORTED, "3D boxes need nx <= 64 (the x axis of a box fits one wave)");
    if (!c.dirs || !c.N || !c.Nbar)
        return fail(FPIC_EINVAL, "dirs, N and Nbar must be non-null host arrays");
    if (c.shape_order != 1 && c.shape_order != 2)
        return fail(FPIC_EUNSUPPORTED,
                    "shape_order must be 1 (linear, cloud in cell) or 2 (quadratic)");
    if (!(c.dt > 0.0) || !std::isfinite(c.dt))
        return fail(FPIC_EINVAL, "dt must be positive and finite");
    for (int a = 0; a < 3; ++a)
        if (!(c.dx[a] > 0.0) || !std::isfinite(c.dx[a]))
            return fail(FPIC_EINVAL, "cell widths must be positive and finite");
    if ((int64_t)c.ncell[0] * c.ncell[1] * c.ncell[2] > ((int64_t)1 << 30))
        return fail(FPIC_EINVAL, "too many cells");
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
    double vmax[3] = {0, 0, 0};
    for (int d = 0; d < c.ndir; ++d) {
        const double *v = c.dirs + 3 * d;
        const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (!std::isfinite(n2) || std::fabs(n2 - 1.0) > 1e-9)
            return fail(FPIC_EINVAL, "directions must be unit vectors");
        if (!std::isfinite(c.N[d]) || !std::isfinite(c.Nbar[d]))
            return fail(FPIC_EINVAL, "weights must be finite");
        for (int a = 0; a < 3; ++a)
            vmax[a] = std::max(vmax[a], std::fabs(v[a]));
    }
    for (int a = 0; a < 3; ++a)
        if (c.ncell[a] > 1 && 0.5 * c.dt * vmax[a] / c.dx[a] >= 1.0 - 1e-9)
            return fail(FPIC_EUNSUPPORTED,
                        "dt too large: a particle may cross a whole cell within one "
                        "Runge-Kutta stage (need dt/2 * max|Omega| < dx)");
    return FPIC_OK;
}

static int layout(const fpic_config &c, const fpic_tuning *t, Layout &L)
{
    int rc = validate(c);
    if (rc)
        return rc;
    const int64_t nc = (int64_t)c.ncell[0] * c.ncell[1] * c.ncell[2];
    const int64_t np = nc * c.ndir;
    const int64_t nrows = (int64_t)c.ncell[1] * c.ncell[2];
    L.waves = (t && t->waves) ? t->waves : 8;
    if (L.waves != 1 && L.waves != 2 && L.waves != 4 && L.waves != MAX_WAVES3)
        return fail(FPIC_EINVAL, "waves must be 1, 2, 4 or 8 for 3D boxes");
    L.dpw = (t && t->dirs_per_wave) ? t->dirs_per_wave : 0;
    if (L.dpw < 0 || L.dpw > 4096)
        return fail(FPIC_EINVAL, "dirs_per_wave out of range");
    if (!L.dpw) {
        // one direction group per row when there are enough rows to fill
        // the chip (about 2048 workgroups), more groups otherwise
        const int64_t groups = std::max<int64_t>(1, (2048 + nrows - 1) / nrows);
        const int64_t dpg = std::max<int64_t>(L.waves, (c.ndir + groups - 1) / groups);
        L.dpw = (int)((dpg + L.waves - 1) / L.waves);
    }
    const int dpg = L.waves * L.dpw;
    L.ngroup = (c.ndir + dpg - 1) / dpg;
    L.spg = (t && t->steps_per_graph) ? t->steps_per_graph : 8;
    if (L.spg < 1 || L.spg > 256)
        return fail(FPIC_EINVAL, "steps_per_graph must be in 1..256");
    size_t off = 0;
    auto take = [&](size_t b) {
        off = al(off);
        size_t o = off;
        off += b;
        return o;
    };
    const size_t st = sizeof(double) * 18 * (size_t)np;
    const size_t sk = sizeof(double) * fpic::NK * (size_t)np;
    L.tab = take(sizeof(double) * 7 * c.ndir);
    L.Y = take(st);
    L.K1 = take(sk);
    L.K2 = take(sk);
    L.K3 = take(sk);
    L.X = take(sizeof(double) * 9 * (size_t)np);
    L.G0 = take(sizeof(double) * NG * (size_t)nc);
    L.G1 = take(sizeof(double) * NG * (size_t)nc);
    L.step = take(sizeof(int64_t));
    L.desc = take(sizeof(Desc3));
    L.scratch = take(sizeof(double) * (18 + 18 * kBlk + 3 * kBlk + 3));
    L.total = al(off);
    return FPIC_OK;
}

int workspace_bytes(const fpic_config &cfg, const fpic_tuning *tune, size_t *bytes)
{
    Layout L;
    int rc = layout(cfg, tune, L);
    if (rc)
        return rc;
    *bytes = L.total;
    return FPIC_OK;
}

// stage `mode` (1..4; 5 = deposit sources of the current state) of the
// particle kernels, and the deposit of the sources, for the box's shape order
static void launch_particle(const Ctx3D *c, int mode, hipStream_t s)
{
    const dim3 pgrid(c->nitems), pblk(c->waves * W);
    const bool q = c->h.shape == 2;
    switch (mode) {
    case 1:
        if (q) particle3q_kernel<1><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        else particle3d_kernel<1><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        break;
    case 2:
        if (q) particle3q_kernel<2><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        else particle3d_kernel<2><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        break;
    case 3:
        if (q) particle3q_kernel<3><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        else particle3d_kernel<3><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        break;
    case 4:
        if (q) particle3q_kernel<4><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        else particle3d_kernel<4><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        break;
    default:  // no interpolation: the same for both shapes
        particle3d_kernel<5><<<pgrid, pblk, 0, s>>>(c->d, c->dpw, c->nitems);
        break;
    }
}

// The stage deposits (traceless sources, NGT grid components); full = true
// for the moments diagnostic (all nine source components, 36 per cell).
static void launch_deposit(const Ctx3D *c, const Desc3 *dd, int half_steps, int out_buf, hipStream_t s,
                           bool full = false)
{
    const dim3 dgrid(deposit_blocks(c->h)), blk(DEP_WAVES * W);
    if (c->h.shape == 2) {
        if (full)
            deposit3q_kernel<9><<<dgrid, blk, 0, s>>>(dd, half_steps, out_buf);
        else
            deposit3q_kernel<NXT><<<dgrid, blk, 0, s>>>(dd, half_steps, out_buf);
    } else {
        if (full)
            deposit3d_kernel<9><<<dgrid, blk, 0, s>>>(dd, half_steps, out_buf);
        else
            deposit3d_kernel<NXT><<<dgrid, blk, 0, s>>>(dd, half_steps, out_buf);
    }
}

static hipError_t launch_step(Ctx3D *c, hipStream_t s)
{
    // stage s reads G[(s-1)&1]; its deposit writes G[s&1]
    launch_particle(c, 1, s);
    launch_deposit(c, c->d, 1, 1, s);
    launch_particle(c, 2, s);
    launch_deposit(c, c->d, 1, 0, s);
    launch_particle(c, 3, s);
    launch_deposit(c, c->d, 2, 1, s);
    launch_particle(c, 4, s);
    launch_deposit(c, c->d, 3, 0, s);
    tick3d<<<1, 64, 0, s>>>(c->d);
    return hipGetLastError();
}

static int capture(Ctx3D *c, int nsteps, hipGraphExec_t *exec)
{
    HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int i = 0; i < nsteps && err == hipSuccess; ++i)
        err = launch_step(c, c->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (err != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return fail(FPIC_EHIP, std::string("launch during capture: ") + hipGetErrorString(err));
    }
    HIPCHECK(e2);
    hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHECK(e3);
    return FPIC_OK;
}

int create(const fpic_config &cfg, const fpic_tuning *tune, void *ws, size_t bytes, fpic_stream stream,
           Ctx3D **out)
{
    Layout L;
    int rc = layout(cfg, tune, L);
    if (rc)
        return rc;
    if (!ws || bytes < L.total || reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(FPIC_EINVAL, "workspace missing, too small or misaligned");
    Ctx3D *c = new Ctx3D();
    c->ws = static_cast<char *>(ws);
    c->stream = static_cast<hipStream_t>(stream);
    c->waves = L.waves;
    c->dpw = L.dpw;
    c->ngroup = L.ngroup;
    c->spg = L.spg;
    c->nitems = cfg.ncell[1] * cfg.ncell[2] * L.ngroup;
    const int nd = cfg.ndir;
    const double dV = cfg.dx[0] * cfg.dx[1] * cfg.dx[2];
    std::vector<double> tab(7 * (size_t)nd);
    for (int d = 0; d < nd; ++d) {
        for (int a = 0; a < 3; ++a)
            tab[a * nd + d] = cfg.dirs[3 * d + a];
        tab[3 * nd + d] = cfg.N[d] / dV;
        tab[4 * nd + d] = cfg.Nbar[d] / dV;
        tab[5 * nd + d] = cfg.N[d];
        tab[6 * nd + d] = cfg.Nbar[d];
    }
    Desc3 &D = c->h;
    std::memset(&D, 0, sizeof D);
    for (int a = 0; a < 3; ++a) {
        D.n[a] = cfg.ncell[a];
        D.dx[a] = cfg.dx[a];
    }
    D.ndir = nd;
    D.ncell = (int64_t)cfg.ncell[0] * cfg.ncell[1] * cfg.ncell[2];
    D.np = D.ncell * nd;
    D.dt = cfg.dt;
    D.shape = cfg.shape_order;
    const double *h = cfg.hvac;
    const double hv[9] = {h[0], h[8], h[16], h[2], h[3], h[4], h[5], h[10], h[11]};
    for (int k = 0; k < 9; ++k) {
        D.hvac[k] = hv[k] + (k < 3 ? cfg.vmat[k] : 0.0);
        D.hvacb[k] = hv[k] - (k < 3 ? cfg.vmat[k] : 0.0);
    }
    const double *tb = reinterpret_cast<const double *>(c->ws + L.tab);
    for (int a = 0; a < 3; ++a)
        D.v[a] = tb + a * nd;
    D.wN = tb + 3 * nd;
    D.wNb = tb + 4 * nd;
    D.Nw = tb + 5 * nd;
    D.Nbw = tb + 6 * nd;
    D.Y = reinterpret_cast<double *>(c->ws + L.Y);
    D.K1 = reinterpret_cast<double *>(c->ws + L.K1);
    D.K2 = reinterpret_cast<double *>(c->ws + L.K2);
    D.K3 = reinterpret_cast<double *>(c->ws + L.K3);
    D.X = reinterpret_cast<double *>(c->ws + L.X);
    D.G[0] = reinterpret_cast<double *>(c->ws + L.G0);
    D.G[1] = reinterpret_cast<double *>(c->ws + L.G1);
    D.step = reinterpret_cast<int64_t *>(c->ws + L.step);
    c->d = reinterpret_cast<Desc3 *>(c->ws + L.desc);
    c->scratch = reinterpret_cast<double *>(c->ws + L.scratch);
    hipError_t e = hipMemcpy(c->ws + L.tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->d, &D, sizeof D, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&c->hbuf), sizeof(double) * 64, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy(c);
        return fail(FPIC_EHIP, std::string("create: ") + hipGetErrorString(e));
    }
    rc = capture(c, 1, &c->g1);
    if (!rc && c->spg > 1)
        rc = capture(c, c->spg, &c->gK);
    if (rc) {
        destroy(c);
        return rc;
    }
    *out = c;
    return FPIC_OK;
}

int set_state(Ctx3D *c, const double *state, int64_t step0)
{
    if (!c || !state)
        return fail(FPIC_EINVAL, "set_state: null argument");
    HIPCHECK(hipMemcpyAsync(c->h.Y, state, sizeof(double) * 18 * c->h.np, hipMemcpyDeviceToDevice, c->stream));
    set_step3d<<<1, 64, 0, c->stream>>>(c->d, step0);
    HIPCHECK(hipGetLastError());
    launch_particle(c, 5, c->stream);
    launch_deposit(c, c->d, 0, 0, c->stream);
    HIPCHECK(hipGetLastError());
    c->state_set = true;
    return FPIC_OK;
}

int get_state(Ctx3D *c, double *state)
{
    if (!c || !state)
        return fail(FPIC_EINVAL, "get_state: null argument");
    HIPCHECK(hipMemcpyAsync(state, c->h.Y, sizeof(double) * 18 * c->h.np, hipMemcpyDeviceToDevice, c->stream));
    return FPIC_OK;
}

int step(Ctx3D *c, int64_t nsteps)
{
    if (!c || nsteps < 0)
        return fail(FPIC_EINVAL, "step: bad argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "step before set_state");
    int64_t left = nsteps;
    while (c->spg > 1 && left >= c->spg) {
        HIPCHECK(hipGraphLaunch(c->gK, c->stream));
        left -= c->spg;
    }
    while (left-- > 0)
        HIPCHECK(hipGraphLaunch(c->g1, c->stream));
    return FPIC_OK;
}

int moments(Ctx3D *c, double *out)
{
    if (!c || !out)
        return fail(FPIC_EINVAL, "moments: null argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "moments before set_state");
    // the deposit kernel writes G[out_buf]; point a copy of the descriptor
    // at the caller's buffer
    Desc3 D = c->h;
    for (int which = 0; which < 2; ++which) {
        D.G[0] = out + (size_t)which * NG * c->h.ncell;
        HIPCHECK(hipMemcpyAsync(c->scratch, &D, sizeof D, hipMemcpyHostToDevice, c->stream));
        const Desc3 *dd = reinterpret_cast<const Desc3 *>(c->scratch);
        momsrc3d_kernel<<<1024, 256, 0, c->stream>>>(dd, which);
        launch_deposit(c, dd, 0, 0, c->stream, true);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(c->stream));   // D is a host temporary
    }
    // (the stage kernels rewrite the deposit sources before every deposit)
    return FPIC_OK;
}

int flavor_totals(Ctx3D *c, double *out)
{
    if (!c || !out)
        return fail(FPIC_EINVAL, "flavor_totals: null argument");
    if (!c->state_set)
        return fail(FPIC_ESTATE, "flavor_totals before set_state");
    double *part = c->scratch + 18;
    totals3d<<<kBlk, 256, 0, c->stream>>>(c->d, part);
    finish_sums<<<1, 64, 0, c->stream>>>(part, kBlk, 18, 0, c->scratch);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->scratch, sizeof(double) * 18, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    std::memcpy(out, c->hbuf, sizeof(double) * 18);
    return FPIC_OK;
}

int check(Ctx3D *c, double r[3])
{
    if (!c->state_set)
        return fail(FPIC_ESTATE, "check before set_state");
    double *part = c->scratch + 18 + 18 * kBlk;
    check3d<<<kBlk, 256, 0, c->stream>>>(c->d, part);
    finish_sums<<<1, 64, 0, c->stream>>>(part, kBlk, 3, 1, c->scratch);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->scratch, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    std::memcpy(r, c->hbuf, sizeof(double) * 3);
    return FPIC_OK;
}

int get_step(Ctx3D *c, int64_t *s)
{
    HIPCHECK(hipMemcpyAsync(c->hbuf, c->h.step, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    std::memcpy(s, c->hbuf, sizeof(int64_t));
    return FPIC_OK;
}

int sync(Ctx3D *c)
{
    HIPCHECK(hipStreamSynchronize(c->stream));
    return FPIC_OK;
}

int profile(Ctx3D *c, int nsteps, double *ms)
{
    if (!c->state_set)
        return fail(FPIC_ESTATE, "profile before set_state");
    hipEvent_t ev[9];
    for (auto &e : ev)
        HIPCHECK(hipEventCreate(&e));
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipStream_t s = c->stream;
    int rc = FPIC_OK;
    for (int n = 0; n < nsteps && !rc; ++n) {
        (void)hipEventRecord(ev[0], s);
        launch_particle(c, 1, s);
        (void)hipEventRecord(ev[1], s);
        launch_deposit(c, c->d, 1, 1, s);
        (void)hipEventRecord(ev[2], s);
        launch_particle(c, 2, s);
        (void)hipEventRecord(ev[3], s);
        launch_deposit(c, c->d, 1, 0, s);
        (void)hipEventRecord(ev[4], s);
        launch_particle(c, 3, s);
        (void)hipEventRecord(ev[5], s);
        launch_deposit(c, c->d, 2, 1, s);
        (void)hipEventRecord(ev[6], s);
        launch_particle(c, 4, s);
        (void)hipEventRecord(ev[7], s);
        launch_deposit(c, c->d, 3, 0, s);
        tick3d<<<1, 64, 0, s>>>(c->d);
        (void)hipEventRecord(ev[8], s);
        hipError_t err = hipGetLastError();
        if (err == hipSuccess)
            err = hipEventSynchronize(ev[8]);
        for (int k = 0; k < 8 && err == hipSuccess; ++k) {
            float t = 0.f;
            err = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
        if (err != hipSuccess)
            rc = fail(FPIC_EHIP, std::string("profile: ") + hipGetErrorString(err));
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    for (int k = 0; k < 8; ++k)
        ms[k] = acc[k] / nsteps;
    return rc;
}

void destroy(Ctx3D *c)
{
    if (!c)
        return;
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    if (c->g1)
        (void)hipGraphExecDestroy(c->g1);
    if (c->gK)
        (void)hipGraphExecDestroy(c->gK);
    if (c->cap)
        (void)hipStreamDestroy(c->cap);
    if (c->hbuf)
        (void)hipHostFree(c->hbuf);
    delete c;
}

int autotune(const fpic_config &cfg, void *ws, size_t bytes, fpic_stream stream, fpic_tuning *best,
             double *ms_per_step)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_ms = 1e300;
    fpic_tuning bt{};
    int tried = 0;
    std::vector<std::pair<int, int>> cands;  // (waves, dirs per wave)
    for (int waves : {2, 4, 8})
        for (int groups : {1, 2, 4}) {
            const int dpw = (cfg.ndir + waves * groups - 1) / (waves * groups);
            if (dpw >= 1 && (groups == 1 || dpw > 1))
                cands.emplace_back(waves, dpw);
        }
    for (auto [waves, dpw] : cands) {
        fpic_tuning t{waves, dpw, 4, 0};
        Ctx3D *c = nullptr;
        int rc = create(cfg, &t, ws, bytes, stream, &c);
        if (rc)
            return rc;
        // any finite state times the same: zeros
        HIPCHECK(hipMemsetAsync(c->h.Y, 0, sizeof(double) * 18 * c->h.np, s));
        c->state_set = true;
        rc = step(c, 2);
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
        if (!rc)
            rc = step(c, 4);
        (void)hipEventRecord(e1, s);
        hipError_t es = hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        destroy(c);
        if (rc)
            return rc;
        if (es != hipSuccess)
            return fail(FPIC_EHIP, hipGetErrorString(es));
        ++tried;
        if (ms / 4 < best_ms) {
            best_ms = ms / 4;
            bt = t;
        }
    }
    if (!tried)
        return fail(FPIC_EINVAL, "no candidate launch shape");
    *best = bt;
    if (ms_per_step)
        *ms_per_step = best_ms;
    return FPIC_OK;
}

}  // namespace fpic3d
