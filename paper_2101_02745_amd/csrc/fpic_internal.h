// Internal declarations shared by the HIP kernels and the host runtime of
// libflavorpic.  Not part of the public ABI (see include/fpic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace fpic {

// Cells per tile = lanes per wave: lane l of every wave of a workgroup owns
// cell tile*TILE + l, so one wave's loads of one direction are contiguous.
constexpr int TILE = 64;
// Combined moments per cell: A = n - nbar^* (9 packed reals), then
// B_x, B_y, B_z = f_i - fbar_i^* (9 each).
constexpr int NG = 36;
// Staged grid tile: cells tile*TILE-1 .. tile*TILE+65 (67 cells, padded)
// for the linear shape function; tile*TILE-2 .. tile*TILE+66 for the
// quadratic one (gt_cells(sh)).
constexpr int GT_CELLS = 67;
constexpr int GT_STRIDE = 68;
constexpr int gt_cells(int sh) { return TILE + 2 * sh + 1; }
constexpr int gt_stride(int sh) { return gt_cells(sh) + 1; }
// Edge partials per tile and direction group: the linear deposit leaves the
// tile only to the right (one cell); the quadratic one two cells to the
// right and one to the left (slots 0, 1: right; 2: left).
constexpr int n_edges(int sh) { return sh == 2 ? 3 : 1; }
constexpr int MAX_WAVES = 8;
// Reals stored per Runge-Kutta slope.  A slope k = -i[H, rho] is traceless
// (the trace of a commutator vanishes), so its first diagonal entry is kept
// as -(k_11 + k_22) and only the other 8 + 8 reals of k and kbar are stored:
// slot q < 8 holds packed component q + 1, slot q >= 8 component q + 2.
constexpr int NK = 16;

enum Mode : int {
    M_S1 = 1,       // RK stage 1: k1 = F(Y), deposit Y + dt/2 k1
    M_S2 = 2,       // stage 2: k2 = F(Y + dt/2 k1), deposit Y + dt/2 k2
    M_S3 = 3,       // stage 3: k3 = F(Y + dt/2 k2), deposit Y + dt k3
    M_S4 = 4,       // stage 4: k4 = F(Y + dt k3), Y += dt/6 (k1+2k2+2k3+k4),
                    //          deposit the new Y (first stage of next step)
    M_DEPOSIT = 5,  // deposit Y at the current step time
    M_MOM_NU = 6,   // deposit N rho alone (moments n, f)
    M_MOM_NUBAR = 7 // deposit Nbar rhobar alone (moments nbar, fbar)
};

// reduction targets: 0..4 -> G[which], RED_GA -> GA, RED_OUT -> explicit
constexpr int RED_GA = 5;
constexpr int RED_OUT = 6;

// One 1D simulation as the kernels see it.  All pointers are device
// pointers into the caller's workspace.
struct SimDesc {
    int32_t ncell;   // cells along z
    int32_t ndir;    // directions
    int32_t ntile;   // ceil(ncell / TILE)
    int32_t ngroup;  // direction groups = workgroups per tile
    int32_t dpw;     // directions per wave
    int32_t dpg;     // directions per group = waves * dpw
    int32_t shape;   // shape-function order: 1 linear, 2 quadratic
    int32_t pad_;
    int64_t np;      // particles = ndir * ncell
    double dt;       // time step
    double dz;       // cell width
    double hvac[9];  // constant part of H: vacuum + matter, packed (diag, Re/Im upper)
    double hvacb[9]; // constant part of Hbar before conjugation: vacuum - matter
    const double *vx, *vy, *vz;  // [ndir] direction components
    const double *wN, *wNb;      // [ndir] N / dV, Nbar / dV
    const double *Nw, *Nbw;      // [ndir] N, Nbar
    double *Y;                   // [18][ndir][ncell] state
    double *Yout;                // where stage 4 writes the new state (normally Y)
    double *K1, *K2, *K3;        // [18][ndir][ncell] stage slopes
    // [36][ncell] deposited moments: stage s reads G[s-1]; the reduction
    // after stage s writes G[s] (G[4] is the next step's G[0]).  A single
    // box cycles four buffers, {g0, g1, g2, g3, g0}, so that the stage-1 and
    // stage-2 grids are still there when stage 4 forms k1 and k2 again.
    double *G[5];
    double *part;                // [ngroup][36][ntile*TILE] per-group partials
    double *edge;                // [ngroup][36][n_edges][ntile] edge partials
    double *red;                 // [nred][18] scratch for reductions
    int64_t *step;               // current step number
    // adjoint (reverse-mode) buffers, null outside the adjoint
    double *GA;                  // [36][ncell] deposited adjoint sources
    double *lam[2];              // [18][ndir][ncell] lambda of step n lives in lam[n & 1]
    double *lcur;                // [18][ndir][ncell] lambda of the latest stage state
    double *dres;                // [18][ndir][ncell] direct part of a stage adjoint
    double *dwN, *dwNb;          // [ndir][ntile] gradients w.r.t. N/dV, Nbar/dV
};

struct WorkItem {
    int32_t sim, tile, group, pad;
};

struct RedItem {
    int32_t sim, tile;
};

// Launchers (fpic_1d.hip).
// stream_policy: streaming cache policy for the data a stage does not read
// again soon (large boxes), else the default policy.  reform: 0 every slope
// stored and read back; 1 stage 1 stores no slope and stages 2 and 4 form k1
// again from the state and G[0]; 2 stage 2 stores none either and stages 3
// and 4 form k1 and k2 again (G[1] as well); G[0] and G[1] must stay intact
// until stage 4
hipError_t launch_stage1d(int mode, const WorkItem *work, int nwork, const SimDesc *sims,
                          int waves, int max_dpw, int shape, bool stream_policy, int reform,
                          hipStream_t s);
hipError_t launch_reduce1d(const RedItem *items, int nitems, const SimDesc *sims, int which,
                           double *override_out, int tick, hipStream_t s);
// adjoint kernels: kind 4 = sources of stage 4 and their deposit; kind 3, 2,
// 1 = gather of the sources of stage kind+1 (stage lambda, step lambda,
// weight gradients) fused with the sources of stage kind; kind 0 = gather of
// the sources of stage 1
hipError_t launch_adj1d(int kind, const WorkItem *work, int nwork, const SimDesc *sims, int waves,
                        int max_dpw, int shape, hipStream_t s);
hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s);
hipError_t launch_tick(const SimDesc *sims, int64_t delta, hipStream_t s);
hipError_t launch_tile_sum(const double *src, int ndir, int ntile, double scale, double *dst,
                           hipStream_t s);
hipError_t launch_set_step(const SimDesc *sims, int sim_lo, int sim_hi, int64_t value,
                           hipStream_t s);
hipError_t launch_totals(const SimDesc *sims, int sim, int nblk, double *out18, hipStream_t s);
hipError_t launch_check(const SimDesc *sims, int sim, int nblk, double *out2, hipStream_t s);
hipError_t launch_fill_state(const SimDesc *sims, int sim, hipStream_t s);

size_t stage1d_smem_bytes(int waves, int max_dpw, int shape);

// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string &msg);

}  // namespace fpic
