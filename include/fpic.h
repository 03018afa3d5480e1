/*
 * fpic.h -- C ABI of libflavorpic: the hot path of the particle-in-cell
 * neutrino flavor method of Richers, Willcox, Ford & Myers, "Particle-in-cell
 * Simulation of the Neutrino Fast Flavor Instability" (arXiv:2101.02745),
 * as hand-written HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * What one step computes (Sec. II.B-II.C):
 *   for each of the four stages of classical RK4 (Sec. II.C),
 *     - deposit every particle's density matrices onto the grid with the
 *       linear (cloud-in-cell) or quadratic shape function (Sec. II.B.1,
 *       eq. pic_deposition), combined as n - nbar^* and f - fbar^*;
 *     - interpolate those moments back to every particle with the same
 *       weights (Sec. II.B.2, eq. pic_interpolation) and form
 *       H = H_vac + diag(V) + (n - nbar^*) - Omega.(f - fbar^*) and
 *       Hbar = H_vac^* - diag(V) - [(n - nbar^*) - Omega.(f - fbar^*)]^*
 *       (Sec. II.A, eq. potentials; V the background matter potential);
 *     - evaluate d rho/dt = -i [H, rho], d rhobar/dt = -i [Hbar, rhobar]
 *       (eq. eom) and form the next stage state.
 *
 * Conventions
 *   - Units: hbar = c = 1, sqrt(2) G_F = 1.
 *   - Every function returns FPIC_OK (0) or a negative FPIC_E* code and
 *     never throws; fpic_last_error() gives the calling thread's last message.
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary host memory.  Host arrays are copied
 *     before the call returns; the caller keeps ownership of everything.
 *   - Device work is enqueued on the stream given at creation (an
 *     hipStream_t passed as void*).  Only functions marked SYNC wait for it.
 *   - The caller owns one device workspace per context (size from
 *     fpic_workspace_bytes); the library never allocates device memory.
 *     The workspace must stay allocated until fpic_destroy.
 *
 * State layout (device or host, float64): state[18][ndir][ncell].  The 18
 * reals of a particle are rho_ee, rho_mumu, rho_tautau, Re/Im rho_emu,
 * Re/Im rho_etau, Re/Im rho_mutau, then the same nine for rhobar (only the
 * diagonal and the upper triangle are stored, Sec. II.B).  Cells are
 * numbered x fastest: cell = (z * ny + y) * nx + x.  Particle (d, c) is the
 * one with direction d that started at the centre of cell c (one particle
 * per direction per cell, Sec. III.A and App. B); at time t it has moved
 * Omega_d t.
 */
#ifndef FPIC_H
#define FPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPIC_OK 0
#define FPIC_EINVAL (-1)       /* bad argument or configuration */
#define FPIC_EHIP (-2)         /* a HIP runtime call failed */
#define FPIC_ESTATE (-3)       /* call out of order (e.g. step before set_state) */
#define FPIC_ENUMERIC (-4)     /* NaN/Inf or trace drift found by fpic_check */
#define FPIC_EUNSUPPORTED (-5) /* valid but not implemented (e.g. dt too large) */

typedef void *fpic_stream; /* hipStream_t */

/* A periodic box with one particle per direction per cell. */
typedef struct fpic_config {
    int32_t ncell[3];    /* cells along x, y, z; a 1D box is {1, 1, nz};
                            any other shape is a 3D box (at most 2^30
                            cells); boxes with nx <= 64 and the linear
                            shape take the fused stage kernels */
    double dx[3];        /* cell widths (cell volume dx*dy*dz) */
    int32_t ndir;        /* directions = particles per cell */
    const double *dirs;  /* host [ndir][3] unit vectors Omega_d */
    const double *N;     /* host [ndir] neutrinos per particle */
    const double *Nbar;  /* host [ndir] antineutrinos per particle */
    double hvac[18];     /* vacuum Hamiltonian, 3x3 complex Hermitian,
                            row-major (re, im) pairs, flavor basis */
    double vmat[3];      /* matter potentials V_e, V_mu, V_tau of the
                            background charged leptons (eq. potentials,
                            their rest frame): H gains diag(V), Hbar
                            -diag(V) (Hbar_mat = -H_mat^*, Sec. II.A);
                            0 = no matter */
    double dt;           /* time step; a stage may move no particle by a
                            whole cell: dt/2 * max|Omega_a| < dx_a */
    int32_t shape_order; /* 1 linear (cloud in cell); 2 quadratic
                            (triangular-shaped cloud, Sec. II.B.1) */
    int32_t flags;       /* reserved, 0 */
} fpic_config;

/* Launch shape.  Zero fields take the built-in choice; fpic_autotune
 * measures candidates on the device and returns the fastest. */
typedef struct fpic_tuning {
    int32_t waves;           /* 64-lane waves per workgroup: 1, 2, 4 or 8 */
    int32_t dirs_per_wave;   /* directions each wave sweeps, >= 1 */
    int32_t steps_per_graph; /* steps captured in one hipGraph, >= 1 */
    int32_t cache_policy;    /* 1D boxes and batches: 1 default caching; 2
                                streaming (nontemporal) loads and stores for
                                the data a stage does not read again soon,
                                which pays when one box's arrays overflow the
                                256 MB Infinity Cache; 0 chooses by size
                                (streaming for a single box of >= 64 MB of
                                state).  3D boxes always stream. */
    int32_t fused;           /* 3D boxes with the linear shape: 0 or 1 one
                                kernel per stage that also deposits, through
                                per-workgroup partial rows and a small
                                reduction; 2 a particle kernel and a deposit
                                kernel per stage (waves and dirs_per_wave
                                apply to these only).  Results differ by
                                rounding only.  Boxes with nx > 64 or more
                                than 1024 directions always take the
                                separate kernels.
                                1D boxes and batches: slopes formed again
                                from the state and the kept stage grids
                                instead of stored and read back.  1: stage 1
                                stores no slope, stages 2 and 4 form k1;
                                0: stage 2 stores none either, stages 3 and
                                4 form k1 and k2; 2: every slope stored.
                                Bitwise the same results.  Per particle-step
                                1360, 976 and 1744 B. */
} fpic_tuning;

typedef struct fpic_ctx fpic_ctx;

/* Bytes of device workspace fpic_create needs for this configuration. */
int fpic_workspace_bytes(const fpic_config *cfg, const fpic_tuning *tune, size_t *bytes);

/* Validate cfg, upload its tables into the workspace (device, caller-owned,
 * >= fpic_workspace_bytes, 256-byte aligned) and record the step graph.
 * tune may be NULL.  stream: hipStream_t for all later work. */
int fpic_create(const fpic_config *cfg, const fpic_tuning *tune, void *workspace,
                size_t workspace_bytes, fpic_stream stream, fpic_ctx **out);

/* Copy a state (device, [18][ndir][ncell]) in, set the step counter to
 * step0 (time step0*dt) and deposit the first-stage moments.  A state read
 * with fpic_get_state after step n and handed to a context of the same
 * configuration and launch shape with step0 = n continues bit for bit as
 * the uninterrupted run does (restart from a checkpoint). */
int fpic_set_state(fpic_ctx *ctx, const double *state, int64_t step0);

/* Copy the current state out (device, [18][ndir][ncell]). */
int fpic_get_state(fpic_ctx *ctx, double *state);

/* Advance nsteps >= 0 classical RK4 steps (Sec. II.C); asynchronous. */
int fpic_step(fpic_ctx *ctx, int64_t nsteps);

/* Deposit the four moment fields of the current state at the current time
 * (eq. pic_deposition, kept separate for neutrinos and antineutrinos):
 * out (device) [72][ncell] = n, f_x, f_y, f_z, nbar, fbar_x, fbar_y,
 * fbar_z, each as 9 packed reals per cell, per unit volume. */
int fpic_moments(fpic_ctx *ctx, double *out);

/* SYNC.  sum_p N_p rho_p and sum_p Nbar_p rhobar_p as 2 x 9 packed reals
 * (host out[18]). */
int fpic_flavor_totals(fpic_ctx *ctx, double *out);

/* SYNC.  Domain averages of the moment magnitudes (the quantities Sec. III.B
 * follows in time): from moments (device [72][ncell], as fpic_moments writes
 * them for this context), for each of n, f_x, nbar, fbar_x the mean over the
 * cells of |X_ee|, |X_mumu|, |X_tautau|, |X_emu|, |X_etau|, |X_mutau| (host
 * out[4][6]).  Fixed summation order. */
int fpic_domain_averages(fpic_ctx *ctx, const double *moments, double *out);

/* SYNC.  Largest |Tr rho - 1| and |Tr rhobar - 1| over all particles (host
 * *max_trace_err); returns FPIC_ENUMERIC if any state entry is NaN/Inf or
 * the trace error exceeds tol. */
int fpic_check(fpic_ctx *ctx, double tol, double *max_trace_err);

/* SYNC.  Current step number (time = step * dt). */
int fpic_get_step(fpic_ctx *ctx, int64_t *step);

/* SYNC.  Wait for all work enqueued by this context. */
int fpic_sync(fpic_ctx *ctx);

/* Free the context's host objects and graphs (not the workspace). */
void fpic_destroy(fpic_ctx *ctx);

/* SYNC.  Measurement: advance nsteps steps launching each kernel on its own
 * (outside the graph) with HIP events between launches, and return the mean
 * milliseconds per launch (host ms[8]) of: stage 1, its reduction, stage 2,
 * its reduction, stage 3, its reduction, stage 4, its reduction (3D boxes
 * with fused stages: each stage kernel, then the reduction of its partial
 * rows; 3D boxes with separate kernels: each stage's particle kernel, then
 * its deposit kernel). */
int fpic_profile(fpic_ctx *ctx, int32_t nsteps, double *ms);

/* Message of the calling thread's last failed call ("" if none). */
const char *fpic_last_error(void);

/* ---------------------------------------------------------------------
 * Batches: many independent 1D boxes of uneven size advanced together,
 * one launch per RK stage over a cost-sorted table of all their tiles,
 * the whole step captured in one hipGraph.  Each simulation keeps its own
 * dt, cell width, directions and weights.  Not in the paper: a throughput
 * device for parameter studies like its Sec. IV.
 * --------------------------------------------------------------------- */
typedef struct fpic_batch fpic_batch;

int fpic_batch_workspace_bytes(int32_t nsim, const fpic_config *cfgs,
                               const fpic_tuning *tune, size_t *bytes);
int fpic_batch_create(int32_t nsim, const fpic_config *cfgs, const fpic_tuning *tune,
                      void *workspace, size_t workspace_bytes, fpic_stream stream,
                      fpic_batch **out);
/* state (device) [18][ndir_sim][ncell_sim] of simulation sim */
int fpic_batch_set_state(fpic_batch *b, int32_t sim, const double *state, int64_t step0);
int fpic_batch_get_state(fpic_batch *b, int32_t sim, double *state);
int fpic_batch_step(fpic_batch *b, int64_t nsteps);
/* SYNC.  host out[nsim][18] */
int fpic_batch_flavor_totals(fpic_batch *b, double *out);
int fpic_batch_sync(fpic_batch *b);
void fpic_batch_destroy(fpic_batch *b);
/* SYNC.  As fpic_profile, for the batch's segmented launches (host ms[8]:
 * each stage kernel over all boxes, then its reduction). */
int fpic_batch_profile(fpic_batch *b, int32_t nsteps, double *ms);

/* ---------------------------------------------------------------------
 * Reverse mode (1D boxes, either shape order).  A hand-written discrete adjoint of the RK4
 * steps above (deposit, interpolation, Hamiltonians, commutators, stage
 * updates), with checkpointing: the forward pass stores the state every
 * ckpt_every steps; the backward pass recomputes each segment (storing its
 * stage slopes and moment grids) and sweeps it in reverse.  Not in the
 * paper: it gives d(loss)/d(initial state) and d(loss)/d(weights N, Nbar),
 * from which the caller forms gradients with respect to the densities,
 * fluxes and perturbation seeds of the initial condition.
 * --------------------------------------------------------------------- */
typedef struct fpic_adjoint_cfg {
    int64_t nsteps;     /* steps of the forward pass, >= 1 */
    int32_t ckpt_every; /* steps between stored states, >= 1 */
    int32_t reserved;
} fpic_adjoint_cfg;

/* Bytes of extra device workspace the adjoint needs for ctx and acfg. */
int fpic_adjoint_workspace_bytes(fpic_ctx *ctx, const fpic_adjoint_cfg *acfg, size_t *bytes);

/* Run acfg->nsteps steps from the context's current state (as fpic_step),
 * storing checkpoints in the adjoint workspace (device, caller-owned,
 * 256-byte aligned, kept until the backward pass). */
int fpic_adjoint_forward(fpic_ctx *ctx, const fpic_adjoint_cfg *acfg, void *workspace,
                         size_t workspace_bytes);

/* SYNC.  Given dL/d(final state) (device [18][ndir][ncell]), write
 * dL/d(state at the start of fpic_adjoint_forward) (device, same shape),
 * and dL/dN, dL/dNbar per direction (host [ndir] each).  The context keeps
 * its final state and step number. */
int fpic_adjoint_backward(fpic_ctx *ctx, const double *dL_dfinal, double *dL_dstart,
                          double *dL_dN, double *dL_dNbar);

/* ---------------------------------------------------------------------
 * Autotuning: time candidate launch shapes for cfg on the device (using a
 * scratch workspace of `bytes`, device) and return the fastest in *best
 * (host).  ms_per_step (host, may be NULL) receives its time.  SYNC.
 * --------------------------------------------------------------------- */
int fpic_autotune(int32_t nsim, const fpic_config *cfgs, void *workspace, size_t bytes,
                  fpic_stream stream, fpic_tuning *best, double *ms_per_step);

/* ---------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * --------------------------------------------------------------------- */
#define FPIC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20) /* 64 MiB per device */

/* SYNC.  The same as fpic_create (workspace, tune) + fpic_set_state(state,
 * step0) + fpic_step(nsteps) + fpic_get_state(state) + fpic_destroy, for a
 * 1D box (ncell = {1, 1, nz}), with identical results, but without any
 * device allocation and without a caller workspace: state (device,
 * [18][ndir][ncell], 8-byte aligned) is advanced in place, and every other
 * buffer lives in a fixed scratch array of FPIC_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device until the process ends.  The kernels are
 * launched one by one on `stream`, which must belong to the calling
 * thread's current device; the call returns when they have finished.
 * Errors: FPIC_EINVAL for a bad configuration or for a box whose buffers
 * exceed the scratch size (about 1.5e5 particles); FPIC_EUNSUPPORTED for
 * 3D boxes.  All calls on one device share its scratch array and leave
 * their data in it: calls that overlap in time on one device (other
 * threads, other streams) race and must be serialised by the caller. */
int fpic_step_noalloc(const fpic_config *cfg, const fpic_tuning *tune, double *state,
                      int64_t step0, int64_t nsteps, fpic_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* FPIC_H */
