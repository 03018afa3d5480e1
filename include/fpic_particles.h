/*
 * fpic_particles.h -- general particle placement for libflavorpic: the same
 * step as fpic.h (Sec. II.B-II.C: deposit, interpolation with the same
 * weights, Hamiltonians, commutator slopes, classical RK4), for particles
 * anywhere in the periodic box, any number per cell, each with its own
 * direction and weights (the general particle form of Sec. II.B).
 *
 * Positions.  A particle's direction never changes (eq. eom: dx/dt = Omega)
 * and RK4 integrates a constant velocity exactly, so its position at time t
 * is x0 + Omega t with x0 its position at t = 0.  Cell centres sit at
 * (j + 1/2) dx; along each axis with more than one cell, u = x / dx - 1/2,
 * the particle lies between centres floor(u) and floor(u) + 1 (periodic) at
 * fraction u - floor(u), and the linear or quadratic shape function
 * (Sec. II.B.1) spreads it over 2 or 3 cells per axis.  Every product and
 * sum in these position formulas is rounded once.
 *
 * Redistribution (Sec. II.C: particles are regrouped by cell as they move).
 * The library keeps its particles sorted by cell for locality: every
 * `sort_every` steps (and at the last step of every fpic_particles_step
 * call) the last Runge-Kutta stage writes each particle next to the other
 * particles of its new cell (a counting sort whose counts are taken before
 * that stage).  The order is internal: states go in and come out
 * in the caller's particle order.
 *
 * Deposits (and the flavor totals) are summed exactly: every contribution
 * is scaled by a power of two fixed at fpic_particles_set (from the
 * particle count and the largest weight) and rounded to an integer, the
 * integers are added as two 64-bit limbs with integer atomics, and the
 * exact sum is rounded once to a double.  Results are therefore bitwise
 * the same from run to run and whatever order the caller gives the
 * particles in; a contribution's rounding error is at most 2^-84 of
 * 16 npart max(|N| + |Nbar|)/dV.  The flag FPIC_PFLOAT_ATOMICS trades this
 * for speed (floating-point atomics; flavor totals stay exact).
 *
 * Conventions are those of fpic.h: FPIC_* status codes, fpic_last_error(),
 * caller-owned device workspace, all device work on the stream given at
 * creation, SYNC marks functions that wait for it.
 *
 * Layouts (device, float64 unless stated): pos0[3][npart] and
 * dirs[3][npart] (x components of all particles, then y, then z);
 * N[npart], Nbar[npart]; state[18][npart] with the 18 reals of fpic.h.
 */
#ifndef FPIC_PARTICLES_H
#define FPIC_PARTICLES_H

#include <stddef.h>
#include <stdint.h>

#include "fpic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* fpic_pconfig.flags: deposit with floating-point atomics instead of the
 * exact limb sums.  Faster, but the sums then depend on the order in which
 * the atomics land: results agree run to run only up to rounding. */
#define FPIC_PFLOAT_ATOMICS 1

typedef struct fpic_pconfig {
    int32_t ncell[3];     /* cells along x, y, z (1D: {1, 1, nz}); >= 1 each */
    double dx[3];         /* cell widths */
    int64_t npart;        /* particles, 1 .. 2^31 - 1 */
    double hvac[18];      /* vacuum Hamiltonian as in fpic_config */
    double vmat[3];       /* matter potentials as in fpic_config */
    double dt;            /* time step, > 0 */
    int32_t shape_order;  /* 1 linear (cloud in cell), 2 quadratic */
    int32_t sort_every;   /* steps between sorts by cell, 1..1024; 0: 4 */
    int32_t flags;        /* 0, or FPIC_PFLOAT_ATOMICS */
    int32_t reserved;
} fpic_pconfig;

typedef struct fpic_pctx fpic_pctx;

/* Bytes of device workspace fpic_particles_create needs. */
int fpic_particles_workspace_bytes(const fpic_pconfig *cfg, size_t *bytes);

/* Validate cfg, lay out the workspace (device, caller-owned, 256-byte
 * aligned, >= fpic_particles_workspace_bytes) and record the step graphs. */
int fpic_particles_create(const fpic_pconfig *cfg, void *workspace, size_t workspace_bytes,
                          fpic_stream stream, fpic_pctx **out);

/* SYNC.  Copy the particles in (device arrays, caller order, see the
 * layouts above): positions at t = 0, unit directions, weights N and Nbar
 * (neutrinos and antineutrinos per particle) and the state at step step0
 * (time step0*dt); sort them by cell and deposit the first-stage moments.
 * FPIC_EINVAL if a position or weight is not finite or a direction is not a
 * unit vector (|Omega|^2 within 1e-9 of 1); with exact sums,
 * FPIC_EUNSUPPORTED if 16 npart max(|N| + |Nbar|)/dV lies outside about
 * 2^-816 .. 2^984 (the range of the fixed-point scale).  With exact sums, a
 * state read with fpic_particles_get_state after step n and handed back with
 * the same particles and step0 = n continues bit for bit as the
 * uninterrupted run does. */
int fpic_particles_set(fpic_pctx *ctx, const double *pos0, const double *dirs, const double *N,
                       const double *Nbar, const double *state, int64_t step0);

/* Copy the current state out in the caller's particle order (device
 * [18][npart]). */
int fpic_particles_get_state(fpic_pctx *ctx, double *state);

/* Advance nsteps >= 0 RK4 steps; asynchronous. */
int fpic_particles_step(fpic_pctx *ctx, int64_t nsteps);

/* The four moment fields at the current time, as fpic_moments: out
 * (device) [72][ncell]. */
int fpic_particles_moments(fpic_pctx *ctx, double *out);

/* SYNC.  sum_p N_p rho_p and sum_p Nbar_p rhobar_p (host out[18]). */
int fpic_particles_flavor_totals(fpic_pctx *ctx, double *out);

/* SYNC.  As fpic_check. */
int fpic_particles_check(fpic_pctx *ctx, double tol, double *max_trace_err);

/* SYNC.  Current step number. */
int fpic_particles_get_step(fpic_pctx *ctx, int64_t *step);

/* SYNC.  Wait for all work enqueued by this context. */
int fpic_particles_sync(fpic_pctx *ctx);

/* SYNC.  Measurement: advance nsteps steps launching each kernel on its own
 * with HIP events between launches, sorting after every step; host ms[6]:
 * mean milliseconds of stage 1, 2, 3, 4 (which also moves every particle to
 * its sorted place, and updates the step counter), the sort's counting and
 * scan, and the whole step. */
int fpic_particles_profile(fpic_pctx *ctx, int32_t nsteps, double *ms);

/* Free the context's host objects and graphs (not the workspace). */
void fpic_particles_destroy(fpic_pctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FPIC_PARTICLES_H */
