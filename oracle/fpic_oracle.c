/*
 * fpic_oracle.c -- plain CPU FP64 reference of the particle-in-cell neutrino
 * flavor method of Richers, Willcox, Ford & Myers, "Particle-in-cell
 * Simulation of the Neutrino Fast Flavor Instability" (arXiv:2101.02745).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the HIP library: it reads the same input *arrays*
 * and nothing else.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   - every particle's density matrices are unpacked into full 3x3 complex
 *     matrices (Sec. II.B stores only the upper triangle);
 *   - deposition follows eq. pic_deposition literally: four moment fields
 *     n, f, nbar, fbar, one particle after another, in particle order;
 *   - interpolation follows eq. pic_interpolation with the same weights;
 *   - the Hamiltonians follow eq. potentials and the antineutrino
 *     conventions of Sec. II.A (Hbar_vac = H_vac^*, Hbar_mat = -H_mat^*,
 *     Hbar_nunu = -H_nunu^*); the matter term is the diagonal potential
 *     V_a = sqrt(2) G_F (n_a - nbar_a) of the background charged leptons in
 *     their rest frame (zero lepton flux), an input;
 *   - the right-hand side is eq. eom, d rho/dt = -i [H, rho], with both
 *     products H rho and rho H formed as full matrix products;
 *   - time integration is the classical fourth-order Runge-Kutta method
 *     (Sec. II.C), all particles together.
 *
 * Units: hbar = c = 1 and sqrt(2) G_F = 1 (densities in units of the
 * reference density, so the self-interaction strength mu is 1).
 *
 * Particle positions.  A particle starts at the centre of its cell and its
 * direction never changes (eq. eom: dx/dt = Omega), so its position at time
 * t is x0 + Omega t.  Runge-Kutta integrates a constant velocity exactly, so
 * the oracle uses that closed form at every stage time.  Along each axis the
 * displacement measured in cells is u = (Omega_a t) / dx_a; the particle
 * lies between the centres of cells (c_a + floor(u)) and (c_a + floor(u) + 1)
 * (periodic), at fraction phi = u - floor(u) of the way.  The linear
 * ("cloud in cell", first-order) shape function then gives weight 1 - phi to
 * the first and phi to the second (Sec. II.B.1 shape functions; order 1);
 * the quadratic one (order 2, the paper's production choice) spreads the
 * particle over the nearest cell centre and its two neighbours.
 * Along an axis with a single cell the particle always lies in cell 0.
 * Stage times are t = n dt + c_s dt with c_s in {0, 1/2, 1/2, 1}, each
 * product and sum rounded once (this file is compiled with
 * -ffp-contract=off).
 *
 * General placement.  A problem may instead list npart particles with their
 * own positions x0 at t = 0, directions and weights (the general particle
 * form of Sec. II.B: particles anywhere in the box, any number per cell).
 * The position at time t is again x0 + Omega t; cell centres sit at
 * (j + 1/2) dx, so along each axis u = x / dx - 1/2, the first cell is
 * floor(u) (periodic) and phi = u - floor(u).  Which cell a particle is
 * stored with does not enter: every particle is deposited and interpolated
 * where it is.
 *
 * State layout: state[18][ndir][ncell], see the input-generator module; the
 * particle with direction d starting in cell c is (d, c); cells are numbered
 * x fastest.  With general placement: state[18][npart].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int64_t ncell[3];   /* cells along x, y, z */
    double dx[3];       /* cell widths */
    int64_t ndir;       /* directions (particles per cell) */
    const double *dirs; /* [ndir][3] unit vectors Omega */
    const double *N;    /* [ndir] neutrinos per particle */
    const double *Nbar; /* [ndir] antineutrinos per particle */
    const double *Hvac; /* [3][3] complex, row-major (re, im) pairs */
    double dt;
    const double *Vmat; /* [3] matter potential V_e, V_mu, V_tau, or NULL (none) */
    int32_t shape_order; /* 1 linear (cloud in cell), 2 quadratic */
    /* general placement: when pos0 is not NULL the particles are these
     * npart ones and ndir, dirs, N, Nbar are not used */
    int64_t npart;
    const double *pos0;  /* [npart][3] positions at t = 0 */
    const double *pdirs; /* [npart][3] unit vectors Omega */
    const double *pN;    /* [npart] neutrinos per particle */
    const double *pNbar; /* [npart] antineutrinos per particle */
} oracle_problem;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */
static int64_t ncell_total(const oracle_problem *P)
{
    return P->ncell[0] * P->ncell[1] * P->ncell[2];
}

static int64_t pmod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

static int64_t nparticles(const oracle_problem *P)
{
    return P->pos0 ? P->npart : P->ndir * ncell_total(P);
}

/* Direction and weights of particle p (lattice: p = d * ncell + c). */
static const double *particle_dir(const oracle_problem *P, int64_t p)
{
    return P->pos0 ? P->pdirs + 3 * p : P->dirs + 3 * (p / ncell_total(P));
}

static double particle_N(const oracle_problem *P, int64_t p)
{
    return P->pos0 ? P->pN[p] : P->N[p / ncell_total(P)];
}

static double particle_Nbar(const oracle_problem *P, int64_t p)
{
    return P->pos0 ? P->pNbar[p] : P->Nbar[p / ncell_total(P)];
}

/* Unpack the 9 stored reals (diagonal, then Re/Im of the e-mu, e-tau and
 * mu-tau entries) of a Hermitian matrix; consecutive reals are `stride`
 * doubles apart. */
static void unpack(const double *s, int64_t stride, cplx m[3][3])
{
    m[0][0] = s[0 * stride];
    m[1][1] = s[1 * stride];
    m[2][2] = s[2 * stride];
    m[0][1] = s[3 * stride] + I * s[4 * stride];
    m[0][2] = s[5 * stride] + I * s[6 * stride];
    m[1][2] = s[7 * stride] + I * s[8 * stride];
    m[1][0] = conj(m[0][1]);
    m[2][0] = conj(m[0][2]);
    m[2][1] = conj(m[1][2]);
}

/* Store the diagonal (real part) and the upper triangle of m. */
static void pack(cplx m[3][3], double *s, int64_t stride)
{
    s[0 * stride] = creal(m[0][0]);
    s[1 * stride] = creal(m[1][1]);
    s[2 * stride] = creal(m[2][2]);
    s[3 * stride] = creal(m[0][1]);
    s[4 * stride] = cimag(m[0][1]);
    s[5 * stride] = creal(m[0][2]);
    s[6 * stride] = cimag(m[0][2]);
    s[7 * stride] = creal(m[1][2]);
    s[8 * stride] = cimag(m[1][2]);
}

static void matmul(cplx a[3][3], cplx b[3][3], cplx out[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++)
                s += a[i][k] * b[k][j];
            out[i][j] = s;
        }
}

/* -i [H, rho] = -i (H rho - rho H) */
static void commutator_rhs(cplx H[3][3], cplx rho[3][3], cplx out[3][3])
{
    cplx Hr[3][3], rH[3][3];
    matmul(H, rho, Hr);
    matmul(rho, H, rH);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            out[i][j] = -I * (Hr[i][j] - rH[i][j]);
}

static void load_hvac(const oracle_problem *P, cplx H[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            H[i][j] = P->Hvac[2 * (3 * i + j)] + I * P->Hvac[2 * (3 * i + j) + 1];
}

static void load_vmat(const oracle_problem *P, double V[3])
{
    for (int a = 0; a < 3; a++)
        V[a] = P->Vmat ? P->Vmat[a] : 0.0;
}

/* ------------------------------------------------------------------ */
/* shape function                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    int64_t cell[27];
    double w[27];
} stencil;

/* Along one axis with n > 1 cells: the particle lies a fraction phi of the
 * way from the centre of cell `left` to the next.  Writes the first cell of
 * the axis stencil and its weights; returns the stencil width. */
static int linear_axis(int64_t left, double phi, int64_t n, int64_t *first, double w[3])
{
    *first = left % n;
    w[0] = 1.0 - phi;
    w[1] = phi;
    return 2;
}

/* Quadratic (triangular-shaped cloud) weights: with j the nearest cell
 * centre and xi = x - x_j in [-1/2, 1/2), cells j - 1, j, j + 1 get
 * (1/2 - xi)^2 / 2, 3/4 - xi^2 and (1/2 + xi)^2 / 2. */
static int quadratic_axis(int64_t left, double phi, int64_t n, int64_t *first, double w[3])
{
    const int up = phi < 0.5 ? 0 : 1;   /* nearest centre: left or left + 1 */
    const double xi = up ? phi - 1.0 : phi;
    *first = pmod(left + up - 1, n);
    w[0] = 0.5 * ((0.5 - xi) * (0.5 - xi));
    w[1] = 0.75 - xi * xi;
    w[2] = 0.5 * ((0.5 + xi) * (0.5 + xi));
    return 3;
}

/* Cells touched by particle p at time t and their weights w_pj: the
 * tensor product of the per-axis weights of the shape function of order
 * P->shape_order (1 linear, 2 quadratic; Sec. II.B.1). */
static void shape_stencil(const oracle_problem *P, int64_t p, double t, stencil *S)
{
    const int64_t nx = P->ncell[0], ny = P->ncell[1], nc = ncell_total(P);
    const int64_t d = p / nc, c = p % nc;
    int64_t home[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
    int64_t first[3];
    double wa[3][3];
    int cnt[3];
    for (int a = 0; a < 3; a++) {
        if (P->ncell[a] == 1) {
            first[a] = 0;
            wa[a][0] = 1.0;
            cnt[a] = 1;
            continue;
        }
        double u, fl, phi;
        int64_t left;
        if (P->pos0) {
            const double x = P->pos0[3 * p + a] + P->pdirs[3 * p + a] * t;
            u = x / P->dx[a] - 0.5;
            fl = floor(u);
            phi = u - fl;
            left = pmod((int64_t)fl, P->ncell[a]);
        } else {
            u = (P->dirs[3 * d + a] * t) / P->dx[a];
            fl = floor(u);
            phi = u - fl;
            left = pmod(home[a] + (int64_t)fl, P->ncell[a]);
        }
        cnt[a] = (P->shape_order == 2) ? quadratic_axis(left, phi, P->ncell[a], &first[a], wa[a])
                                       : linear_axis(left, phi, P->ncell[a], &first[a], wa[a]);
    }
    S->n = 0;
    for (int bz = 0; bz < cnt[2]; bz++)
        for (int by = 0; by < cnt[1]; by++)
            for (int bx = 0; bx < cnt[0]; bx++) {
                int64_t ix = (first[0] + bx) % P->ncell[0];
                int64_t iy = (first[1] + by) % P->ncell[1];
                int64_t iz = (first[2] + bz) % P->ncell[2];
                double w = wa[0][bx] * wa[1][by];
                w = w * wa[2][bz];
                S->cell[S->n] = (iz * ny + iy) * nx + ix;
                S->w[S->n] = w;
                S->n++;
            }
}

/* ------------------------------------------------------------------ */
/* deposition (eq. pic_deposition)                                      */
/* ------------------------------------------------------------------ */
/* Moment fields, per cell: n[3][3], f[axis][3][3], nbar, fbar. */
typedef struct {
    cplx n[3][3];
    cplx f[3][3][3];
    cplx nb[3][3];
    cplx fb[3][3][3];
} moments;

/* Add particle p's contributions (eq. pic_deposition) into grid g. */
static void deposit_particle(const oracle_problem *P, const double *state, double t,
                             int64_t p, moments *grid)
{
    const int64_t np = nparticles(P);
    const double *v = particle_dir(P, p);
    const double N = particle_N(P, p), Nb = particle_Nbar(P, p);
    cplx rho[3][3], rhob[3][3];
    unpack(state + p, np, rho);
    unpack(state + 9 * np + p, np, rhob);
    stencil S;
    shape_stencil(P, p, t, &S);
    for (int s = 0; s < S.n; s++) {
        moments *g = grid + S.cell[s];
        const double wN = S.w[s] * N;
        const double wNb = S.w[s] * Nb;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                g->n[i][j] += wN * rho[i][j];
                g->nb[i][j] += wNb * rhob[i][j];
                for (int a = 0; a < 3; a++) {
                    g->f[a][i][j] += wN * rho[i][j] * v[a];
                    g->fb[a][i][j] += wNb * rhob[i][j] * v[a];
                }
            }
    }
}

/* Number of particle ranges the deposition sum is split into.  It depends
 * on the problem size only, never on the thread count: at most 64 ranges of
 * at least 4096 particles, and at most 4 GiB of range grids.  Problems of
 * fewer than 8192 particles are summed in one range, in particle order. */
static int64_t deposit_ranges(const oracle_problem *P)
{
    const int64_t np = nparticles(P);
    const double grid_bytes = (double)sizeof(moments) * (double)ncell_total(P);
    int64_t k = np / 4096;
    if (k > 64)
        k = 64;
    while (k > 1 && (double)k * grid_bytes > 4294967296.0)
        k--;
    return k < 1 ? 1 : k;
}

/* A grid buffer for deposit(): the moment fields of every cell, followed
 * by one grid per particle range when there is more than one range. */
static moments *grid_alloc(const oracle_problem *P)
{
    const int64_t nr = deposit_ranges(P);
    return malloc(sizeof(moments) * (size_t)ncell_total(P) * (size_t)(nr > 1 ? nr + 1 : 1));
}

/* Moment fields of eq. pic_deposition at time t into grid[0 .. ncell), a
 * buffer from grid_alloc().  The sum over particles is split into
 * deposit_ranges() contiguous ranges of the particle index; each range is
 * summed in particle order into a grid of its own, and the range grids are
 * then added cell by cell in range order, so the result is the same
 * whatever the number of threads. */
static void deposit(const oracle_problem *P, const double *state, double t,
                    moments *grid)
{
    const int64_t nc = ncell_total(P), np = nparticles(P);
    const double dV = P->dx[0] * P->dx[1] * P->dx[2];
    const int64_t nr = deposit_ranges(P);
    moments *part = nr > 1 ? grid + nc : grid;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) if (nr > 1)
#endif
    for (int64_t r = 0; r < nr; r++) {
        const int64_t p0 = np * r / nr, p1 = np * (r + 1) / nr;
        memset(part + r * nc, 0, sizeof(moments) * (size_t)nc);
        for (int64_t p = p0; p < p1; p++)
            deposit_particle(P, state, t, p, part + r * nc);
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (nc * nr >= 4096)
#endif
    for (int64_t c = 0; c < nc; c++) {
        moments *g = grid + c;
        if (nr > 1) {
            *g = part[c];
            for (int64_t r = 1; r < nr; r++) {
                const moments *q = part + r * nc + c;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        g->n[i][j] += q->n[i][j];
                        g->nb[i][j] += q->nb[i][j];
                        for (int a = 0; a < 3; a++) {
                            g->f[a][i][j] += q->f[a][i][j];
                            g->fb[a][i][j] += q->fb[a][i][j];
                        }
                    }
            }
        }
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                g->n[i][j] /= dV;
                g->nb[i][j] /= dV;
                for (int a = 0; a < 3; a++) {
                    g->f[a][i][j] /= dV;
                    g->fb[a][i][j] /= dV;
                }
            }
    }
}

/* ------------------------------------------------------------------ */
/* interpolation, Hamiltonians, right-hand side                         */
/* ------------------------------------------------------------------ */
static void interpolate(const moments *grid, const stencil *S, moments *out)
{
    memset(out, 0, sizeof(moments));
    for (int s = 0; s < S->n; s++) {
        const moments *g = grid + S->cell[s];
        const double w = S->w[s];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                out->n[i][j] += w * g->n[i][j];
                out->nb[i][j] += w * g->nb[i][j];
                for (int a = 0; a < 3; a++) {
                    out->f[a][i][j] += w * g->f[a][i][j];
                    out->fb[a][i][j] += w * g->fb[a][i][j];
                }
            }
    }
}

/* Hamiltonians of a particle with direction v from its interpolated
 * moments (eq. potentials):
 *   H_nunu = (n - nbar^*) - v.(f - fbar^*),  H_mat = diag(V),
 *   H = H_vac + H_mat + H_nunu,
 *   Hbar = H_vac^* - H_mat^* - H_nunu^*  (antineutrino conventions of
 *   Sec. II.A). */
static void hamiltonians(const moments *m, const double *v, cplx Hv[3][3], const double Vm[3],
                         cplx H[3][3], cplx Hb[3][3])
{
    cplx Hnn[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx h = m->n[i][j] - conj(m->nb[i][j]);
            for (int a = 0; a < 3; a++)
                h -= v[a] * (m->f[a][i][j] - conj(m->fb[a][i][j]));
            Hnn[i][j] = h;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            H[i][j] = Hv[i][j] + Hnn[i][j];
            Hb[i][j] = conj(Hv[i][j]) - conj(Hnn[i][j]);
        }
    for (int a = 0; a < 3; a++) {
        H[a][a] += Vm[a];
        Hb[a][a] -= Vm[a];
    }
}

/* Right-hand side of eq. eom for every particle at time t. */
static void rhs(const oracle_problem *P, const double *state, double t,
               moments *grid, double *out)
{
    const int64_t np = nparticles(P);
    cplx Hv[3][3];
    double Vm[3];
    load_hvac(P, Hv);
    load_vmat(P, Vm);
    deposit(P, state, t, grid);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (np >= 4096)
#endif
    for (int64_t p = 0; p < np; p++) {
        const double *v = particle_dir(P, p);
        stencil S;
        shape_stencil(P, p, t, &S);
        moments m;
        interpolate(grid, &S, &m);
        cplx H[3][3], Hb[3][3];
        hamiltonians(&m, v, Hv, Vm, H, Hb);
        cplx rho[3][3], rhob[3][3], k[3][3], kb[3][3];
        unpack(state + p, np, rho);
        unpack(state + 9 * np + p, np, rhob);
        commutator_rhs(H, rho, k);
        commutator_rhs(Hb, rhob, kb);
        pack(k, out + p, np);
        pack(kb, out + 9 * np + p, np);
    }
}

static double stage_time(int64_t n, double dt, double c)
{
    double tn = (double)n * dt;
    return tn + c * dt;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* One evaluation of the right-hand side at time t; out has the state's
 * shape. */
int oracle_rhs(const oracle_problem *P, const double *state, double t, double *out)
{
    moments *grid = grid_alloc(P);
    if (!grid)
        return -1;
    rhs(P, state, t, grid, out);
    free(grid);
    return 0;
}

/* nsteps classical RK4 steps, in place, starting at step number n0
 * (time n0 * dt). */
int oracle_step(const oracle_problem *P, double *state, int64_t n0, int64_t nsteps)
{
    const int64_t len = 18 * nparticles(P);
    const double dt = P->dt;
    moments *grid = grid_alloc(P);
    double *k = malloc(sizeof(double) * (size_t)len);
    double *ks = malloc(sizeof(double) * (size_t)len);
    double *ys = malloc(sizeof(double) * (size_t)len);
    if (!grid || !k || !ks || !ys) {
        free(grid); free(k); free(ks); free(ys);
        return -1;
    }
    for (int64_t n = n0; n < n0 + nsteps; n++) {
        /* k1 */
        rhs(P, state, stage_time(n, dt, 0.0), grid, k);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (len >= 65536)
#endif
        for (int64_t i = 0; i < len; i++) {
            ks[i] = k[i];
            ys[i] = state[i] + (0.5 * dt) * k[i];
        }
        /* k2 */
        rhs(P, ys, stage_time(n, dt, 0.5), grid, k);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (len >= 65536)
#endif
        for (int64_t i = 0; i < len; i++) {
            ks[i] = ks[i] + 2.0 * k[i];
            ys[i] = state[i] + (0.5 * dt) * k[i];
        }
        /* k3 */
        rhs(P, ys, stage_time(n, dt, 0.5), grid, k);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (len >= 65536)
#endif
        for (int64_t i = 0; i < len; i++) {
            ks[i] = ks[i] + 2.0 * k[i];
            ys[i] = state[i] + dt * k[i];
        }
        /* k4 */
        rhs(P, ys, stage_time(n, dt, 1.0), grid, k);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (len >= 65536)
#endif
        for (int64_t i = 0; i < len; i++) {
            ks[i] = ks[i] + k[i];
            state[i] = state[i] + (dt / 6.0) * ks[i];
        }
    }
    free(grid); free(k); free(ks); free(ys);
    return 0;
}

/* The four moment fields at time t, out[72][ncell]: n, f_x, f_y, f_z,
 * nbar, fbar_x, fbar_y, fbar_z, each as 9 packed reals. */
int oracle_moments(const oracle_problem *P, const double *state, double t, double *out)
{
    const int64_t nc = ncell_total(P);
    moments *grid = grid_alloc(P);
    if (!grid)
        return -1;
    deposit(P, state, t, grid);
    for (int64_t c = 0; c < nc; c++) {
        moments *g = grid + c;
        pack(g->n, out + 0 * 9 * nc + c, nc);
        for (int a = 0; a < 3; a++)
            pack(g->f[a], out + (1 + a) * 9 * nc + c, nc);
        pack(g->nb, out + 4 * 9 * nc + c, nc);
        for (int a = 0; a < 3; a++)
            pack(g->fb[a], out + (5 + a) * 9 * nc + c, nc);
    }
    free(grid);
    return 0;
}

/* Interpolate an arbitrary cell field G[ncomp][ncell] to every particle
 * at time t (eq. pic_interpolation applied component-wise):
 * out[ncomp][ndir][ncell]. */
int oracle_gather(const oracle_problem *P, const double *G, int64_t ncomp, double t,
                  double *out)
{
    const int64_t nc = ncell_total(P), np = nparticles(P);
    for (int64_t p = 0; p < np; p++) {
        stencil S;
        shape_stencil(P, p, t, &S);
        for (int64_t q = 0; q < ncomp; q++) {
            double s = 0.0;
            for (int i = 0; i < S.n; i++)
                s += S.w[i] * G[q * nc + S.cell[i]];
            out[q * np + p] = s;
        }
    }
    return 0;
}

/* Sum over particles of N rho and Nbar rhobar: out[2][9] packed reals. */
int oracle_flavor_totals(const oracle_problem *P, const double *state, double *out)
{
    const int64_t np = nparticles(P);
    for (int k = 0; k < 18; k++)
        out[k] = 0.0;
    for (int64_t p = 0; p < np; p++)
        for (int k = 0; k < 9; k++) {
            out[k] += particle_N(P, p) * state[k * np + p];
            out[9 + k] += particle_Nbar(P, p) * state[(9 + k) * np + p];
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* reverse mode (reference adjoint)                                     */
/* ------------------------------------------------------------------ */
/* The discrete adjoint of the steps above, derived independently of any
 * other implementation: every operation's transpose is written out with
 * full complex matrices.  A real-valued loss L depends on a Hermitian
 * matrix M through its packed reals m; a matrix cotangent X means
 * dL = Re Tr(X^dagger dM).  Conversions:
 *   packed gradient of X:  (Re X_aa, Re X_ab + Re X_ba, Im X_ab - Im X_ba)
 *   matrix form of a packed cotangent g (used for the slopes):
 *                          X_aa = g_aa, X_ab = (g_re + i g_im) / 2,
 *                          X_ba = conj(X_ab). */
static void packed_to_cotangent(const double *g, int64_t stride, cplx X[3][3])
{
    X[0][0] = g[0 * stride];
    X[1][1] = g[1 * stride];
    X[2][2] = g[2 * stride];
    X[0][1] = 0.5 * (g[3 * stride] + I * g[4 * stride]);
    X[0][2] = 0.5 * (g[5 * stride] + I * g[6 * stride]);
    X[1][2] = 0.5 * (g[7 * stride] + I * g[8 * stride]);
    X[1][0] = conj(X[0][1]);
    X[2][0] = conj(X[0][2]);
    X[2][1] = conj(X[1][2]);
}

static void cotangent_to_packed_add(cplx X[3][3], double *g, int64_t stride)
{
    g[0 * stride] += creal(X[0][0]);
    g[1 * stride] += creal(X[1][1]);
    g[2 * stride] += creal(X[2][2]);
    g[3 * stride] += creal(X[0][1]) + creal(X[1][0]);
    g[4 * stride] += cimag(X[0][1]) - cimag(X[1][0]);
    g[5 * stride] += creal(X[0][2]) + creal(X[2][0]);
    g[6 * stride] += cimag(X[0][2]) - cimag(X[2][0]);
    g[7 * stride] += creal(X[1][2]) + creal(X[2][1]);
    g[8 * stride] += cimag(X[1][2]) - cimag(X[2][1]);
}

/* VJP of the right-hand side at (t, y): given g = dL/dk (state-shaped),
 * add dL/dy into gy and dL/dN, dL/dNbar into gN, gNb. */
static void rhs_vjp(const oracle_problem *P, const double *y, double t, const double *g,
                    moments *grid, moments *cot, double *gy, double *gN, double *gNb)
{
    const int64_t nc = ncell_total(P), nd = P->ndir, np = nc * nd;
    const double dV = P->dx[0] * P->dx[1] * P->dx[2];
    cplx Hv[3][3];
    double Vm[3];
    load_hvac(P, Hv);
    load_vmat(P, Vm);
    deposit(P, y, t, grid);
    memset(cot, 0, sizeof(moments) * (size_t)nc);
    /* commutators, Hamiltonians and the transpose of the interpolation */
    for (int64_t p = 0; p < np; p++) {
        const int64_t d = p / nc;
        const double *v = P->dirs + 3 * d;
        stencil S;
        shape_stencil(P, p, t, &S);
        moments m;
        interpolate(grid, &S, &m);
        cplx H[3][3], Hb[3][3];
        hamiltonians(&m, v, Hv, Vm, H, Hb);
        cplx rho[3][3], rhob[3][3], Gc[3][3], Gb[3][3];
        unpack(y + p, np, rho);
        unpack(y + 9 * np + p, np, rhob);
        packed_to_cotangent(g + p, np, Gc);
        packed_to_cotangent(g + 9 * np + p, np, Gb);
        /* k = -i[H, rho]:  cot(rho) = -i[G, H],  cot(H) = -i[rho, G] */
        cplx Xr[3][3], Xh[3][3], Xrb[3][3], Xhb[3][3];
        commutator_rhs(Gc, H, Xr);
        commutator_rhs(rho, Gc, Xh);
        commutator_rhs(Gb, Hb, Xrb);
        commutator_rhs(rhob, Gb, Xhb);
        cotangent_to_packed_add(Xr, gy + p, np);
        cotangent_to_packed_add(Xrb, gy + 9 * np + p, np);
        /* H = Hv + Hm + Hnn, Hbar = Hv^* - Hm^* - Hnn^*: cot(Hnn) = Xh - conj(Xhb) */
        cplx Xn[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                Xn[i][j] = Xh[i][j] - conj(Xhb[i][j]);
        /* Hnn = n - nb^* - sum_a v_a (f_a - fb_a^*), then the interpolation
         * transposed onto the cells */
        for (int s = 0; s < S.n; s++) {
            moments *q = cot + S.cell[s];
            const double w = S.w[s];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    q->n[i][j] += w * Xn[i][j];
                    q->nb[i][j] -= w * conj(Xn[i][j]);
                    for (int a = 0; a < 3; a++) {
                        q->f[a][i][j] -= w * v[a] * Xn[i][j];
                        q->fb[a][i][j] += w * v[a] * conj(Xn[i][j]);
                    }
                }
        }
    }
    /* transpose of the deposition: n_j = sum_q w N rho_q / dV etc. */
    for (int64_t p = 0; p < np; p++) {
        const int64_t d = p / nc;
        const double *v = P->dirs + 3 * d;
        stencil S;
        shape_stencil(P, p, t, &S);
        cplx Z[3][3], Zb[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                Z[i][j] = 0;
                Zb[i][j] = 0;
            }
        for (int s = 0; s < S.n; s++) {
            const moments *q = cot + S.cell[s];
            const double w = S.w[s];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    cplx zn = q->n[i][j], zb = q->nb[i][j];
                    for (int a = 0; a < 3; a++) {
                        zn += v[a] * q->f[a][i][j];
                        zb += v[a] * q->fb[a][i][j];
                    }
                    Z[i][j] += w * zn / dV;
                    Zb[i][j] += w * zb / dV;
                }
        }
        cplx rho[3][3], rhob[3][3], XN[3][3], XNb[3][3];
        unpack(y + p, np, rho);
        unpack(y + 9 * np + p, np, rhob);
        double dn = 0.0, dnb = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                XN[i][j] = P->N[d] * Z[i][j];
                XNb[i][j] = P->Nbar[d] * Zb[i][j];
                dn += creal(conj(Z[i][j]) * rho[i][j]);
                dnb += creal(conj(Zb[i][j]) * rhob[i][j]);
            }
        cotangent_to_packed_add(XN, gy + p, np);
        cotangent_to_packed_add(XNb, gy + 9 * np + p, np);
        gN[d] += dn;
        gNb[d] += dnb;
    }
}

/* Reverse mode of nsteps RK4 steps from step n0 starting at state0: given
 * lam = dL/d(final state), return dL/d(state0) in lam (in place) and add
 * dL/dN, dL/dNbar into gN, gNb.  All intermediate states are kept in
 * memory (small problems only). */
int oracle_adjoint(const oracle_problem *P, const double *state0, int64_t n0, int64_t nsteps,
                   double *lam, double *gN, double *gNb)
{
    if (P->pos0)
        return -2; /* the reverse mode covers the lattice placement only */
    const int64_t nc = ncell_total(P), len = 18 * P->ndir * nc;
    const double dt = P->dt;
    double *traj = malloc(sizeof(double) * (size_t)len * (size_t)(nsteps + 1));
    moments *grid = grid_alloc(P);
    moments *cot = malloc(sizeof(moments) * (size_t)nc);
    double *k = malloc(sizeof(double) * (size_t)len * 3);
    double *ys = malloc(sizeof(double) * (size_t)len * 4);
    double *gs = malloc(sizeof(double) * (size_t)len);
    double *ls = malloc(sizeof(double) * (size_t)len);
    double *lsum = malloc(sizeof(double) * (size_t)len);
    if (!traj || !grid || !cot || !k || !ys || !gs || !ls || !lsum) {
        free(traj); free(grid); free(cot); free(k); free(ys); free(gs); free(ls); free(lsum);
        return -1;
    }
    memcpy(traj, state0, sizeof(double) * (size_t)len);
    for (int64_t s = 0; s < nsteps; s++) {
        memcpy(traj + (s + 1) * len, traj + s * len, sizeof(double) * (size_t)len);
        if (oracle_step(P, traj + (s + 1) * len, n0 + s, 1)) {
            free(traj); free(grid); free(cot); free(k); free(ys); free(gs); free(ls); free(lsum);
            return -1;
        }
    }
    for (int64_t s = nsteps - 1; s >= 0; s--) {
        const int64_t n = n0 + s;
        const double *Y = traj + s * len;
        double *k1 = k, *k2 = k + len, *k3 = k + 2 * len;
        double *y1 = ys, *y2 = ys + len, *y3 = ys + 2 * len, *y4 = ys + 3 * len;
        /* recompute the stage states */
        memcpy(y1, Y, sizeof(double) * (size_t)len);
        rhs(P, y1, stage_time(n, dt, 0.0), grid, k1);
        for (int64_t i = 0; i < len; i++)
            y2[i] = Y[i] + (0.5 * dt) * k1[i];
        rhs(P, y2, stage_time(n, dt, 0.5), grid, k2);
        for (int64_t i = 0; i < len; i++)
            y3[i] = Y[i] + (0.5 * dt) * k2[i];
        rhs(P, y3, stage_time(n, dt, 0.5), grid, k3);
        for (int64_t i = 0; i < len; i++)
            y4[i] = Y[i] + dt * k3[i];
        /* Y' = Y + dt/6 (k1 + 2 k2 + 2 k3 + k4): walk the stages backwards;
         * gs = dL/dk_s, ls = dL/dy_s, lsum = dL/dY */
        memcpy(lsum, lam, sizeof(double) * (size_t)len);
        /* stage 4 */
        for (int64_t i = 0; i < len; i++) {
            gs[i] = (dt / 6.0) * lam[i];
            ls[i] = 0.0;
        }
        rhs_vjp(P, y4, stage_time(n, dt, 1.0), gs, grid, cot, ls, gN, gNb);
        for (int64_t i = 0; i < len; i++) {
            lsum[i] += ls[i];
            gs[i] = (dt / 3.0) * lam[i] + dt * ls[i];
            ls[i] = 0.0;
        }
        /* stage 3 */
        rhs_vjp(P, y3, stage_time(n, dt, 0.5), gs, grid, cot, ls, gN, gNb);
        for (int64_t i = 0; i < len; i++) {
            lsum[i] += ls[i];
            gs[i] = (dt / 3.0) * lam[i] + (0.5 * dt) * ls[i];
            ls[i] = 0.0;
        }
        /* stage 2 */
        rhs_vjp(P, y2, stage_time(n, dt, 0.5), gs, grid, cot, ls, gN, gNb);
        for (int64_t i = 0; i < len; i++) {
            lsum[i] += ls[i];
            gs[i] = (dt / 6.0) * lam[i] + (0.5 * dt) * ls[i];
            ls[i] = 0.0;
        }
        /* stage 1 */
        rhs_vjp(P, y1, stage_time(n, dt, 0.0), gs, grid, cot, ls, gN, gNb);
        for (int64_t i = 0; i < len; i++)
            lam[i] = lsum[i] + ls[i];
    }
    free(traj); free(grid); free(cot); free(k); free(ys); free(gs); free(ls); free(lsum);
    return 0;
}
