/*
 * pic_oracle.c -- plain FP64 CPU oracle for the 1D electrostatic
 * particle-in-cell (PIC) cycle of S. Markidis and G. Lapenta, "Development and
 * performance analysis of a UPC Particle-in-Cell code" (PGAS10).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only code allowed to load this library.
 * The GPU engine never links, includes or calls it, and this file includes
 * nothing of the engine's.  Everything here is sequential double precision in
 * the most direct form of the paper's definitions, so that it can be checked
 * against the paper by eye; speed is not a goal.
 *
 * Model (Sec. 2): one spatial dimension, electrostatic, only electrons move,
 * immobile uniform ion background; normalised units with epsilon_0 = 1.
 *
 * Conventions taken from the paper:
 *   - grid nodes at x_g = (g + 1/2) dx, g = 0..ng-1, dx = L/ng (Appendix A,
 *     node-coordinate initialisation);
 *   - particle charge Q = sign(qm) rho0 L / np and uniform ion density rho0
 *     added to the charge density (Appendix A, charge normalisation and
 *     background ions);
 *   - two-node linear ("cloud-in-cell") weighting for both the deposit and
 *     the field interpolation (Sec. 2.3);
 *   - leapfrog push x^{n+1} = x^n + v^{n+1/2} dt,
 *     v^{n+1/2} = v^{n-1/2} + (q/m) E_p^n dt (Sec. 2.1);
 *   - three-point Poisson equation
 *     phi_{g+1} - 2 phi_g + phi_{g-1} = -rho_g dx^2 (Sec. 2.2) and the
 *     central-difference field E_g = -(phi_{g+1} - phi_{g-1}) / (2 dx)
 *     (Sec. 2.2), both periodic.
 *
 * Readings where the paper is silent or loose (each one also listed with the
 * project's design notes):
 *   R1 weights: node j = floor(x/dx - 1/2) receives 1-f and node j+1 receives
 *      f, f = x/dx - 1/2 - j (the triangle kernel max(0, 1 - |x - x_g|/dx)),
 *      indices modulo ng.  Sec. 2.3 names w1 and w2 loosely; this is the
 *      assignment that the appendix's code performs.
 *   R2 field solve: the periodic system of Sec. 2.2 is solved exactly (zero
 *      mean potential) after removing the mean of rho, instead of the
 *      fixed-iteration CG of Sec. 2.2 / 3.3, which does not converge at
 *      large ng.  The CG is also provided (ora_cg_paper) for comparison.
 *   R3 wrap: x <- x - L floor(x/L), so positions live in [0, L).
 *   R4 fixed-point deposit (the engine's exact-charge form): see
 *      ora_deposit_fixed.
 *   R5 cell order (the engine's optional locality sort, not in the paper):
 *      stable by the left stencil node; see ora_cell_order.
 *
 * Parity status: every function below is pinned by tests against brute force,
 * dense linear algebra, closed forms or physical invariants; none is marked
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double  L;     /* periodic domain length                       */
    int32_t ng;    /* number of cells (= grid nodes)               */
    int32_t solver; /* field solve of whole steps: 0 exact, 1 the paper's CG */
    int64_t np;    /* number of computational particles            */
    double  dt;    /* time step                                     */
    double  qm;    /* charge-to-mass ratio of the mobile species    */
    double  rho0;  /* density of the immobile ion background        */
    int32_t cg_iters; /* CG iterations for solver 1 (0: the paper's 150) */
    int32_t pad_;
} ora_params;

#define TWO32 4294967296.0

static double cell_width(const ora_params *p) { return p->L / (double)p->ng; }

/* Particle charge (Appendix A charge normalisation): the total particle
 * charge cancels the ion background rho0 * L. */
static double particle_charge(const ora_params *p)
{
    double s = p->qm < 0.0 ? -1.0 : 1.0;
    return s * p->rho0 * p->L / (double)p->np;
}

/* Particle mass m = Q / (q/m). */
static double particle_mass(const ora_params *p) { return particle_charge(p) / p->qm; }

static int64_t wrap_index(int64_t j, int64_t ng)
{
    int64_t r = j % ng;
    return r < 0 ? r + ng : r;
}

double ora_particle_charge(const ora_params *p) { return particle_charge(p); }
double ora_particle_mass(const ora_params *p) { return particle_mass(p); }

/* Cloud-in-cell weights of a position (Sec. 2.3, reading R1). */
static void cic_weights(const ora_params *p, double x, int64_t *j0, int64_t *j1, double *f)
{
    double t = x / cell_width(p) - 0.5;
    double j = floor(t);
    *f = t - j;
    *j0 = wrap_index((int64_t)j, p->ng);
    *j1 = wrap_index((int64_t)j + 1, p->ng);
}

/* Charge density with plain FP64 accumulation (Sec. 2.3 and Appendix A):
 * rho_g = rho0 + (Q/dx) * sum_p W(x_p - x_g). */
void ora_deposit_plain(const ora_params *p, const double *x, double *rho)
{
    double qdx = particle_charge(p) / cell_width(p);
    for (int32_t g = 0; g < p->ng; ++g)
        rho[g] = p->rho0;
    for (int64_t i = 0; i < p->np; ++i) {
        int64_t j0, j1;
        double f;
        cic_weights(p, x[i], &j0, &j1, &f);
        rho[j0] += (1.0 - f) * qdx;
        rho[j1] += f * qdx;
    }
}

/* Exact fixed-point form of the same deposit (reading R4).  The normalised
 * position u = x/dx is scaled by 2^32 and truncated; shifting by half a cell
 * gives the left node j and a 32-bit fraction F; node j receives 2^32 - F and
 * node j+1 receives F.  Every particle adds exactly 2^32, so the total is
 * np * 2^32 in any summation order.  u*2^32 is exact in double for the
 * positions used here (|u| < 2^21), and so is the truncation. */
void ora_deposit_fixed(int32_t ng, int64_t np, const double *u, int64_t *S)
{
    for (int32_t g = 0; g < ng; ++g)
        S[g] = 0;
    for (int64_t i = 0; i < np; ++i) {
        int64_t U = (int64_t)floor(u[i] * TWO32);
        int64_t Us = U - ((int64_t)1 << 31);
        int64_t j = Us >> 32;                 /* floor((U - 2^31) / 2^32) */
        int64_t F = Us - j * ((int64_t)1 << 32); /* in [0, 2^32) */
        S[wrap_index(j, ng)] += ((int64_t)1 << 32) - F;
        S[wrap_index(j + 1, ng)] += F;
    }
}

/* Cell key of a normalised position u = x/dx in [0, ng): the left node of
 * its two-node stencil before wrapping, floor(u - 1/2) in [-1, ng-1]
 * (Sec. 2.3, reading R1), shifted to [0, ng].  Values outside the range
 * (not produced by a valid state) are clamped to the end keys. */
static int64_t cell_key(int32_t ng, double u)
{
    double j = floor(u - 0.5);
    if (j < -1.0)
        j = -1.0;
    if (j > (double)(ng - 1))
        j = (double)(ng - 1);
    return (int64_t)j + 1;
}

/* Stable order of the particles by cell key: perm[k] is the index of the
 * particle that goes to position k, particles with equal keys keep their
 * input order.  This is not a step of the paper's cycle (its loops visit the
 * particles in any order and the result does not depend on it); it states
 * what the engine's optional locality reordering produces.  A counting sort
 * written out directly: count the keys, turn the counts into first
 * positions, then place the particles in input order. */
void ora_cell_order(int32_t ng, int64_t np, const double *u, int64_t *perm)
{
    int64_t *first = calloc((size_t)ng + 2, sizeof *first);
    for (int64_t i = 0; i < np; ++i)
        first[cell_key(ng, u[i]) + 1] += 1;
    for (int32_t k = 1; k <= ng + 1; ++k)
        first[k] += first[k - 1];
    for (int64_t i = 0; i < np; ++i)
        perm[first[cell_key(ng, u[i])]++] = i;
    free(first);
}

/* Phase-space counts: the (x, v) plane that the two-stream figure of Sec. 4
 * plots particle by particle, as an nv x nx image.  Particle (x, v) belongs
 * to column floor(x nx / L) and row floor((v - vmin) nv / (vmax - vmin)); rows
 * outside [0, nv) are counted in *outside.  Not a step of the cycle: an
 * output of it.  The particles come in the engine's state form u = x/dx,
 * w = v dt/dx, and each bin is decided in FP64 from those values with one
 * subtraction and one product (the engine decides the same way):
 * column min(floor(u nx/ng), nx - 1), y = (w - vmin c) (nv / ((vmax - vmin) c)),
 * c = dt/dx. */
void ora_phase_space(const ora_params *p, int64_t np, const double *u, const double *w, int32_t nx, int32_t nv,
                     double vmin, double vmax, uint32_t *counts, int64_t *outside)
{
    double c = p->dt / cell_width(p);
    double xs = (double)nx / (double)p->ng;
    double w_lo = vmin * c;
    double w_bin = (double)nv / ((vmax - vmin) * c);
    int64_t out = 0;
    for (int64_t b = 0; b < (int64_t)nx * nv; ++b)
        counts[b] = 0;
    for (int64_t i = 0; i < np; ++i) {
        double y = (w[i] - w_lo) * w_bin;
        if (!(y >= 0.0 && y < (double)nv)) {
            out += 1;
            continue;
        }
        int64_t col = (int64_t)floor(u[i] * xs);
        if (col > nx - 1)
            col = nx - 1;
        int64_t row = (int64_t)floor(y);
        counts[row * nx + col] += 1;
    }
    *outside = out;
}

/* Charge density from the fixed-point sums: rho_g = rho0 + (Q/dx) S_g 2^-32. */
void ora_density_fixed(const ora_params *p, const int64_t *S, double *rho)
{
    double qdx = particle_charge(p) / cell_width(p);
    for (int32_t g = 0; g < p->ng; ++g)
        rho[g] = p->rho0 + qdx * ((double)S[g] / TWO32);
}

/* Periodic Poisson solve and node field (Sec. 2.2, reading R2).
 *
 * With the face field F_{g+1/2} = -(phi_{g+1} - phi_g)/dx the three-point
 * equation reads F_{g+1/2} - F_{g-1/2} = rho_g dx, so F is a running sum of
 * rho dx; periodicity of phi fixes the constant by sum_g F_{g+1/2} = 0, and
 * the central-difference node field is E_g = (F_{g-1/2} + F_{g+1/2}) / 2.
 * The mean of rho is removed first (a periodic system has a solution only
 * for zero net charge).  phi is returned with zero mean; phi may be NULL. */
void ora_solve(const ora_params *p, const double *rho, double *E, double *phi)
{
    int32_t ng = p->ng;
    double dx = cell_width(p);
    double *face = (double *)malloc(sizeof(double) * (size_t)ng);
    double mean = 0.0;
    for (int32_t g = 0; g < ng; ++g)
        mean += rho[g];
    mean /= (double)ng;
    double run = 0.0;
    for (int32_t g = 0; g < ng; ++g) {
        run += (rho[g] - mean) * dx;
        face[g] = run;                       /* F_{g+1/2} up to a constant */
    }
    double c = 0.0;
    for (int32_t g = 0; g < ng; ++g)
        c += face[g];
    c /= (double)ng;
    for (int32_t g = 0; g < ng; ++g)
        face[g] -= c;
    for (int32_t g = 0; g < ng; ++g) {
        double left = face[g == 0 ? ng - 1 : g - 1];
        E[g] = 0.5 * (left + face[g]);
    }
    if (phi) {
        double acc = 0.0, pm = 0.0;
        phi[0] = 0.0;
        for (int32_t g = 0; g + 1 < ng; ++g) {
            acc -= dx * face[g];
            phi[g + 1] = acc;
        }
        for (int32_t g = 0; g < ng; ++g)
            pm += phi[g];
        pm /= (double)ng;
        for (int32_t g = 0; g < ng; ++g)
            phi[g] -= pm;
    }
    free(face);
}

/* The paper's field solver (Sec. 2.2 and 3.3): conjugate gradient on the
 * three-point system with phi_0 held at zero, started from phi = 0 and run
 * for `maxit` iterations (the paper fixes 150), followed by the central
 * difference for E.  The operator keeps row 0 as the identity on the pinned
 * unknown and closes the last row with phi_ng = phi_0 = 0.  Returns the
 * number of iterations performed. */
int32_t ora_cg_paper(const ora_params *p, const double *rho, int32_t maxit,
                     double *phi, double *E)
{
    int32_t ng = p->ng;
    double dx = cell_width(p);
    size_t sz = sizeof(double) * (size_t)ng;
    double *r = (double *)malloc(sz), *d = (double *)malloc(sz), *z = (double *)malloc(sz);
    for (int32_t g = 0; g < ng; ++g) {
        phi[g] = 0.0;
        r[g] = g == 0 ? 0.0 : -rho[g] * dx * dx;
        d[g] = r[g];
    }
    double rr = 0.0;
    for (int32_t g = 0; g < ng; ++g)
        rr += r[g] * r[g];
    int32_t it = 0;
    if (sqrt(rr) > 1e-16) {
        for (; it < maxit; ++it) {
            for (int32_t g = 0; g < ng; ++g) {
                if (g == 0)
                    z[g] = d[0];
                else {
                    double right = g + 1 < ng ? d[g + 1] : 0.0;
                    z[g] = d[g - 1] - 2.0 * d[g] + right;
                }
            }
            double zd = 0.0;
            for (int32_t g = 0; g < ng; ++g)
                zd += z[g] * d[g];
            if (zd == 0.0)
                break;
            double alpha = rr / zd;
            for (int32_t g = 0; g < ng; ++g) {
                phi[g] += alpha * d[g];
                r[g] -= alpha * z[g];
            }
            double rr_new = 0.0;
            for (int32_t g = 0; g < ng; ++g)
                rr_new += r[g] * r[g];
            double beta = rr_new / rr;
            for (int32_t g = 0; g < ng; ++g)
                d[g] = beta * d[g] + r[g];
            rr = rr_new;
        }
    }
    for (int32_t g = 0; g < ng; ++g) {
        double right = phi[g + 1 < ng ? g + 1 : 0];
        double left = phi[g == 0 ? ng - 1 : g - 1];
        E[g] = -(right - left) / (2.0 * dx);
    }
    free(r);
    free(d);
    free(z);
    return it;
}

/* The field solve of a whole step: the exact periodic solve (reading R2),
 * or the paper's fixed-iteration CG when the parameters ask for it. */
static void field_solve(const ora_params *p, const double *rho, double *E)
{
    if (p->solver == 1) {
        double *phi = (double *)malloc(sizeof(double) * (size_t)p->ng);
        ora_cg_paper(p, rho, p->cg_iters > 0 ? p->cg_iters : 150, phi, E);
        free(phi);
    } else {
        ora_solve(p, rho, E, NULL);
    }
}

/* Field at particle positions with the deposit's weights (Sec. 2.3). */
void ora_gather(const ora_params *p, const double *x, const double *E, double *Ep)
{
    for (int64_t i = 0; i < p->np; ++i) {
        int64_t j0, j1;
        double f;
        cic_weights(p, x[i], &j0, &j1, &f);
        Ep[i] = (1.0 - f) * E[j0] + f * E[j1];
    }
}

static double wrap_position(const ora_params *p, double x)
{
    x -= p->L * floor(x / p->L);
    if (x >= p->L)
        x -= p->L;
    return x;
}

/* Leapfrog kick and drift with periodic wrap (Sec. 2.1, reading R3), for a
 * given field at the particles.  Accumulates sum v_old^2, sum v_new^2 and
 * sum v_new into acc[0..2] when acc is not NULL. */
void ora_push(const ora_params *p, double *x, double *v, const double *Ep, double *acc)
{
    double s_old2 = 0.0, s_new2 = 0.0, s_new = 0.0;
    for (int64_t i = 0; i < p->np; ++i) {
        double v_old = v[i];
        double v_new = v_old + p->qm * Ep[i] * p->dt;
        s_old2 += v_old * v_old;
        s_new2 += v_new * v_new;
        s_new += v_new;
        v[i] = v_new;
        x[i] = wrap_position(p, x[i] + v_new * p->dt);
    }
    if (acc) {
        acc[0] = s_old2;
        acc[1] = s_new2;
        acc[2] = s_new;
    }
}

/* Electrostatic field energy W_E = 1/2 sum_g E_g^2 dx. */
double ora_field_energy(const ora_params *p, const double *E)
{
    double s = 0.0;
    for (int32_t g = 0; g < p->ng; ++g)
        s += E[g] * E[g];
    return 0.5 * s * cell_width(p);
}

enum { ORA_DEPOSIT_PLAIN = 0, ORA_DEPOSIT_FIXED = 1 };

/* Charge density of positions x with either deposit form. */
void ora_density(const ora_params *p, const double *x, int32_t mode, double *rho, int64_t *S_out)
{
    if (mode == ORA_DEPOSIT_FIXED) {
        double dx = cell_width(p);
        double *u = (double *)calloc((size_t)(p->np > 0 ? p->np : 1), sizeof(double));
        int64_t *S = S_out ? S_out : (int64_t *)malloc(sizeof(int64_t) * (size_t)p->ng);
        for (int64_t i = 0; i < p->np; ++i)
            u[i] = x[i] / dx;
        ora_deposit_fixed(p->ng, p->np, u, S);
        ora_density_fixed(p, S, rho);
        if (!S_out)
            free(S);
        free(u);
    } else {
        ora_deposit_plain(p, x, rho);
    }
}

/* One PIC cycle (Sec. 2.4) from the state (x^n, v^{n-1/2}, E^n):
 * gather E^n, kick to v^{n+1/2}, drift and wrap to x^{n+1}, deposit rho^{n+1},
 * solve for E^{n+1} (written back into E).
 * row[0] = KE^n   = (m/2) sum_p (v_old^2 + v_new^2)/2   (time-centred)
 * row[1] = W_E^n  = field energy of the input E^n
 * row[2] = P^{n+1/2} = m sum_p v^{n+1/2}
 * row[3] = K^{n+1/2} = (m/2) sum_p (v^{n+1/2})^2
 * rho (ng) receives rho^{n+1}; Ep is caller scratch of np doubles. */
void ora_step(const ora_params *p, double *x, double *v, double *E, int32_t mode,
              double *rho, double *Ep, double *row)
{
    double acc[3];
    double m = particle_mass(p);
    double we = ora_field_energy(p, E);
    ora_gather(p, x, E, Ep);
    ora_push(p, x, v, Ep, acc);
    ora_density(p, x, mode, rho, NULL);
    field_solve(p, rho, E);
    if (row) {
        row[0] = 0.25 * m * (acc[0] + acc[1]);
        row[1] = we;
        row[2] = m * acc[2];
        row[3] = 0.5 * m * acc[1];
    }
}

/* Initial field from the initial positions, then `nsteps` cycles.
 * hist: nsteps x 4 rows (see ora_step); E_hist (optional): nsteps x ng, the
 * field E^n used by step n.  On return x, v hold x^N, v^{N-1/2}, E holds E^N
 * and rho holds rho^N. */
void ora_run(const ora_params *p, double *x, double *v, int64_t nsteps, int32_t mode,
             double *E, double *rho, double *hist, double *E_hist)
{
    double *Ep = (double *)malloc(sizeof(double) * (size_t)(p->np > 0 ? p->np : 1));
    ora_density(p, x, mode, rho, NULL);
    field_solve(p, rho, E);
    for (int64_t n = 0; n < nsteps; ++n) {
        if (E_hist)
            memcpy(E_hist + n * p->ng, E, sizeof(double) * (size_t)p->ng);
        ora_step(p, x, v, E, mode, rho, Ep, hist ? hist + 4 * n : NULL);
    }
    free(Ep);
}

/* The cycle in the appendix's own order: drift with the current velocity,
 * wrap, deposit, solve, then gather and kick (the initial velocity is used
 * for the first drift; there is no half-step back-push).  Runs `ncycles`
 * cycles from (x, v) and leaves the final positions, velocities and field.
 * It differs from ora_run only in where the leapfrog starts: N cycles here
 * equal one drift, N - 1 steps of ora_run and a closing gather and kick
 * (the reading of the leapfrog start; pinned by the tests). */
void ora_run_literal(const ora_params *p, double *x, double *v, int64_t ncycles, int32_t mode,
                     double *E, double *rho)
{
    double *Ep = (double *)malloc(sizeof(double) * (size_t)(p->np > 0 ? p->np : 1));
    for (int64_t n = 0; n < ncycles; ++n) {
        for (int64_t i = 0; i < p->np; ++i)
            x[i] = wrap_position(p, x[i] + v[i] * p->dt);
        ora_density(p, x, mode, rho, NULL);
        field_solve(p, rho, E);
        ora_gather(p, x, E, Ep);
        for (int64_t i = 0; i < p->np; ++i)
            v[i] = v[i] + p->qm * Ep[i] * p->dt;
    }
    free(Ep);
}
