/*
 * dsm_oracle.c -- plain FP64 CPU oracle of the diffuse-solid ternary
 * lattice Boltzmann step (arXiv 2504.19941, Sec. II.B).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the GPU library.
 *
 * Written for checking by eye against the paper: one loop per stage of the
 * step, in the order the method applies them, every array a full field, no
 * blocking or fusion.  Sums over directions run i = 0..Q-1 and reductions
 * over nodes run in index order, so results do not depend on the thread
 * count.  Where the paper is silent, garbled or self-contradictory the
 * reading used is stated at the spot.
 */
#include "dsm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Lattices.  D2Q9 exactly as listed in Sec. II.B; D3Q19 (the paper has no
 * 3D LBM) in the same style: rest, then each velocity next to its opposite. */
static const int D2Q9_C[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double D2Q9_W[9] = {
    4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int D3Q19_C[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double D3Q19_W[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* speed of sound squared, c_s^2 = 1/3 */
#define CS2 (1.0 / 3.0)

struct dsmo_sim {
    dsmo_params p;
    int Q;
    const int (*c)[3];
    const double* w;
    int opp[19];
    long N;
    unsigned char* mask; /* solid region S */
    double* C1;          /* solid component (frozen in the fluid stage) */
    double *f, *g;       /* post-stream populations, [Q][N] */
    double *fs, *gs;     /* post-collision populations, [Q][N] */
    double *phi, *mu, *p_t;
    double *F, *u;       /* [3][N] */
    double *rho, *grho;  /* local density [N] and its gradient [3][N] */
    long* nb;            /* nb[i*N + n] = index of n + c_i (periodic) */
    int stage;           /* 0 nothing live, 1 solid stage live, 2 fluid stage live */
    /* solid-stage settings of the live solid-stage state */
    double beta, omega, tau_s, tau_gs;
};

/* ------------------------------------------------------------------ */
/* small helpers */

static long wrap(long a, long n) {
    a %= n;
    return a < 0 ? a + n : a;
}

/* index of node n shifted by (dx, dy, dz), periodic in every axis */
static long shift(const dsmo_sim* s, long n, int dx, int dy, int dz) {
    long nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    long x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    x = wrap(x + dx, nx);
    y = wrap(y + dy, ny);
    z = wrap(z + dz, nz);
    return x + nx * (y + ny * z);
}

/* neighbour n + c_i (sign +1) or n - c_i (sign -1), from the table filled
 * once by shift() at creation */
static long nbr(const dsmo_sim* s, long n, int i, int sign) {
    int j = sign > 0 ? i : s->opp[i];
    return s->nb[(size_t)j * s->N + n];
}

static int threads_of(const dsmo_sim* s) { return s->p.threads > 1 ? s->p.threads : 1; }

/* Isotropic central differences on the lattice stencil (Sec. II.B states a
 * second-order isotropic central difference but not its stencil):
 *   gradient  G[a](x) = (1/c_s^2) sum_i w_i c_i a(x + c_i)
 *   Laplacian L[a](x) = (2/c_s^2) sum_i w_i (a(x + c_i) - a(x))           */
static void grad(const dsmo_sim* s, const double* a, long n, double out[3]) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int i = 0; i < s->Q; ++i) {
        double v = a[nbr(s, n, i, +1)];
        gx += s->w[i] * s->c[i][0] * v;
        gy += s->w[i] * s->c[i][1] * v;
        gz += s->w[i] * s->c[i][2] * v;
    }
    out[0] = gx / CS2;
    out[1] = gy / CS2;
    out[2] = gz / CS2;
}

static double lap(const dsmo_sim* s, const double* a, long n) {
    double acc = 0.0;
    for (int i = 0; i < s->Q; ++i) acc += s->w[i] * (a[nbr(s, n, i, +1)] - a[n]);
    return 2.0 * acc / CS2;
}

/* A node belongs to the solid when C1 > 1/2 (the solid locations are
 * redefined as C1 > 0.5 in Sec. II.B).  Only the fluid stage has solid
 * nodes; while the solid forms, every node is fluid. */
static int is_solid(const dsmo_sim* s, long n) {
    return s->stage == 2 && s->C1[n] > 0.5;
}

/* ------------------------------------------------------------------ */
/* Local formulas of Sec. II.B */

/* s_i(u): advective part of the equilibria.  Read with a minus sign on the
 * u.u term (with the typeset plus sign the weights no longer sum s_i to
 * zero and the scheme stops conserving mass). */
static double s_i(const int c[3], const double u[3]) {
    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
}

int dsmo_lattice(int dim, int* c, double* w) {
    int Q = dim == 2 ? 9 : (dim == 3 ? 19 : 0);
    if (!Q) return DSMO_EINVAL;
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) {
            if (c) c[3 * i + d] = dim == 2 ? D2Q9_C[i][d] : D3Q19_C[i][d];
        }
        if (w) w[i] = dim == 2 ? D2Q9_W[i] : D3Q19_W[i];
    }
    return Q;
}

/* Incompressible hydrodynamic equilibrium, f_eq,i = w_i (p~ + rho s_i(u)),
 * where p~ = P / c_s^2 is the zeroth moment of f (the paper's P appears in
 * f_eq divided by c_s^2, while its moment formula carries no 1/c_s^2; the
 * two are reconciled by taking the moment to be P / c_s^2). */
void dsmo_equilibrium_f(int dim, double p_tilde, double rho, const double u[3], double* feq) {
    int c[19 * 3];
    double w[19];
    int Q = dsmo_lattice(dim, c, w);
    for (int i = 0; i < Q; ++i) feq[i] = w[i] * (p_tilde + rho * s_i(&c[3 * i], u));
}

/* Cahn-Hilliard equilibrium (Sec. II.B, after Zheng et al.):
 *   g_eq,i = w_i mu + w_i C s_i(u)       for i != 0,
 *   g_eq,0 = C - sum_{i != 0} g_eq,i     (the rest population closes the
 *                                          zeroth moment to C; the typeset
 *                                          rest formula carries the opposite
 *                                          sign on (1 - w_0) mu). */
void dsmo_equilibrium_g(int dim, double C, double mu, const double u[3], double* geq) {
    int c[19 * 3];
    double w[19];
    int Q = dsmo_lattice(dim, c, w);
    double rest = C;
    for (int i = 1; i < Q; ++i) {
        geq[i] = w[i] * mu + w[i] * C * s_i(&c[3 * i], u);
        rest -= geq[i];
    }
    geq[0] = rest;
}

/* Forcing term (Sec. II.B):
 *   F_i = (1 - 1/(2 tau)) w_i [ ((c_i - u) . grad rho) s_i(u) + c_i . F / c_s^2 ]
 * with tau the local hydrodynamic relaxation time (the density enters
 * only through grad rho). */
void dsmo_forcing(int dim, double tau, double rho, const double u[3],
                  const double grad_rho[3], const double F[3], double* Fi) {
    (void)rho;
    int c[19 * 3];
    double w[19];
    int Q = dsmo_lattice(dim, c, w);
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < Q; ++i) {
        const int* ci = &c[3 * i];
        double cmu_gr = (ci[0] - u[0]) * grad_rho[0] + (ci[1] - u[1]) * grad_rho[1] +
                        (ci[2] - u[2]) * grad_rho[2];
        double cF = ci[0] * F[0] + ci[1] * F[1] + ci[2] * F[2];
        Fi[i] = pref * w[i] * (cmu_gr * s_i(ci, u) + cF / CS2);
    }
}

/* ------------------------------------------------------------------ */
/* create / destroy */

static void* zalloc(size_t n) { return calloc(n ? n : 1, 1); }

int dsmo_create(const dsmo_params* p, const unsigned char* mask, dsmo_sim** out) {
    if (!p || !out) return DSMO_EINVAL;
    *out = NULL;
    if (p->dim != 2 && p->dim != 3) return DSMO_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return DSMO_EINVAL;
    if (p->dim == 2 && p->nz != 1) return DSMO_EINVAL;
    if (!(p->tau > 0.5) || !(p->mobility > 0.0) || !(p->alpha > 0.0)) return DSMO_EINVAL;
    if (!(p->rho_liquid > 0.0) || !(p->rho_gas > 0.0) || !(p->tau_gas > 0.5)) return DSMO_EINVAL;
    if (p->force_reading != DSMO_FORCE_POTENTIAL && p->force_reading != DSMO_FORCE_AS_TYPESET)
        return DSMO_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(p->kappa[k] >= 0.0)) return DSMO_EINVAL;

    dsmo_sim* s = (dsmo_sim*)zalloc(sizeof(dsmo_sim));
    if (!s) return DSMO_ENOMEM;
    s->p = *p;
    s->Q = p->dim == 2 ? 9 : 19;
    s->c = p->dim == 2 ? D2Q9_C : D3Q19_C;
    s->w = p->dim == 2 ? D2Q9_W : D3Q19_W;
    s->opp[0] = 0;
    for (int i = 1; i < s->Q; ++i) s->opp[i] = (i % 2) ? i + 1 : i - 1;
    s->N = (long)p->nx * p->ny * p->nz;
    size_t N = (size_t)s->N, Q = (size_t)s->Q;
    s->mask = (unsigned char*)zalloc(N);
    s->C1 = (double*)zalloc(N * sizeof(double));
    s->f = (double*)zalloc(Q * N * sizeof(double));
    s->g = (double*)zalloc(Q * N * sizeof(double));
    s->fs = (double*)zalloc(Q * N * sizeof(double));
    s->gs = (double*)zalloc(Q * N * sizeof(double));
    s->phi = (double*)zalloc(N * sizeof(double));
    s->mu = (double*)zalloc(N * sizeof(double));
    s->p_t = (double*)zalloc(N * sizeof(double));
    s->F = (double*)zalloc(3 * N * sizeof(double));
    s->u = (double*)zalloc(3 * N * sizeof(double));
    s->rho = (double*)zalloc(N * sizeof(double));
    s->grho = (double*)zalloc(3 * N * sizeof(double));
    s->nb = (long*)zalloc(Q * N * sizeof(long));
    if (!s->nb) {
        dsmo_destroy(s);
        return DSMO_ENOMEM;
    }
    for (size_t i = 0; i < Q; ++i)
        for (size_t n = 0; n < N; ++n)
            s->nb[i * N + n] = shift(s, (long)n, s->c[i][0], s->c[i][1], s->c[i][2]);
    if (!s->mask || !s->C1 || !s->f || !s->g || !s->fs || !s->gs || !s->phi || !s->mu ||
        !s->p_t || !s->F || !s->u || !s->rho || !s->grho) {
        dsmo_destroy(s);
        return DSMO_ENOMEM;
    }
    if (mask)
        for (size_t n = 0; n < N; ++n) s->mask[n] = mask[n] ? 1 : 0;
    /* the solid starts as the sharp indicator of S (Sec. II.A, II.B) */
    for (size_t n = 0; n < N; ++n) s->C1[n] = s->mask[n] ? 1.0 : 0.0;
    *out = s;
    return DSMO_OK;
}

void dsmo_destroy(dsmo_sim* s) {
    if (!s) return;
    free(s->mask);
    free(s->C1);
    free(s->f);
    free(s->g);
    free(s->fs);
    free(s->gs);
    free(s->phi);
    free(s->mu);
    free(s->p_t);
    free(s->F);
    free(s->u);
    free(s->rho);
    free(s->grho);
    free(s->nb);
    free(s);
}

int dsmo_num_directions(const dsmo_sim* s) { return s ? s->Q : 0; }

/* ------------------------------------------------------------------ */
/* The stages of one step.  The evolving order parameter phi is C1 in the
 * solid stage and C2 in the fluid stage. */

/* zeroth moment of g: C = sum_i g_i (Sec. II.B) */
static void stage_moment(dsmo_sim* s) {
    long N = s->N;
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double acc = 0.0;
        for (int i = 0; i < s->Q; ++i) acc += s->g[(size_t)i * N + n];
        s->phi[n] = acc;
    }
}

/* derivative of the confining potential beta (C1 - 1/2)^2 on its active
 * branch.  Reading (the stated purpose of the potential): active where solid
 * has left S (C1 > 1/2 outside S) or fluid has entered S (C1 < 1/2 inside S).
 * The typeset case conditions are the opposite pair and are kept only as a
 * test switch. */
static double confine_derivative(const dsmo_sim* s, long n, double C1) {
    int inS = s->mask[n] != 0;
    int active;
    if (s->p.confine_reading == DSMO_CONFINE_AS_TYPESET)
        active = (C1 > 0.5 && inS) || (C1 < 0.5 && !inS);
    else
        active = (C1 < 0.5 && inS) || (C1 > 0.5 && !inS);
    return active ? 2.0 * s->beta * (C1 - 0.5) : 0.0;
}

/* Chemical potentials.
 * Fluid stage: mu = d Psi / d C2 of the frozen-solid free energy (Sec. II.B)
 *   mu = k2 C2 (1-C2)(1-2 C2) + k3 S (1-S)(1-2 S)
 *        - a^2 k2 L[C2] - a^2 k3 (L[C1] + L[C2]),        S = C1 + C2.
 * This is the variational derivative of that functional; the typeset bulk
 * polynomial differs from it inside interfaces and the typeset gradient part
 * lacks the k3 L[C2] term, and both would break the tensions of Supp. B.
 * Solid stage: mu_1 = d Psi / d C1 of the solid-relaxation functional
 *   mu_1 = (k1+k3) C1 (1-C1)(1-2 C1) + d Psi_cf / d C1 - a^2 (k1+k3) L[C1]
 *          + 2 W C1 H(-C1) - 2 W (1-C1) H(C1-1),
 * with the stabilising Omega terms read as penalties outside [0, 1] (as
 * typeset their Heaviside arguments make them act inside (0, 1)), H(0) = 0. */
static void stage_chemical_potential(dsmo_sim* s) {
    long N = s->N;
    double a2 = s->p.alpha * s->p.alpha;
    double k1 = s->p.kappa[0], k2 = s->p.kappa[1], k3 = s->p.kappa[2];
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        if (s->stage == 2) {
            double C2 = s->phi[n], C1 = s->C1[n], S = C1 + C2;
            double bulk = k2 * C2 * (1.0 - C2) * (1.0 - 2.0 * C2) +
                          k3 * S * (1.0 - S) * (1.0 - 2.0 * S);
            double l2 = lap(s, s->phi, n), l1 = lap(s, s->C1, n);
            s->mu[n] = bulk - a2 * k2 * l2 - a2 * k3 * (l1 + l2);
        } else {
            double C1 = s->phi[n], k13 = k1 + k3;
            double m = k13 * C1 * (1.0 - C1) * (1.0 - 2.0 * C1);
            m += confine_derivative(s, n, C1);
            m -= a2 * k13 * lap(s, s->phi, n);
            if (C1 < 0.0) m += 2.0 * s->omega * C1;
            if (C1 > 1.0) m -= 2.0 * s->omega * (1.0 - C1);
            s->mu[n] = m;
        }
    }
}

/* Force (Sec. II.B): the surface-tension force plus, in the fluid stage, the
 * body force on the liquid F_g = C2 g.  Zero at solid nodes.
 * The surface-tension force is taken in the potential form F_s = mu grad phi,
 * the form that the paper's velocity moment carries.  The paper also states
 * F_s = -phi grad mu; the two differ by grad(phi mu), which the pressure of
 * the incompressible model absorbs, so they describe the same flow and the
 * same static equilibria.  The typeset form is kept behind force_reading so
 * that the two can be compared. */
static void stage_force(dsmo_sim* s) {
    long N = s->N;
    int body = s->stage == 2;
    int typeset = s->p.force_reading == DSMO_FORCE_AS_TYPESET;
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        if (!is_solid(s, n)) {
            double gp[3];
            double ph = s->phi[n], m = s->mu[n];
            if (typeset) {
                grad(s, s->mu, n, gp);
                Fx = -ph * gp[0];
                Fy = -ph * gp[1];
                Fz = -ph * gp[2];
            } else {
                grad(s, s->phi, n, gp);
                Fx = m * gp[0];
                Fy = m * gp[1];
                Fz = m * gp[2];
            }
            if (body) {
                Fx += ph * s->p.gravity[0];
                Fy += ph * s->p.gravity[1];
                Fz += ph * s->p.gravity[2];
            }
        }
        s->F[0 * N + n] = Fx;
        s->F[1 * N + n] = Fy;
        s->F[2 * N + n] = Fz;
    }
}

/* Local density of the fluid stage (Sec. II.B):
 *   rho = rho_3 + (rho_2 - rho_3) C2 / (C2 + C3),
 * where C2 + C3 = 1 - C1.  Inside the solid both fluid concentrations
 * vanish, so the fraction is read with its denominator floored at 1e-6 and
 * the fraction clamped to [0, 1] (the paper does not say what the ratio is
 * where no fluid is present).  grad rho by the isotropic central difference
 * used for every other gradient.  The solid stage has rho = 1. */
static double density_at(const dsmo_sim* s, long n) {
    if (s->stage != 2) return 1.0;
    double C2 = s->phi[n], C3 = 1.0 - s->C1[n] - C2;
    double den = C2 + C3;
    if (den < 1e-6) den = 1e-6;
    double frac = C2 / den;
    if (frac < 0.0) frac = 0.0;
    if (frac > 1.0) frac = 1.0;
    return s->p.rho_gas + (s->p.rho_liquid - s->p.rho_gas) * frac;
}

static void stage_density(dsmo_sim* s) {
    long N = s->N;
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) s->rho[n] = density_at(s, n);
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double gr[3];
        grad(s, s->rho, n, gr);
        s->grho[0 * N + n] = gr[0];
        s->grho[1 * N + n] = gr[1];
        s->grho[2 * N + n] = gr[2];
    }
}

/* Hydrodynamic moments (Sec. II.B):
 *   rho u = sum_i c_i f_i + F/2,   p~ = sum_i f_i + u . grad rho / 2.
 * The half-force correction uses the same total force F that enters the
 * forcing term, mu grad phi plus the body force (the typeset correction
 * names only the surface-tension part).  Solid nodes carry u = 0, p~ = 0. */
static void stage_velocity(dsmo_sim* s) {
    long N = s->N;
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        if (is_solid(s, n)) {
            s->u[0 * N + n] = s->u[1 * N + n] = s->u[2 * N + n] = 0.0;
            s->p_t[n] = 0.0;
            continue;
        }
        double m0 = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
        for (int i = 0; i < s->Q; ++i) {
            double fi = s->f[(size_t)i * N + n];
            m0 += fi;
            mx += s->c[i][0] * fi;
            my += s->c[i][1] * fi;
            mz += s->c[i][2] * fi;
        }
        const double rho = s->rho[n];
        double ux = (mx + 0.5 * s->F[0 * N + n]) / rho;
        double uy = (my + 0.5 * s->F[1 * N + n]) / rho;
        double uz = (mz + 0.5 * s->F[2 * N + n]) / rho;
        s->u[0 * N + n] = ux;
        s->u[1 * N + n] = uy;
        s->u[2 * N + n] = uz;
        s->p_t[n] = m0 + 0.5 * (ux * s->grho[0 * N + n] + uy * s->grho[1 * N + n] + uz * s->grho[2 * N + n]);
    }
}

/* Local relaxation time: tau_s in the solid stage; in the fluid stage
 * tau = tau_3 + (tau_2 - tau_3) H(C2 - C3) (Sec. II.B), with the step
 * H(x) = 1 for x > 0 and 0 otherwise. */
static double relax_tau(const dsmo_sim* s, long n) {
    if (s->stage == 1) return s->tau_s;
    double C2 = s->phi[n], C3 = 1.0 - s->C1[n] - C2;
    return C2 - C3 > 0.0 ? s->p.tau : s->p.tau_gas;
}
static double relax_tau_g(const dsmo_sim* s) {
    return s->stage == 1 ? s->tau_gs : 0.5 + s->p.mobility / CS2;
}

/* BGK collisions with forcing, f* = f - (f - f_eq)/tau + F_i and
 * g* = g - (g - g_eq)/tau_g (Sec. II.B). */
static void stage_collide(dsmo_sim* s) {
    long N = s->N;
    int Q = s->Q, dim = s->p.dim;
    double tau_g = relax_tau_g(s);
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double u[3] = {s->u[0 * N + n], s->u[1 * N + n], s->u[2 * N + n]};
        double feq[19], geq[19], Fi[19];
        if (is_solid(s, n)) {
            for (int i = 0; i < Q; ++i) s->fs[(size_t)i * N + n] = 0.0;
        } else {
            double tau = relax_tau(s, n);
            double gr[3] = {s->grho[0 * N + n], s->grho[1 * N + n], s->grho[2 * N + n]};
            double F[3] = {s->F[0 * N + n], s->F[1 * N + n], s->F[2 * N + n]};
            dsmo_equilibrium_f(dim, s->p_t[n], s->rho[n], u, feq);
            dsmo_forcing(dim, tau, s->rho[n], u, gr, F, Fi);
            for (int i = 0; i < Q; ++i) {
                double fi = s->f[(size_t)i * N + n];
                s->fs[(size_t)i * N + n] = fi - (fi - feq[i]) / tau + Fi[i];
            }
        }
        dsmo_equilibrium_g(dim, s->phi[n], s->mu[n], u, geq);
        for (int i = 0; i < Q; ++i) {
            double gi = s->g[(size_t)i * N + n];
            s->gs[(size_t)i * N + n] = gi - (gi - geq[i]) / tau_g;
        }
    }
}

/* Wall fraction of the link from fluid node n along direction k (Sec. II.B,
 * interpolated bounce-back).  The solid is taken to follow the planar tanh
 * profile normal to the wall, so the distance of n from the C1 = 1/2 level
 * is xi = 2 alpha artanh(1 - 2 C1(n)); the wall normal is
 * n = grad C1 / |grad C1|, and along the link the distance is
 * D = xi / (n . c_k/|c_k|), as a fraction q = D / |c_k| of the link.
 * Readings: q is clamped to [0, 1]; a vanishing gradient or a link that does
 * not point towards the wall gives the halfway value q = 1/2. */
static double link_q(const dsmo_sim* s, long n, int k) {
    double t = 1.0 - 2.0 * s->C1[n];
    if (t < 0.0) t = 0.0;
    if (t > 1.0 - 1e-12) t = 1.0 - 1e-12;
    double xi = 2.0 * s->p.alpha * atanh(t);
    double gc[3];
    grad(s, s->C1, n, gc);
    double gn = sqrt(gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2]);
    if (gn < 1e-12) return 0.5;
    const int* ck = s->c[k];
    double len = sqrt((double)(ck[0] * ck[0] + ck[1] * ck[1] + ck[2] * ck[2]));
    double cos_nc = (gc[0] * ck[0] + gc[1] * ck[1] + gc[2] * ck[2]) / (gn * len);
    if (cos_nc <= 1e-6) return 0.5;
    double q = xi / cos_nc / len;
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    return q;
}

int dsmo_get_mask(const dsmo_sim* s, unsigned char* mask) {
    if (!s || !mask) return DSMO_EINVAL;
    memcpy(mask, s->mask, (size_t)s->N);
    return DSMO_OK;
}

double dsmo_link_q(dsmo_sim* s, long n, int k) {
    if (!s || n < 0 || n >= s->N || k < 1 || k >= s->Q) return -1.0;
    return link_q(s, n, k);
}

/* Streaming.  g streams at every node (periodic).  f streams at fluid nodes;
 * where the upstream node is solid the population is rebuilt with the
 * linear interpolated bounce-back of Bouzidi et al. (2001), using the wall
 * fraction q of the link from the node towards the wall (direction
 * k = opposite of i):
 *   q <  1/2:  f_i(x) = 2q f*_k(x) + (1 - 2q) f*_k(x + c_i)
 *   q >= 1/2:  f_i(x) = f*_k(x)/(2q) + (2q - 1)/(2q) f*_i(x)
 * When x + c_i is solid as well the second form is used with q >= 1/2.
 * Solid nodes hold f = 0. */
static void stage_stream(dsmo_sim* s) {
    long N = s->N;
    int Q = s->Q;
#pragma omp parallel for num_threads(threads_of(s)) schedule(static)
    for (long n = 0; n < N; ++n) {
        for (int i = 0; i < Q; ++i) s->g[(size_t)i * N + n] = s->gs[(size_t)i * N + nbr(s, n, i, -1)];
        if (is_solid(s, n)) {
            for (int i = 0; i < Q; ++i) s->f[(size_t)i * N + n] = 0.0;
            continue;
        }
        for (int i = 0; i < Q; ++i) {
            long up = nbr(s, n, i, -1);
            if (!is_solid(s, up)) {
                s->f[(size_t)i * N + n] = s->fs[(size_t)i * N + up];
                continue;
            }
            int k = s->opp[i];
            double q = link_q(s, n, k);
            long down = nbr(s, n, i, +1);
            int down_solid = is_solid(s, down);
            double v;
            if (q < 0.5 && !down_solid) {
                v = 2.0 * q * s->fs[(size_t)k * N + n] + (1.0 - 2.0 * q) * s->fs[(size_t)k * N + down];
            } else {
                if (down_solid && q < 0.5) q = 0.5;
                v = s->fs[(size_t)k * N + n] / (2.0 * q) +
                    (2.0 * q - 1.0) / (2.0 * q) * s->fs[(size_t)i * N + n];
            }
            s->f[(size_t)i * N + n] = v;
        }
    }
}

/* macroscopic fields of the current state: phi, mu, F, u, p~ */
static void observe(dsmo_sim* s) {
    stage_moment(s);
    stage_chemical_potential(s);
    stage_force(s);
    stage_density(s);
    stage_velocity(s);
}

/* one step: moments, chemical potential, force, velocity and pressure,
 * collision, streaming (the order of the method in Sec. II.B) */
/* One step; DSMO_EUNSTABLE (the step not taken) if the state it starts from
 * holds a non-finite C or u. */
static int one_step(dsmo_sim* s) {
    observe(s);
    long N = s->N;
    for (long n = 0; n < N; ++n)
        if (!isfinite(s->phi[n]) || !isfinite(s->u[n]) || !isfinite(s->u[N + n]) || !isfinite(s->u[2 * N + n]))
            return DSMO_EUNSTABLE;
    stage_collide(s);
    stage_stream(s);
    return DSMO_OK;
}

/* ------------------------------------------------------------------ */
/* initial conditions */

/* f = 0, g = g_eq(phi, mu(phi), u = 0) at every node, from phi held in
 * s->phi; the state is post-stream at t = 0 */
static void init_populations_from_phi(dsmo_sim* s) {
    long N = s->N;
    int Q = s->Q;
    stage_chemical_potential(s);
    memset(s->f, 0, (size_t)Q * N * sizeof(double));
    const double zero[3] = {0.0, 0.0, 0.0};
    for (long n = 0; n < N; ++n) {
        double geq[19];
        dsmo_equilibrium_g(s->p.dim, s->phi[n], s->mu[n], zero, geq);
        for (int i = 0; i < Q; ++i) s->g[(size_t)i * N + n] = geq[i];
    }
}

int dsmo_init_solid(dsmo_sim* s, int n_steps, double beta, double omega, double tau_s,
                    double mobility_s, int flags) {
    if (!s || n_steps < 0 || !(beta >= 0.0) || !(omega >= 0.0) || !(tau_s > 0.5) ||
        !(mobility_s > 0.0))
        return DSMO_EINVAL;
    s->beta = beta;
    s->omega = omega;
    s->tau_s = tau_s;
    s->tau_gs = 0.5 + mobility_s / CS2;
    if ((flags & DSMO_SOLID_RESET) || s->stage != 1) {
        /* sharp start C1 = 1[S] */
        s->stage = 1;
        for (long n = 0; n < s->N; ++n) s->phi[n] = s->mask[n] ? 1.0 : 0.0;
        init_populations_from_phi(s);
    }
    for (int t = 0; t < n_steps; ++t) {
        int rc = one_step(s);
        if (rc) return rc; /* C1 is not frozen from a non-finite state */
    }
    stage_moment(s);
    memcpy(s->C1, s->phi, (size_t)s->N * sizeof(double));
    if (flags & DSMO_SOLID_REMASK)
        for (long n = 0; n < s->N; ++n) s->mask[n] = s->C1[n] > 0.5 ? 1 : 0;
    return DSMO_OK;
}

int dsmo_set_solid_field(dsmo_sim* s, const double* C1) {
    if (!s || !C1) return DSMO_EINVAL;
    memcpy(s->C1, C1, (size_t)s->N * sizeof(double));
    if (s->stage == 1) s->stage = 0;
    return DSMO_OK;
}

int dsmo_set_liquid(dsmo_sim* s, const double* C2) {
    if (!s || !C2) return DSMO_EINVAL;
    s->stage = 2;
    memcpy(s->phi, C2, (size_t)s->N * sizeof(double));
    init_populations_from_phi(s);
    return DSMO_OK;
}

int dsmo_set_gravity(dsmo_sim* s, const double g[3]) {
    if (!s || !g) return DSMO_EINVAL;
    for (int d = 0; d < 3; ++d) s->p.gravity[d] = g[d];
    return DSMO_OK;
}

int dsmo_step(dsmo_sim* s, int n) {
    if (!s || n < 0) return DSMO_EINVAL;
    if (s->stage != 2) return DSMO_ESTATE;
    for (int t = 0; t < n; ++t) {
        int rc = one_step(s);
        if (rc) return rc;
    }
    return DSMO_OK;
}

/* ------------------------------------------------------------------ */
/* observables */

/* Discrete free energy, written so that its derivative with respect to the
 * evolving order parameter at a node is exactly the chemical potential used
 * by the step: the square-gradient terms are link sums
 *   (a^2 k / 2) |grad c|^2  ->  (a^2 k / (2 c_s^2)) sum_i w_i (c(x+c_i) - c(x))^2
 * (since sum_i w_i (c_i . grad c)^2 = c_s^2 |grad c|^2), whose derivative
 * with respect to c at a node is -a^2 k L[c].
 * Fluid stage: the three-component functional without its constant C1 terms,
 *   sum_x [k2/2 C2^2 (1-C2)^2 + k3/2 C3^2 (1-C3)^2] + gradient links of C2, C3.
 * Solid stage: the solid-relaxation functional, including the confining and
 * Omega terms.  Ekin = sum over fluid nodes of rho |u|^2 / 2. */
int dsmo_free_energy(dsmo_sim* s, double* Fout, double* Ekin) {
    if (!s) return DSMO_EINVAL;
    if (s->stage == 0) return DSMO_ESTATE;
    observe(s);
    long N = s->N;
    double a2 = s->p.alpha * s->p.alpha;
    double k1 = s->p.kappa[0], k2 = s->p.kappa[1], k3 = s->p.kappa[2];
    double link = a2 / (2.0 * CS2);
    double F = 0.0, E = 0.0;
    for (long n = 0; n < N; ++n) {
        if (s->stage == 2) {
            double C2 = s->phi[n], C3 = 1.0 - s->C1[n] - C2;
            double e = 0.5 * k2 * C2 * C2 * (1.0 - C2) * (1.0 - C2) +
                       0.5 * k3 * C3 * C3 * (1.0 - C3) * (1.0 - C3);
            for (int i = 0; i < s->Q; ++i) {
                long m = nbr(s, n, i, +1);
                double d2 = s->phi[m] - C2;
                double d3 = (1.0 - s->C1[m] - s->phi[m]) - C3;
                e += link * s->w[i] * (k2 * d2 * d2 + k3 * d3 * d3);
            }
            F += e;
        } else {
            double C1 = s->phi[n], k13 = k1 + k3;
            double e = 0.5 * k13 * C1 * C1 * (1.0 - C1) * (1.0 - C1);
            if (confine_derivative(s, n, C1) != 0.0) e += s->beta * (C1 - 0.5) * (C1 - 0.5);
            if (C1 < 0.0) e += s->omega * C1 * C1;
            if (C1 > 1.0) e += s->omega * (1.0 - C1) * (1.0 - C1);
            for (int i = 0; i < s->Q; ++i) {
                double d = s->phi[nbr(s, n, i, +1)] - C1;
                e += link * s->w[i] * k13 * d * d;
            }
            F += e;
        }
        if (!is_solid(s, n)) {
            double ux = s->u[n], uy = s->u[N + n], uz = s->u[2 * N + n];
            E += 0.5 * s->rho[n] * (ux * ux + uy * uy + uz * uz);
        }
    }
    if (Fout) *Fout = F;
    if (Ekin) *Ekin = E;
    return DSMO_OK;
}

int dsmo_mass(dsmo_sim* s, double m[3]) {
    if (!s || !m) return DSMO_EINVAL;
    if (s->stage == 0) return DSMO_ESTATE;
    stage_moment(s);
    double m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (long n = 0; n < s->N; ++n) {
        double C1 = s->stage == 2 ? s->C1[n] : s->phi[n];
        double C2 = s->stage == 2 ? s->phi[n] : 0.0;
        m1 += C1;
        m2 += C2;
        m3 += 1.0 - C1 - C2;
    }
    m[0] = m1;
    m[1] = m2;
    m[2] = m3;
    return DSMO_OK;
}

int dsmo_fields(dsmo_sim* s, double* C1, double* C2, double* C3, double* u, double* p) {
    if (!s) return DSMO_EINVAL;
    if (s->stage == 0) return DSMO_ESTATE;
    observe(s);
    long N = s->N;
    for (long n = 0; n < N; ++n) {
        double c1 = s->stage == 2 ? s->C1[n] : s->phi[n];
        double c2 = s->stage == 2 ? s->phi[n] : 0.0;
        if (C1) C1[n] = c1;
        if (C2) C2[n] = c2;
        if (C3) C3[n] = 1.0 - c1 - c2;
        if (p) p[n] = CS2 * s->p_t[n];
    }
    if (u)
        for (int d = 0; d < s->p.dim; ++d)
            memcpy(u + (size_t)d * N, s->u + (size_t)d * N, (size_t)N * sizeof(double));
    return DSMO_OK;
}

int dsmo_chemical_potential(dsmo_sim* s, double* mu) {
    if (!s || !mu) return DSMO_EINVAL;
    if (s->stage == 0) return DSMO_ESTATE;
    stage_moment(s);
    stage_chemical_potential(s);
    memcpy(mu, s->mu, (size_t)s->N * sizeof(double));
    return DSMO_OK;
}

int dsmo_get_populations(dsmo_sim* s, double* f, double* g) {
    if (!s) return DSMO_EINVAL;
    size_t bytes = (size_t)s->Q * s->N * sizeof(double);
    if (f) memcpy(f, s->f, bytes);
    if (g) memcpy(g, s->g, bytes);
    return DSMO_OK;
}

int dsmo_set_populations(dsmo_sim* s, const double* f, const double* g) {
    if (!s || !f || !g) return DSMO_EINVAL;
    if (s->stage == 0) s->stage = 2;
    size_t bytes = (size_t)s->Q * s->N * sizeof(double);
    memcpy(s->f, f, bytes);
    memcpy(s->g, g, bytes);
    return DSMO_OK;
}

int dsmo_set_postcollision(dsmo_sim* s, const double* fs, const double* gs) {
    if (!s || !fs || !gs) return DSMO_EINVAL;
    if (s->stage == 0) s->stage = 2;
    size_t bytes = (size_t)s->Q * s->N * sizeof(double);
    memcpy(s->fs, fs, bytes);
    memcpy(s->gs, gs, bytes);
    stage_stream(s);
    return DSMO_OK;
}
