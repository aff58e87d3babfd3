/*
 * dsm_oracle.h -- plain FP64 CPU oracle of the diffuse-solid ternary
 * free-energy lattice Boltzmann step (Oktasendra et al., "The Diffuse Solid
 * Method for Wetting and Multiphase Fluid Simulations in Complex
 * Geometries", arXiv 2504.19941, Sec. II.B).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Conventions
 *   component 1 = diffuse solid (C1), 2 = liquid (C2), 3 = gas (C3 = 1-C1-C2)
 *   node index n = x + nx*(y + ny*z), x fastest; dim 2 uses nz = 1
 *   populations are stored as [Q][N] planes, direction-major
 *   dim 2 -> D2Q9 (velocity set and weights as printed in Sec. II.B)
 *   dim 3 -> D3Q19 (rest, 6 axis links, 12 edge links, opposite pairs adjacent)
 *   all boundaries are periodic
 *
 * State between calls is the post-stream distribution at time t; one step is
 * collide (BGK with forcing) followed by streaming with interpolated
 * bounce-back at the diffuse solid.
 */
#ifndef DSM_ORACLE_H
#define DSM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DSMO_OK = 0,
    DSMO_EINVAL = -1,
    DSMO_ENOMEM = -2,
    DSMO_EUNSTABLE = -4,
    DSMO_ESTATE = -5
};

/* readings of the confining potential's case conditions (Sec. II.A and II.B):
 * 0 = penalise solid outside S and fluid inside S (the stated purpose),
 * 1 = the case conditions exactly as typeset (kept only so that a test can
 *     show that they fail to confine the solid). */
enum { DSMO_CONFINE_PURPOSE = 0, DSMO_CONFINE_AS_TYPESET = 1 };

/* readings of the surface-tension force (Sec. II.B states F_s = -C grad mu
 * and also writes the velocity moment with mu grad C):
 * 0 = F_s = mu grad C, the potential form the velocity moment carries,
 * 1 = F_s = -C grad mu as typeset (kept so that a test can compare them). */
enum { DSMO_FORCE_POTENTIAL = 0, DSMO_FORCE_AS_TYPESET = 1 };

/* init_solid flags */
enum { DSMO_SOLID_RESET = 1, DSMO_SOLID_REMASK = 2 };

typedef struct {
    int dim, nx, ny, nz;
    double kappa[3];     /* kappa_1 (solid), kappa_2 (liquid), kappa_3 (gas) */
    double alpha;        /* interface width */
    double tau;          /* hydrodynamic relaxation time (> 1/2) */
    double mobility;     /* Cahn-Hilliard mobility M > 0; tau_g = 1/2 + 3M */
    double gravity[3];   /* body-force density acting on the liquid: F_g = C2 g */
    int confine_reading; /* DSMO_CONFINE_* */
    int threads;         /* OpenMP threads for node loops (<= 1: serial) */
    /* Density and viscosity contrast of the fluid stage (Sec. II.B):
     * rho = rho_3 + (rho_2 - rho_3) C2 / (C2 + C3) and
     * tau = tau_3 + (tau_2 - tau_3) H(C2 - C3), with tau_2 = tau above.
     * rho_liquid = rho_gas = 1 and tau_gas = tau give the uniform fluid. */
    double rho_liquid;   /* rho_2 > 0 */
    double rho_gas;      /* rho_3 > 0 */
    double tau_gas;      /* tau_3 > 1/2 */
    int force_reading;   /* DSMO_FORCE_* */
} dsmo_params;

typedef struct dsmo_sim dsmo_sim;

int  dsmo_create(const dsmo_params* p, const unsigned char* mask, dsmo_sim** out);
void dsmo_destroy(dsmo_sim* s);
int  dsmo_num_directions(const dsmo_sim* s);

/* Solid stage (Sec. II.B, solid relaxation).  flags: RESET starts from the
 * sharp indicator C1 = 1[S]; otherwise the live solid-stage state continues.
 * REMASK replaces S by {C1 > 1/2} after the run.  C1 is frozen to the sum of
 * the solid-stage g populations when the call returns, unless a step meets
 * a non-finite state (DSMO_EUNSTABLE, nothing frozen). */
int  dsmo_init_solid(dsmo_sim* s, int n_steps, double beta, double omega,
                     double tau_s, double mobility_s, int flags);
/* Alternative to the solid stage: an externally given diffuse C1. */
int  dsmo_set_solid_field(dsmo_sim* s, const double* C1);
/* Liquid initial condition: f = 0, g = g_eq(C2, mu(C2), u = 0). */
int  dsmo_set_liquid(dsmo_sim* s, const double* C2);
int  dsmo_set_gravity(dsmo_sim* s, const double g[3]);
/* n fluid-stage steps.  DSMO_EUNSTABLE when a step starts from a state whose
 * order parameter or velocity is not finite at some node (that step is not
 * taken; the state is left as computed). */
int  dsmo_step(dsmo_sim* s, int n);

/* Observables of the current state. */
int  dsmo_free_energy(dsmo_sim* s, double* F, double* Ekin);
int  dsmo_mass(dsmo_sim* s, double m[3]);
/* C1, C2, C3, p: N values each; u: dim planes of N.  NULL skips a field.
 * p is the reported pressure c_s^2 * p~. */
int  dsmo_fields(dsmo_sim* s, double* C1, double* C2, double* C3, double* u, double* p);
int  dsmo_chemical_potential(dsmo_sim* s, double* mu);

/* Raw populations, [Q][N] each. */
int  dsmo_get_populations(dsmo_sim* s, double* f, double* g);
int  dsmo_set_populations(dsmo_sim* s, const double* f, const double* g);
/* Sets the state to stream(f*, g*): the given arrays are post-collision
 * populations, and the oracle performs its own streaming step on them. */
int  dsmo_set_postcollision(dsmo_sim* s, const double* fs, const double* gs);

/* The solid region S currently held (N bytes, 1 in S); after a solid stage
 * run with REMASK it is {C1 > 1/2}. */
int  dsmo_get_mask(const dsmo_sim* s, unsigned char* mask);

/* Wall fraction q of the link leaving fluid node n along direction k. */
double dsmo_link_q(dsmo_sim* s, long n, int k);

/* Lattice and local formulas, exposed for the moment identities. */
int  dsmo_lattice(int dim, int* c /* Q*3 */, double* w /* Q */);
void dsmo_equilibrium_f(int dim, double p_tilde, double rho, const double u[3], double* feq);
void dsmo_equilibrium_g(int dim, double C, double mu, const double u[3], double* geq);
void dsmo_forcing(int dim, double tau, double rho, const double u[3],
                  const double grad_rho[3], const double F[3], double* Fi);

#ifdef __cplusplus
}
#endif
#endif
