/*
 * dsm.h -- C ABI of libdsm.so, the MI355X (gfx950) implementation of the
 * diffuse-solid ternary free-energy lattice Boltzmann step of
 * Oktasendra, Rennick, Avis, Panter and Kusumaatmaja, "The Diffuse Solid
 * Method for Wetting and Multiphase Fluid Simulations in Complex
 * Geometries" (arXiv 2504.19941), Sec. II.B.
 *
 * Components: 1 = diffuse solid (C1), 2 = liquid (C2), 3 = gas
 * (C3 = 1 - C1 - C2, Sec. II.A).  dim 2 runs D2Q9 (velocity set and weights
 * of Sec. II.B), dim 3 runs D3Q19; every axis is periodic.
 *
 * Layout.  Host fields are arrays of N = nx*ny*nz doubles in node order
 * n = x + nx*(y + ny*z) (x fastest; nz = 1 in 2D).  Vector fields (u) are
 * dim consecutive planes of N.  Population arrays are Q planes of N
 * ([Q][N], direction-major) in the direction order: rest, then each velocity
 * followed by its opposite -- D2Q9: (0,0) (1,0) (-1,0) (0,1) (0,-1) (1,1)
 * (-1,-1) (1,-1) (-1,1); D3Q19: (0,0,0) +-x +-y +-z (1,1,0) (-1,-1,0)
 * (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1)
 * (0,1,-1) (0,-1,1).
 *
 * Ownership.  The caller allocates ONE device buffer of dsm_required_bytes()
 * bytes (e.g. a torch uint8 CUDA tensor) and keeps it alive until
 * dsm_destroy(); the library carves every device array out of it and never
 * allocates device memory.  The library owns only the small host handle.
 * Host arrays passed in or out belong to the caller; any output pointer may
 * be NULL to skip that field.
 *
 * Ordering.  Every call enqueues its device work on the HIP stream given to
 * dsm_create().  dsm_step() returns without synchronising except when it
 * reaches a stability check (every reduce_every steps).  Calls that return
 * host data synchronise the stream.  A handle must not be used from two
 * threads at once.
 *
 * Errors.  Calls return DSM_OK (0) or a negative DSM_E* code; the message of
 * the last failure on the calling thread is returned by dsm_last_error().
 * Arguments are validated before any device work is issued, so invalid
 * arguments never touch the GPU.
 *
 * Arithmetic is FP32 on the device, with FP64 for the global reductions
 * (masses, free energy, kinetic energy).
 */
#ifndef DSM_H
#define DSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DSM_OK = 0,
    DSM_EINVAL = -1,    /* invalid argument                                   */
    DSM_ENOMEM = -2,    /* device buffer smaller than dsm_required_bytes()    */
    DSM_EDEVICE = -3,   /* a HIP call failed                                  */
    DSM_EUNSTABLE = -4, /* non-finite values found by the stability check     */
    DSM_ESTATE = -5     /* call out of order (e.g. dsm_step before a liquid)  */
};

/* flags of dsm_init_solid */
enum { DSM_SOLID_RESET = 1, DSM_SOLID_REMASK = 2 };

/* step implementations: the single fused kernel, or three kernels
 * (moment, chemical potential, collide-stream) kept as a cross-check */
enum { DSM_KERNEL_FUSED = 0, DSM_KERNEL_SPLIT = 1 };

/* population storage in device memory.  Arithmetic is FP32 either way.
 * FP16 stores every f and every moving g (i > 0) as an FP16 number holding
 * 4096 times the value (the populations of this scheme are deviations from
 * the rest state: f vanishes at rest and the moving g are small), which
 * halves the population traffic.  The rest population g_0, which carries
 * nearly all of the concentration C, is kept in FP64 in both modes and is
 * written as C minus the stored moving populations, so the component masses
 * are conserved to FP64 rounding in both modes. */
enum { DSM_STORAGE_FP32 = 0, DSM_STORAGE_FP16 = 1 };

typedef struct {
    int dim;             /* 2 (D2Q9, nz must be 1) or 3 (D3Q19)                  */
    int nx, ny, nz;      /* lattice size, each >= 4 (nz = 1 in 2D)               */
    double kappa[3];     /* kappa_1 solid, kappa_2 liquid, kappa_3 gas (>= 0,
                            kappa_2 + kappa_3 > 0); Sec. II.A bulk and gradient
                            energies with kappa'_n = alpha^2 kappa_n              */
    double alpha;        /* interface width (> 0); the paper uses 1               */
    double tau;          /* hydrodynamic relaxation time tau_2 of the liquid
                            (> 1/2); the gas takes tau_gas                       */
    double mobility;     /* Cahn-Hilliard mobility M (> 0): tau_g = 1/2 + 3 M    */
    double gravity[3];   /* body-force density on the liquid, F_g = C2 g          */
    int reduce_every;    /* K > 0: dsm_step checks for non-finite values every
                            K steps (synchronising); 0 disables the check        */
    int kernel;          /* DSM_KERNEL_FUSED (default) or DSM_KERNEL_SPLIT        */
    int storage;         /* DSM_STORAGE_FP32 (default) or DSM_STORAGE_FP16        */
    double rho[2];       /* densities rho_2 (liquid), rho_3 (gas) of Sec. II.B:
                            rho = rho_3 + (rho_2 - rho_3) C2 / (C2 + C3); each
                            > 0, or 0 for 1                                       */
    double tau_gas;      /* tau_3 of Sec. II.B: tau = tau_3 + (tau - tau_3)
                            H(C2 - C3); > 1/2, or 0 for tau (no contrast)         */
} dsm_params;

typedef struct dsm_sim dsm_sim;

/* Bytes of device memory a simulation with these parameters needs; 0 if the
 * parameters are invalid.  Pure host function. */
size_t dsm_required_bytes(const dsm_params* p);

/* Problem statement of Sec. II: lattice, solid region S (Sec. II.A, the
 * region the confining potential holds the solid to), kappa_m and alpha
 * (Sec. II.A), tau and M (Sec. II.B), body force.
 *   mask      host, N bytes, 1 where the node lies in S (may be NULL: S empty).
 *             The solid starts as the sharp indicator C1 = 1[S], with the
 *             cut links of interpolated bounce-back (Sec. II.B) built from
 *             it, so a liquid may be set on it without a solid stage (if
 *             they overflow the table, dsm_set_liquid returns DSM_ESTATE
 *             until a solid stage or dsm_set_solid_field succeeds).
 *   dev_buf   device pointer to dev_bytes >= dsm_required_bytes(p) bytes,
 *             256-byte aligned, owned by the caller.
 *   stream    hipStream_t (NULL = default stream) for all device work.
 *   out       receives the handle.
 * Errors: DSM_EINVAL (bad parameter or pointer), DSM_ENOMEM (dev_bytes too
 * small), DSM_EDEVICE. */
int dsm_create(const dsm_params* p, const uint8_t* mask, void* dev_buf, size_t dev_bytes,
               void* stream, dsm_sim** out);

/* Solid stage (Sec. II.B, the solid-relaxation functional "Free Energy1"
 * with the confining potential of Sec. II.A): n_steps lattice Boltzmann
 * steps with confining strength beta and range penalty Omega, relaxation
 * times tau_s and tau_g = 1/2 + 3 mobility_s, every node fluid, no body
 * force.  flags: DSM_SOLID_RESET restarts from C1 = 1[S] (otherwise the
 * solid stage continues from its live state, so a schedule can change beta
 * and Omega between calls); DSM_SOLID_REMASK replaces S by {C1 > 1/2} after
 * the run (the two-step initialisation for sharp corners of Sec. II.B).  On
 * return C1 is frozen to the relaxed field and the cut-link table of the
 * fluid stage is rebuilt from it; a liquid must then be set with
 * dsm_set_liquid.  Any stability flag of an earlier run is cleared first.
 * Errors: DSM_EINVAL, DSM_EUNSTABLE (non-finite values during the run),
 * DSM_EDEVICE.  After an error the handle holds no usable solid: the cut
 * links are dropped and dsm_set_liquid returns DSM_ESTATE until a solid
 * stage or dsm_set_solid_field succeeds. */
int dsm_init_solid(dsm_sim* s, int n_steps, double beta, double omega, double tau_s,
                   double mobility_s, int flags);

/* Alternative to the solid stage: a given diffuse solid C1 (host, N values
 * in node order; stored in FP32), e.g. the tanh profile of a signed distance
 * that the equilibrium interface of Sec. II.A takes (eqn:tanh).  Nodes with
 * C1 > 1/2 become solid nodes of the fluid stage (Sec. II.B) and the cut
 * links of interpolated bounce-back are rebuilt.  Invalidates any liquid
 * state.  Errors: DSM_EINVAL (NULL argument, or more cut links than the
 * table holds), DSM_EDEVICE. */
int dsm_set_solid_field(dsm_sim* s, const double* C1);

/* Liquid initial condition at t = 0 of the fluid stage (Sec. II.B; host,
 * N values of C2 in node order, with C3 = 1 - C1 - C2 as in Sec. II.A):
 * f = 0 and g = g_eq(C2, mu(C2), u = 0) at every node, with the equilibrium
 * g_eq and the chemical potential mu of the frozen-solid functional of
 * Sec. II.B.  Resets the step count and the stability flag.  Errors:
 * DSM_EINVAL, DSM_ESTATE (the last solid stage or solid field failed),
 * DSM_EDEVICE. */
int dsm_set_liquid(dsm_sim* s, const double* C2);

/* Replaces the body-force density g of the force F_g = C2 g on the liquid
 * (host, 3 values; the gravitational energy of Sec. III.B and the force on
 * the droplet of Sec. IV.B), between steps, e.g. for a ramp.  Takes effect
 * at the next step; no device work.  Errors: DSM_EINVAL (NULL, non-finite,
 * or g[2] != 0 when dim == 2). */
int dsm_set_gravity(dsm_sim* s, const double g[3]);

/* n fluid-stage time steps (Sec. II.B, frozen solid), stream-ordered.
 * Errors: DSM_EINVAL (n < 0), DSM_ESTATE (no liquid set), DSM_EUNSTABLE
 * (stability check failed; the state is left as computed), DSM_EDEVICE. */
int dsm_step(dsm_sim* s, int n);

/* dsm_step with HIP events recorded around every launch (synchronises at the
 * end): the mean duration, in ms, of the fused step kernel and of the
 * bounce-back link kernel that precedes it.  For measurement; the events add
 * a little time between launches.  Fused kernel only.  Errors: DSM_EINVAL,
 * DSM_ESTATE, DSM_EUNSTABLE, DSM_EDEVICE. */
int dsm_step_timed(dsm_sim* s, int n, double* step_ms, double* links_ms);

/* Discrete free energy of the current state (FP64 reduction; synchronises):
 * fluid stage, the frozen-solid functional of Sec. II.B without its constant
 * C1 terms; solid stage, the solid-relaxation functional.  Square gradients
 * are lattice link sums whose node derivative equals the step's chemical
 * potential.  E_kin = sum over fluid nodes of rho |u|^2 / 2.  Either pointer
 * may be NULL.  Errors: DSM_ESTATE, DSM_EDEVICE. */
int dsm_free_energy(dsm_sim* s, double* F, double* E_kin);

/* Total amounts m[k] = sum_x C_{k+1} (FP64 reduction; synchronises).  The
 * scheme conserves each component's amount (Sec. II.B: the zeroth moment of
 * g is C and both the collision and the streaming preserve it); the evolving
 * component is summed from the stored populations themselves, so a drift
 * measures the stored state.  Errors: DSM_EINVAL, DSM_ESTATE, DSM_EDEVICE. */
int dsm_mass(dsm_sim* s, double m[3]);

/* Macroscopic fields of the current state (synchronises; host arrays of N
 * doubles in node order): C1, C2, C3 = 1 - C1 - C2 (Sec. II.A), the velocity
 * u (dim planes; rho u = sum_i c_i f_i + F/2, Sec. II.B) and the pressure
 * P = p~ / 3, where p~ = sum_i f_i + u . grad(rho) / 2 is the zeroth moment
 * of f (Sec. II.B).  Solid nodes report u = 0 and P = 0.  Any pointer may be
 * NULL; only the requested outputs are computed and copied (u and P need a
 * pass of the velocity kernels, C1 and C2 one device-to-host copy each, C3
 * both copies).  Errors: DSM_EINVAL, DSM_ESTATE, DSM_EDEVICE. */
int dsm_fields(dsm_sim* s, double* C1, double* C2, double* C3, double* u, double* p);

/* Global diagnostics of the current state, from one FP64 reduction over
 * every node (synchronises): the amounts of dsm_mass, the free energy and
 * kinetic energy of dsm_free_energy, the largest speed max_x |u(x)| (u as in
 * dsm_fields, which measures how far a run is from a static equilibrium),
 * and the number of nodes holding a non-finite C1, C2 or u. */
typedef struct {
    double mass[3];
    double free_energy;
    double kinetic_energy;
    double max_speed;
    double nonfinite_nodes;
} dsm_diag;
int dsm_diagnostics(dsm_sim* s, dsm_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * results as dsm_diagnostics, bit for bit (the same kernels and grid), with
 * the reduction's workspace -- 1024 rows of 8 FP64 partial sums plus the 8
 * final sums, 65 600 bytes -- taken from a static device array that the
 * library holds on each GPU it runs on until the process ends, instead of
 * from the handle's buffer.  The workspace does not grow with the lattice,
 * so every lattice a handle accepts fits.  No call allocates or frees device
 * or pinned memory.  Calls on one GPU share the array: calls that overlap on
 * one GPU (from several threads or streams) race.  Synchronises the handle's
 * stream.  Errors: DSM_EINVAL (NULL argument), DSM_ESTATE (no live state),
 * DSM_EDEVICE. */
int dsm_diagnostics_noalloc(dsm_sim* s, dsm_diag* out);

/* The solid region S the confining potential currently holds the solid to
 * (Sec. II.A; host, N bytes in node order, 1 in S): the mask given to
 * dsm_create, or {C1 > 1/2} after a solid stage run with DSM_SOLID_REMASK
 * (the redefinition of the solid locations in the two-step initialisation of
 * Sec. II.B).  Synchronises.  Errors: DSM_EINVAL, DSM_EDEVICE. */
int dsm_solid_region(dsm_sim* s, uint8_t* mask);

/* Chemical potential mu of the current state (host, N values). */
int dsm_chemical_potential(dsm_sim* s, double* mu);

/* Post-stream populations of the current state as FP64 [Q][N] arrays, and
 * the inverse (the given arrays become the state at the current time).
 * Errors: DSM_ESTATE, DSM_EDEVICE. */
int dsm_get_populations(dsm_sim* s, double* f, double* g);
int dsm_set_populations(dsm_sim* s, const double* f, const double* g);

/* Sets the state to the streaming of the given post-collision populations
 * (FP64 [Q][N]); the next step starts by streaming them, with bounce-back. */
int dsm_set_postcollision(dsm_sim* s, const double* fs, const double* gs);

/* Checkpoint: an opaque byte image of the live state (populations, C1, S,
 * body force, step counter).  dsm_set_state on a handle created with the same
 * parameters continues bit-for-bit.  Errors: DSM_EINVAL (size mismatch),
 * DSM_ESTATE, DSM_EDEVICE. */
size_t dsm_state_bytes(const dsm_sim* s);
int dsm_get_state(dsm_sim* s, void* host, size_t bytes);
int dsm_set_state(dsm_sim* s, const void* host, size_t bytes);

/* Steps taken in the fluid stage since the last dsm_set_liquid. */
long long dsm_step_count(const dsm_sim* s);

/* Launch shape of the fused step kernel: the workgroup tile (variant in
 * [0, dsm_tiling_variants(dim)); 3D: 0 = 64x4, 1 = 64x8, 2 = 128x4 columns;
 * 2D: 0 = 256, 1 = 128, 2 = 64 columns) and the number of planes (1..4096)
 * each workgroup marches through along the slowest axis.  Every choice
 * computes bit-identical populations (each node's arithmetic does not depend
 * on the tile).  Defaults: 3D variant 2 with the march of 8, 16, 32, 48, 64,
 * 96 or 128 planes that takes the fewest whole rounds of tiles (at the
 * kernel's tiles per compute unit) times planes; 2D variant 0 with 16 planes, or 8 when the
 * lattice has too few 256-column tiles to give every compute unit whole
 * rounds of 16-plane marches.  dsm_create replaces that default by another
 * variant and a march of 8, 16 or 32 planes (in 2D also 4, for a variant
 * whose 8-plane grid makes less than one round of resident workgroups) when
 * a model of the step's duration (work over resident waves, per-variant wave
 * cost, fill planes and tail) predicts it at least 10 % faster, as for
 * narrow 2D rows, small lattices and rows just wider than a tile.  A
 * lattice whose default grid fills at most half a round of resident
 * workgroups is instead scored by whole rounds of its longest march, over
 * marches of 2 to 32 planes in 3D and 1 to 32 rows in 2D (small lattices,
 * whose marches all run at once).
 * Errors: DSM_EINVAL. */
int dsm_set_tiling(dsm_sim* s, int variant, int planes);
/* The launch shape in use (the default chosen by dsm_create, or the last
 * dsm_set_tiling): *variant and *planes as in dsm_set_tiling.  Either pointer
 * may be NULL.  Errors: DSM_EINVAL (s is NULL). */
int dsm_get_tiling(const dsm_sim* s, int* variant, int* planes);
int dsm_tiling_variants(int dim);

/* Measured tiling tuner: times every tile variant with each march of 2, 4,
 * 8, 16, 32, 48, 64, 96 and 128 planes (3D) or 1, 2, 4, 8, 16, 32, 64 and 128 (2D),
 * marches of Z planes or more timed once, on the lattice itself (one
 * untimed step, then reps steps timed as dsm_step_timed times them) and
 * installs the fastest.  Results do not depend on the tiling; the lattice
 * advances by 1 + reps steps per candidate (dsm_step_count tells how many).
 * *ms_per_step (may be NULL) receives the fused kernel's time per step under
 * the chosen tiling.  Fluid stage, fused kernel only; reps in [1, 1000].  On
 * an error the previous tiling is restored.  Errors: DSM_EINVAL, DSM_ESTATE,
 * DSM_EUNSTABLE, DSM_EDEVICE. */
int dsm_tune_tiling(dsm_sim* s, int reps, double* ms_per_step);

/* Releases the host handle (the device buffer stays the caller's). */
int dsm_destroy(dsm_sim* s);

/* ---- Batched form --------------------------------------------------------
 *
 * Many independent lattices of uneven sizes (2D and 3D, the same population
 * storage) advance together: each step is one bounce-back launch over the cut
 * links of every lattice, then one persistent launch of the fused step per
 * lattice type, in which every workgroup takes (lattice, tile) work items
 * from a shared counter until the list is drained.  The launches of one or
 * two steps are captured once in a HIP graph and replayed.  Each lattice's
 * result is bit-identical to stepping it alone with dsm_step (the per-node
 * arithmetic is the same code and does not depend on the tile; Sec. II,
 * eqns. of the fluid stage).
 *
 * Ownership.  The members stay owned by the caller and must outlive the
 * batch; the batch keeps its tables (descriptors, work items, link runs,
 * counters) in ONE caller-owned device buffer of dsm_batch_required_bytes()
 * bytes, 256-byte aligned, and never allocates device memory.  Between
 * batch calls a member may be used on its own (fields, energies, single
 * steps); dsm_batch_step picks up each member's current state.
 *
 * A member must be in the fluid stage and have taken at least one step since
 * dsm_set_liquid (its populations are then post-collision values, which is
 * the form the persistent kernel reads).  Members must be distinct and share
 * one population storage.  Errors: DSM_EINVAL, DSM_ESTATE, DSM_ENOMEM,
 * DSM_EDEVICE. */
typedef struct dsm_batch dsm_batch;

/* Work schedule of one lattice type in a batch. */
typedef struct dsm_batch_schedule {
    int variant;       /* workgroup tile, as in dsm_set_tiling */
    int planes;        /* planes per work item, 1..4096 */
    int blocks_per_cu; /* persistent workgroups per compute unit; 0 = as many as are resident at once */
} dsm_batch_schedule;

/* Bytes of the batch's device buffer for these members (0 if invalid). */
size_t dsm_batch_required_bytes(dsm_sim* const* sims, int count);

/* Builds the batch and its tables on `stream` (synchronises it).  Default
 * schedules: 3D variant 2 with 16 planes, 2D variant 0 with 32 planes, all
 * resident workgroups. */
int dsm_batch_create(dsm_sim* const* sims, int count, void* dev_buf, size_t dev_bytes, void* stream,
                     dsm_batch** out);

/* Schedule of the dim-dimensional members (dim 2 or 3). */
int dsm_batch_set_schedule(dsm_batch* b, int dim, const dsm_batch_schedule* sched);
int dsm_batch_get_schedule(const dsm_batch* b, int dim, dsm_batch_schedule* sched);

/* Autotuner, for each lattice type present (cost may be NULL; index 0: 2D,
 * 1: 3D; 0 where absent).  reps in [0, 1000].
 * reps == 0, modelled: scores every tile variant with each of the plane
 * counts 4, 8, 16, 32, 64 and 128 by a model of the batched step over the
 * members' actual shapes (waves per work item, the resident waves the
 * dynamic queue keeps busy, the tail left by the longest item, and a
 * per-variant cost of one wave-plane fitted to step times measured on
 * MI355X), and installs the best.  No device work is issued, so the
 * members' states and step counts are unchanged.  cost receives the
 * modelled cost, in wave-plane units.
 * reps > 0, measured: times every tile variant with each of those plane
 * counts and each count of resident workgroups per CU (0 = as many as fit,
 * then 1 .. min(fit - 1, 4)) on the batch itself: one untimed step, then
 * reps steps between two HIP events, synchronising before the next
 * candidate; installs the fastest.  Every member advances by 1 + reps steps
 * per candidate (dsm_step_count tells how many); results stay those of the
 * same lattices stepped alone.  cost receives the best time per step, in
 * ms.  Errors: DSM_EINVAL, DSM_ESTATE, DSM_EUNSTABLE, DSM_EDEVICE. */
int dsm_batch_tune(dsm_batch* b, int reps, double cost[2]);

/* Advances every member by n steps (n >= 0), then synchronises and checks
 * the members' stability flags: DSM_EUNSTABLE if any member holds
 * non-finite values (dsm_last_error names the first). */
int dsm_batch_step(dsm_batch* b, int n);

/* As dsm_batch_step, and reports the mean time per step (HIP events around
 * the graph launches, on the batch's stream). */
int dsm_batch_step_timed(dsm_batch* b, int n, double* ms_per_step);

/* Number of members; work items of the current schedules (2D, 3D). */
int dsm_batch_size(const dsm_batch* b);
int dsm_batch_items(const dsm_batch* b, int dim);

/* Releases the batch (its device buffer stays the caller's). */
int dsm_batch_destroy(dsm_batch* b);

/* Message of the last failed call on this thread ("" if none). */
const char* dsm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
