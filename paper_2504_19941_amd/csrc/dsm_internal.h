// dsm_internal.h -- declarations shared by the host side of libdsm.so
// (dsm_api.hip) and the kernel launchers (dsm_kernels.hip, dsm_fused.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsm_lattice.h"

namespace dsm {

// Reduction slots (FP64).
enum {
    RED_C1 = 0,
    RED_C2 = 1,
    RED_C3 = 2,
    RED_FREE = 3,
    RED_EKIN = 4,
    RED_UMAX = 5,
    RED_NONFINITE = 6,
    RED_SLOTS = 8
};
constexpr int kReduceBlocks = 1024;  // partial sums per reduction (fixed order)
constexpr int kLinksPerNode = 2;     // capacity of the cut-link table, per lattice node

// One cut link of the fluid stage: f[dst] = ca f[a] + cb f[b] (population
// indices in the device layout).
struct LinkRec {
    unsigned dst, a, b;
    float ca, cb;
};

// One lattice of a batch as the batched step kernel sees it (the buffer
// pairs f[k], g[k] alternate with the step parity).
struct BatchInst {
    Geom geom;
    Phys phys;
    void* f[2];
    void* g[2];
    const float* c1;
    const uint8_t* mask;
    int* flag;
    const LinkRec* links;
    int nlinks;
    int half;
};
// One work item of the batched step: a tile of one lattice.
struct BatchItem {
    int inst, x0, y0, z0;
};
// A run of up to kBatchChunk consecutive cut links of one lattice, for the
// batched bounce-back.
constexpr int kBatchChunk = 256;
struct BatchChunk {
    int inst, first;
};

// Device arrays of one simulation, carved from the caller's buffer.
struct DevArrays {
    void* f[2];       // Q*N population elements each (FP32 or FP16)
    void* g[2];       // Q*N population elements, then the FP64 rest plane
    float* c1;        // [N]
    uint8_t* mask;    // [N]
    float* phi;       // [N] evolving order parameter (scratch)
    float* mu;        // [N] chemical potential (scratch)
    float* aux;       // [4][N] velocity planes and pressure (scratch)
    double* partials; // [kReduceBlocks][RED_SLOTS]
    double* red;      // [RED_SLOTS]
    int* flag;        // [4] non-finite flag of the step kernels
    int2* ent;        // [N] boundary nodes of the fluid stage: (node, mask of cut links)
    LinkRec* links;   // [kLinksPerNode * N] cut links as two-term records
    int* nlinks;      // [2] number of entries, number of records
};

// --- launchers (dsm_kernels.hip) -------------------------------------------
// pull != 0: the state buffers hold post-collision populations and the
// kernel streams them (with bounce-back) on the fly; pull == 0: they hold
// post-stream populations.
hipError_t launch_c1_from_mask(const uint8_t* mask, float* c1, long long N, hipStream_t st);
hipError_t launch_remask(const float* c1, uint8_t* mask, long long N, hipStream_t st);
hipError_t launch_copy(const float* src, float* dst, long long N, hipStream_t st);

hipError_t launch_moment(int dim, const Geom& g, Pop gsrc, float* phi, int pull, hipStream_t st);
hipError_t launch_mu(int dim, const Geom& g, const Phys& ph, const float* phi, const float* c1,
                     const uint8_t* mask, float* mu, hipStream_t st);
hipError_t launch_collide_split(int dim, const Geom& g, const Phys& ph, Pop fsrc,
                                Pop gsrc, Pop fdst, Pop gdst, const float* c1,
                                const float* phi, const float* mu, int pull, int* flag, hipStream_t st);
hipError_t launch_observe(int dim, const Geom& g, const Phys& ph, Pop fsrc, const float* c1,
                          const float* phi, const float* mu, int pull, float* aux, hipStream_t st);
hipError_t launch_init_populations(int dim, const Geom& g, const float* phi, const float* mu,
                                   Pop fdst, Pop gdst, hipStream_t st);
hipError_t launch_pull_state(int dim, const Geom& g, const Phys& ph, Pop fsrc,
                             Pop gsrc, const float* c1, Pop fdst, Pop gdst,
                             hipStream_t st);
hipError_t launch_reduce(int dim, const Geom& g, const Phys& ph, const float* c1, const float* phi,
                         const uint8_t* mask, const float* aux, Pop gsrc, int pull, double* partials,
                         double* red, hipStream_t st);

// --- interpolated bounce-back (dsm_links.hip) ------------------------------
// find: lists the fluid nodes with cut links (C1 fixed), count[0] entries;
// build: one record per cut link, count[1] records; bounce: writes the rebuilt
// populations into the solid slots they are pulled from, in the
// post-collision buffer f.
hipError_t launch_find_links(int dim, const Geom& g, const float* c1, int2* ent, int* count, hipStream_t st);
hipError_t launch_build_links(int dim, const Geom& g, double alpha, const float* c1, const int2* ent, int nent,
                              LinkRec* rec, long long cap, int* count, hipStream_t st);
hipError_t launch_bounce(Pop f, const LinkRec* rec, int count, hipStream_t st);

// --- fused step (dsm_fused.hip) ---------------------------------------------
// variant selects the workgroup tile (3D: 0 = 64x4, 1 = 64x8, 2 = 128x4
// columns; 2D: 0 = 256, 1 = 128, 2 = 64 columns); TZ is the number of planes
// each workgroup marches through.  In the fluid stage with pull != 0 the
// bounce-back slots of fsrc must have been written by launch_bounce.
int fused_tile_variants(int dim);
void fused_tile_shape(int dim, int variant, int* tx, int* ty);
hipError_t launch_step_batch(int dim, int variant, int half, int rho, const BatchInst* inst, const BatchItem* items,
                             int nitems, int* counter, int grid, int parity, int TZ, hipStream_t st);
int batch_blocks_per_cu(int dim, int variant, int half, int rho);
// workgroups of the single-lattice fused kernel (fluid stage) resident per CU
int fused_blocks_per_cu(int dim, int variant, int half, int rho);
// Modelled duration of one step of one lattice under a tiling (dsm_batch.hip):
// the schedule model of the batched step with this lattice as its only member
// and blocks_per_cu workgroups resident per CU.
double lattice_schedule_cost(const Geom& g, int dim, int variant, int planes, int blocks_per_cu, int cus);
hipError_t launch_bounce_batch(const BatchInst* inst, const BatchChunk* chunks, int nchunks, int parity,
                               int* counters, int ncounters, hipStream_t st);
hipError_t launch_batch_flags(const BatchInst* inst, int count, int* out, hipStream_t st);
hipError_t launch_step_fused(int dim, const Geom& g, const Phys& ph, Pop fsrc, Pop gsrc, Pop fdst, Pop gdst,
                             const float* c1, const uint8_t* mask, int pull, int* flag, int variant, int TZ,
                             hipStream_t st);

}  // namespace dsm
