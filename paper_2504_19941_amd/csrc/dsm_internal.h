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

// Device arrays of one simulation, carved from the caller's buffer.
struct DevArrays {
    float* f[2];      // [Q][N] each
    float* g[2];      // [Q][N] each
    float* c1;        // [N]
    uint8_t* mask;    // [N]
    float* phi;       // [N] evolving order parameter (scratch)
    float* mu;        // [N] chemical potential (scratch)
    float* aux;       // [4][N] velocity planes and pressure (scratch)
    double* partials; // [kReduceBlocks][RED_SLOTS]
    double* red;      // [RED_SLOTS]
    int* flag;        // [4] non-finite flag of the step kernels
};

// --- launchers (dsm_kernels.hip) -------------------------------------------
// pull != 0: the state buffers hold post-collision populations and the
// kernel streams them (with bounce-back) on the fly; pull == 0: they hold
// post-stream populations.
hipError_t launch_c1_from_mask(const uint8_t* mask, float* c1, long long N, hipStream_t st);
hipError_t launch_remask(const float* c1, uint8_t* mask, long long N, hipStream_t st);
hipError_t launch_copy(const float* src, float* dst, long long N, hipStream_t st);

hipError_t launch_moment(int dim, const Geom& g, const float* gsrc, float* phi, int pull, hipStream_t st);
hipError_t launch_mu(int dim, const Geom& g, const Phys& ph, const float* phi, const float* c1,
                     const uint8_t* mask, float* mu, hipStream_t st);
hipError_t launch_collide_split(int dim, const Geom& g, const Phys& ph, const float* fsrc,
                                const float* gsrc, float* fdst, float* gdst, const float* c1,
                                const float* phi, const float* mu, int pull, int* flag, hipStream_t st);
hipError_t launch_observe(int dim, const Geom& g, const Phys& ph, const float* fsrc, const float* c1,
                          const float* phi, const float* mu, int pull, float* aux, hipStream_t st);
hipError_t launch_init_populations(int dim, const Geom& g, const float* phi, const float* mu,
                                   float* fdst, float* gdst, hipStream_t st);
hipError_t launch_pull_state(int dim, const Geom& g, const Phys& ph, const float* fsrc,
                             const float* gsrc, const float* c1, float* fdst, float* gdst,
                             hipStream_t st);
hipError_t launch_reduce(int dim, const Geom& g, const Phys& ph, const float* c1, const float* phi,
                         const uint8_t* mask, const float* aux, double* partials, double* red,
                         hipStream_t st);

// --- fused step (dsm_fused.hip) ---------------------------------------------
// variant selects the workgroup tile (3D: 0 = 32x8, 1 = 64x4, 2 = 64x8,
// 3 = 32x16 columns; 2D: 0 = 128, 1 = 256, 2 = 64 columns); TZ is the number
// of planes each workgroup marches through.
int fused_tile_variants(int dim);
hipError_t launch_step_fused(int dim, const Geom& g, const Phys& ph, const float* fsrc,
                             const float* gsrc, float* fdst, float* gdst, const float* c1,
                             const uint8_t* mask, int pull, int* flag, int variant, int TZ,
                             hipStream_t st);

}  // namespace dsm
