// dsm_host.h -- host-side state shared by the C-ABI sources (not installed).
#pragma once

#include <string>
#include <vector>

#include "dsm.h"
#include "dsm_internal.h"

// One lattice: parameters, carved device arrays and step bookkeeping.
struct dsm_sim {
    dsm_params p;
    int Q;
    long long N;
    dsm::Geom geom;
    hipStream_t stream;
    dsm::DevArrays d;
    int cur;       // buffer pair holding the live state
    int pull;      // 1: live buffers hold post-collision populations
    int stage;     // 0: no live state, 1: solid stage live, 2: fluid stage live
    long long steps;
    double beta, omega, tau_s, taug_s;
    int nlinks;        // boundary nodes with cut links (fluid stage)
    int solid_failed;  // the last solid stage failed: C1 and its cut links are unusable
    int tile_variant;  // workgroup tile of the fused step
    int tile_planes;   // planes marched per workgroup
    int half;      // populations stored in FP16 (value * kHalfScale)
    int es;        // bytes per population element
    std::vector<float> stage_buf;  // host staging for conversions
    std::vector<uint16_t> stage16;
};

namespace dsm {

// Records msg as the calling thread's last error and returns code.
int set_error(int code, const std::string& msg);
// Step parameters of stage 1 (solid) or 2 (fluid) of a lattice.
Phys sim_phys(const dsm_sim* s, int stage);
// Modelled duration of one step of a lattice whose grid makes a fraction of
// a round, where the step lasts whole rounds of its longest march
// (dsm_batch.hip; the throughput form is lattice_schedule_cost).
double lattice_latency_cost(const Geom& g, int dim, int variant, int planes, int blocks_per_cu, int cus, int half);

}  // namespace dsm
