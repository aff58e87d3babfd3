// dsm_lattice.h -- device-side lattice descriptions and small helpers for the
// gfx950 kernels of libdsm.so.
//
// D2Q9 is the velocity set and weight vector of Sec. II.B; D3Q19 is used for
// 3D.  Both list the rest velocity first and then each velocity next to its
// opposite, so opp(i) = i + 1 for odd i and i - 1 for even i > 0.
//
// The 2D lattice is laid out as a 3D one with ny = 1: a 2D node (x, y) is
// stored at x + nx*y, i.e. the 3D position (x, 0, y), and a D2Q9 velocity
// (cx, cy) acts as (cx, 0, cy).  Every kernel is therefore written once for
// "planes" along the slowest axis.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsm {

template <int D>
struct Lattice;

template <>
struct Lattice<2> {
    static constexpr int Q = 9;
    // components along the stored (x, y, z) axes: D2Q9's y is the stored z
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int cz[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr float w[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                                   1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

template <>
struct Lattice<3> {
    static constexpr int Q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr float w[19] = {1.f / 3.f,
                                    1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Storage geometry: X fastest, Z slowest.  For dim 2, Y == 1.  Node-indexed
// arrays (C1, the mask, the split kernels' fields) are dense, n = x + X*row;
// population rows and the FP64 rest plane use the row pitch XP >= X, a whole
// number of 128-byte lines (see pop_index).
struct Geom {
    int X, Y, Z;
    long long N;   // X*Y*Z
    int XP;        // row pitch of the population and rest-plane layouts, in elements
    long long NP;  // XP*Y*Z
};

// Row pitch for populations of elem_bytes bytes: X rounded up to a multiple
// of 128 bytes, so every direction row of every lattice row starts on a line
// (a wave's 64 consecutive elements then fill whole lines, which the HBM
// writes without merging partial lines).
__host__ __device__ __forceinline__ int row_pitch(int X, int elem_bytes) {
    const int k = 128 / elem_bytes;
    return (X + k - 1) / k * k;
}

// Physical and scheme parameters in the form the kernels use them.
struct Phys {
    float k1, k2, k3;    // kappa_1..3
    float a2;            // alpha^2
    float alpha;
    float inv_tau;       // 1 / tau
    float inv_taug;      // 1 / tau_g
    float fpref;         // 1 - 1 / (2 tau)
    float grav[3];       // body force per unit liquid (stored axes)
    float beta, omega;   // solid stage
    int stage;           // 1 = solid stage (C1 evolves), 2 = fluid stage (C2 evolves)
    // density and viscosity contrast of the fluid stage: rho_2, rho_3, and
    // for the gas side (C2 <= C3) 1/tau_3 and 1 - 1/(2 tau_3)
    float rho2, rho3;
    float inv_tau3, fpref_gas;
    int contrast;        // 1: any of rho_2, rho_3 != 1 or tau_3 != tau
};

// Local density of the fluid stage, rho_3 + (rho_2 - rho_3) C2 / (C2 + C3)
// with C2 + C3 = 1 - C1 floored at 1e-6 and the fraction clamped to [0, 1].
__device__ __forceinline__ float local_density(const Phys& ph, float C2, float C1) {
    const float den = fmaxf(1.f - C1, 1e-6f);
    const float frac = fminf(fmaxf(C2 / den, 0.f), 1.f);
    return ph.rho3 + (ph.rho2 - ph.rho3) * frac;
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ long long node_index(const Geom& g, int x, int y, int z) {
    return (long long)x + (long long)g.X * ((long long)y + (long long)g.Y * (long long)z);
}

// Population layout in HBM, "row-interleaved": the Q populations of the X
// nodes of one lattice row (fixed stored y and z) are contiguous and
// direction-major, each direction row padded to the pitch XP, so population
// i of node n = x + X*row lives at (row*Q + i)*XP + x.  A wave reading one
// direction of one row segment then touches one contiguous, line-aligned
// run, and a node's Q values sit within Q*XP elements.  Padding is never
// read or written by the kernels.
// Population storage.  FP32 (4-byte) or FP16 (2-byte) elements; FP16 holds
// value * kHalfScale, since the populations of this scheme are deviations
// from the rest state (f is zero at rest, and the moving g are w_i mu plus
// advection, both small) whose magnitudes (1e-6 .. 1e-1) would otherwise sit
// in the subnormal range of FP16.
constexpr float kHalfScale = 4096.f;

// The g populations of one buffer: the Q*NP slots of the population layout,
// of which the moving directions i > 0 are used, followed (256-byte aligned)
// by the rest population g_0 of every node in FP64, rows of pitch XP
// (rest_index).  The rest
// population carries nearly all of C, so storing it in FP64 keeps the liquid
// mass from drifting by rounding at the scale of C (the moving populations
// are small and their rounding is negligible).
__host__ __device__ __forceinline__ long long pop_bytes(int Q, long long N, int elem_bytes) {
    return ((long long)Q * N * elem_bytes + 255) / 256 * 256;
}
__host__ __device__ __forceinline__ double* rest_plane(void* g, int Q, long long N, int elem_bytes) {
    return reinterpret_cast<double*>(reinterpret_cast<char*>(g) + pop_bytes(Q, N, elem_bytes));
}
__host__ __device__ __forceinline__ const double* rest_plane(const void* g, int Q, long long N, int elem_bytes) {
    return reinterpret_cast<const double*>(reinterpret_cast<const char*>(g) + pop_bytes(Q, N, elem_bytes));
}

// A population buffer as the non-fused kernels see it: element loads and
// stores in FP32 whatever the storage.
struct Pop {
    void* p;
    int half;  // 0: FP32 elements, 1: FP16 elements holding value * kHalfScale
    __device__ __forceinline__ float ld(long long k) const {
        if (half) return __half2float(reinterpret_cast<const __half*>(p)[k]) * (1.f / kHalfScale);
        return reinterpret_cast<const float*>(p)[k];
    }
    // stores v and returns the value as stored (after rounding)
    __device__ __forceinline__ float st(long long k, float v) const {
        if (half) {
            const __half h = __float2half(v * kHalfScale);
            reinterpret_cast<__half*>(p)[k] = h;
            return __half2float(h) * (1.f / kHalfScale);
        }
        reinterpret_cast<float*>(p)[k] = v;
        return v;
    }
    __device__ __forceinline__ double* rest(int Q, long long N) const { return rest_plane(p, Q, N, half ? 2 : 4); }
};

__host__ __device__ __forceinline__ long long pop_index(const Geom& g, int Q, int i, long long n) {
    const long long row = n / g.X;
    return (row * Q + i) * g.XP + (n - row * g.X);
}

// Element of node n in the FP64 rest plane.
__host__ __device__ __forceinline__ long long rest_index(const Geom& g, long long n) {
    const long long row = n / g.X;
    return row * g.XP + (n - row * g.X);
}

}  // namespace dsm
