// dsm_links.hip -- interpolated bounce-back at the diffuse solid (gfx950).
//
// Sec. II.B imposes no-slip on the solid with the interpolated bounce-back of
// Bouzidi et al., the wall distance taken from the tanh profile of C1
// (eqn:tanh).  In the pull scheme a fluid node x receives f_i from x - c_i;
// when that node is solid (C1 > 1/2) the link is cut and the population is
// rebuilt from post-collision values at fluid nodes:
//   q <  1/2 (x + c_i fluid):  f_i(x) = 2q f*_k(x) + (1 - 2q) f*_k(x + c_i)
//   otherwise:                 f_i(x) = f*_k(x)/(2q) + (2q - 1)/(2q) f*_i(x),
//                              with q raised to 1/2 when x + c_i is solid,
// where k is the direction opposite to i and q the wall fraction of the link
// from x towards the wall:
//   xi = 2 alpha artanh(1 - 2 C1(x)) (distance of x from the C1 = 1/2 level,
//        argument clamped to [0, 1 - 1e-12]),  n = G[C1](x) / |G[C1](x)|,
//   q = xi / (n . c_k/|c_k|) / |c_k| clamped to [0, 1]; q = 1/2 when |G[C1]|
//   vanishes or the link does not point towards the wall.
//
// The solid does not move in the fluid stage, so the cut links are found and
// their wall fractions evaluated (FP64) once, when C1 is fixed: each link
// becomes a record f[dst] = ca f[a] + cb f[b] over population indices.
// Before each fused step, k_bounce writes each rebuilt value into the slot the
// fluid node pulls from, i.e. population i of the solid node x - c_i, which
// carries no population of its own.  Each such slot has exactly one reader
// (x), and the records read only slots of fluid nodes, so the update runs in
// place without races, and the fused step needs no boundary code at all.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void decode3(const Geom& g, long long n, int& x, int& y, int& z) {
    x = (int)(n % g.X);
    const long long r = n / g.X;
    y = (int)(r % g.Y);
    z = (int)(r / g.Y);
}

template <int D>
__device__ __forceinline__ long long nb(const Geom& g, int x, int y, int z, int i, int s) {
    using L = Lattice<D>;
    return node_index(g, wrap(x + s * L::cx[i], g.X), wrap(y + s * L::cy[i], g.Y), wrap(z + s * L::cz[i], g.Z));
}

// One entry per fluid node with at least one cut link: (node, mask of cut
// directions i).
template <int D>
__global__ void __launch_bounds__(kBlock) k_find_links(Geom g, const float* __restrict__ c1, int2* __restrict__ ent,
                                                       int* __restrict__ count) {
    using L = Lattice<D>;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    if (c1[n] > 0.5f) return;
    int x, y, z;
    decode3(g, n, x, y, z);
    unsigned cut = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
        if (c1[nb<D>(g, x, y, z, i, -1)] > 0.5f) cut |= 1u << i;
    if (!cut) return;
    const int at = atomicAdd(count, 1);
    ent[at] = make_int2((int)n, (int)cut);
}

// For every cut link of every entry, the rebuilt population as a two-term
// combination of post-collision populations of fluid nodes, written to the
// slot it is pulled from: f[dst] = ca f[a] + cb f[b].  The wall geometry is
// evaluated in FP64.  count[1] reserves record slots; records beyond cap are
// not written (the caller checks the total).
template <int D>
__global__ void __launch_bounds__(kBlock) k_build_links(Geom g, double alpha, const float* __restrict__ c1,
                                                        const int2* __restrict__ ent, int nent,
                                                        LinkRec* __restrict__ rec, long long cap,
                                                        int* __restrict__ count) {
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    const long long n = ent[e].x;
    const unsigned cut = (unsigned)ent[e].y;
    int x, y, z;
    decode3(g, n, x, y, z);
    // G[C1](x) = 3 sum_i w_i c_i C1(x + c_i)
    double gc0 = 0.0, gc1 = 0.0, gc2 = 0.0;
    for (int i = 1; i < Q; ++i) {
        const double v = (double)c1[nb<D>(g, x, y, z, i, +1)];
        const int l2 = L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
        const double wi = l2 == 1 ? (D == 2 ? 1.0 / 9.0 : 1.0 / 18.0) : 1.0 / 36.0;
        gc0 += wi * L::cx[i] * v;
        gc1 += wi * L::cy[i] * v;
        gc2 += wi * L::cz[i] * v;
    }
    gc0 *= 3.0;
    gc1 *= 3.0;
    gc2 *= 3.0;
    const double gn = sqrt(gc0 * gc0 + gc1 * gc1 + gc2 * gc2);
    double tt = 1.0 - 2.0 * (double)c1[n];
    tt = tt < 0.0 ? 0.0 : (tt > 1.0 - 1e-12 ? 1.0 - 1e-12 : tt);
    const double xi = 2.0 * alpha * atanh(tt);
    const long long base = atomicAdd(count + 1, __popc(cut));
    long long r = base;
    for (int i = 1; i < Q; ++i) {
        if (!((cut >> i) & 1u)) continue;
        const int k = opp(i);
        double q = 0.5;
        if (gn >= 1e-12) {
            const int l2 = L::cx[k] * L::cx[k] + L::cy[k] * L::cy[k] + L::cz[k] * L::cz[k];
            const double len = l2 == 1 ? 1.0 : 1.4142135623730951;
            const double cosnc = (gc0 * L::cx[k] + gc1 * L::cy[k] + gc2 * L::cz[k]) / (gn * len);
            if (cosnc > 1e-6) {
                q = xi / cosnc / len;
                q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
            }
        }
        const long long dn = nb<D>(g, x, y, z, i, +1);
        LinkRec lr;
        lr.dst = (unsigned)pop_index(g, Q, i, nb<D>(g, x, y, z, i, -1));
        lr.a = (unsigned)pop_index(g, Q, k, n);
        if (q < 0.5 && !(c1[dn] > 0.5f)) {
            lr.b = (unsigned)pop_index(g, Q, k, dn);
            lr.ca = (float)(2.0 * q);
            lr.cb = (float)(1.0 - 2.0 * q);
        } else {
            if (q < 0.5) q = 0.5;
            lr.b = (unsigned)pop_index(g, Q, i, n);
            lr.ca = (float)(1.0 / (2.0 * q));
            lr.cb = (float)((2.0 * q - 1.0) / (2.0 * q));
        }
        if (r < cap) rec[r] = lr;
        ++r;
    }
}

// Per step: one thread per cut link.  All reads are populations of fluid
// nodes and all writes go to slots of solid nodes, so the threads are
// independent and the update runs in place.
__global__ void __launch_bounds__(kBlock) k_bounce(Pop f, const LinkRec* __restrict__ rec, int count) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const LinkRec lr = rec[r];
    f.st(lr.dst, lr.ca * f.ld(lr.a) + lr.cb * f.ld(lr.b));
}

// Batched form: one workgroup per run of kBatchChunk links of one lattice.
// Workgroup 0 also resets the work counters of the batched step kernels that
// follow it on the stream.
__global__ void __launch_bounds__(kBatchChunk)
    k_bounce_batch(const BatchInst* __restrict__ inst, const BatchChunk* __restrict__ chunks, int nchunks,
                   int parity, int* __restrict__ counters, int ncounters) {
    if (blockIdx.x == 0 && (int)threadIdx.x < ncounters) counters[threadIdx.x] = 0;
    if ((int)blockIdx.x >= nchunks) return;
    const BatchChunk ch = chunks[blockIdx.x];
    const BatchInst& d = inst[ch.inst];
    const int r = ch.first + (int)threadIdx.x;
    if (r >= d.nlinks) return;
    const LinkRec lr = d.links[r];
    const Pop f{d.f[parity], d.half};
    f.st(lr.dst, lr.ca * f.ld(lr.a) + lr.cb * f.ld(lr.b));
}

// out[k] = flag word of lattice k (non-zero: non-finite values were seen).
__global__ void __launch_bounds__(kBlock) k_batch_flags(const BatchInst* __restrict__ inst, int count,
                                                        int* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) out[k] = inst[k].flag[0];
}

}  // namespace

hipError_t launch_bounce_batch(const BatchInst* inst, const BatchChunk* chunks, int nchunks, int parity,
                               int* counters, int ncounters, hipStream_t st) {
    const unsigned blocks = (unsigned)(nchunks > 0 ? nchunks : 1);
    hipLaunchKernelGGL(k_bounce_batch, dim3(blocks), dim3(kBatchChunk), 0, st, inst, chunks, nchunks, parity,
                       counters, ncounters);
    return hipGetLastError();
}

hipError_t launch_batch_flags(const BatchInst* inst, int count, int* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_batch_flags, dim3(blocks), dim3(kBlock), 0, st, inst, count, out);
    return hipGetLastError();
}

hipError_t launch_find_links(int dim, const Geom& g, const float* c1, int2* ent, int* count, hipStream_t st) {
    const unsigned blocks = (unsigned)((g.N + kBlock - 1) / kBlock);
    hipError_t e = hipMemsetAsync(count, 0, 2 * sizeof(int), st);
    if (e != hipSuccess) return e;
    if (dim == 2)
        hipLaunchKernelGGL(k_find_links<2>, dim3(blocks), dim3(kBlock), 0, st, g, c1, ent, count);
    else
        hipLaunchKernelGGL(k_find_links<3>, dim3(blocks), dim3(kBlock), 0, st, g, c1, ent, count);
    return hipGetLastError();
}

hipError_t launch_build_links(int dim, const Geom& g, double alpha, const float* c1, const int2* ent, int nent,
                              LinkRec* rec, long long cap, int* count, hipStream_t st) {
    if (nent <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((nent + kBlock - 1) / kBlock);
    if (dim == 2)
        hipLaunchKernelGGL(k_build_links<2>, dim3(blocks), dim3(kBlock), 0, st, g, alpha, c1, ent, nent, rec, cap,
                           count);
    else
        hipLaunchKernelGGL(k_build_links<3>, dim3(blocks), dim3(kBlock), 0, st, g, alpha, c1, ent, nent, rec, cap,
                           count);
    return hipGetLastError();
}

hipError_t launch_bounce(Pop f, const LinkRec* rec, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_bounce, dim3(blocks), dim3(kBlock), 0, st, f, rec, count);
    return hipGetLastError();
}

}  // namespace dsm
