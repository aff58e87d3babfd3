// dsm_kernels.hip -- set-up, observation, reduction and three-kernel step
// kernels of libdsm.so (gfx950).
//
// The three-kernel step (moment -> chemical potential -> collide/stream) is
// the straightforward form of one time step of Sec. II.B: each kernel is one
// pass over the nodes, with neighbours read through the caches.  It is kept
// beside the fused single-pass kernel (dsm_fused.hip) as an independent GPU
// formulation of the same step.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long N, int block = kBlock) {
    long long b = (N + block - 1) / block;
    return (unsigned)(b < 1 ? 1 : b);
}

__device__ __forceinline__ void decode(const Geom& g, long long n, int& x, int& y, int& z) {
    x = (int)(n % g.X);
    long long r = n / g.X;
    y = (int)(r % g.Y);
    z = (int)(r / g.Y);
}

// index of (x, y, z) + s * c_i, periodic
template <int D>
__device__ __forceinline__ long long shifted(const Geom& g, int x, int y, int z, int i, int s) {
    using L = Lattice<D>;
    return node_index(g, wrap(x + s * L::cx[i], g.X), wrap(y + s * L::cy[i], g.Y),
                      wrap(z + s * L::cz[i], g.Z));
}

// L[a](x) = 6 sum_i w_i (a(x + c_i) - a(x))
template <int D>
__device__ __forceinline__ float laplacian(const Geom& g, const float* a, int x, int y, int z, float a0) {
    using L = Lattice<D>;
    float acc = 0.f;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) acc += L::w[i] * (a[shifted<D>(g, x, y, z, i, +1)] - a0);
    return 6.f * acc;
}

// G[a](x) = 3 sum_i w_i c_i a(x + c_i), written as differences of opposite pairs
template <int D>
__device__ __forceinline__ void gradient(const Geom& g, const float* a, int x, int y, int z, float out[3]) {
    using L = Lattice<D>;
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        float d = a[shifted<D>(g, x, y, z, i, +1)] - a[shifted<D>(g, x, y, z, i + 1, +1)];
        gx += L::w[i] * L::cx[i] * d;
        gy += L::w[i] * L::cy[i] * d;
        gz += L::w[i] * L::cz[i] * d;
    }
    out[0] = 3.f * gx;
    out[1] = 3.f * gy;
    out[2] = 3.f * gz;
}

__device__ __forceinline__ float s_i(float cu, float uu) { return 3.f * cu + 4.5f * cu * cu - 1.5f * uu; }

// G[rho](x) for the local density of the fluid stage, from C2 = phi and C1
template <int D>
__device__ __forceinline__ void density_gradient(const Geom& g, const Phys& ph, const float* phi, const float* c1,
                                                 int x, int y, int z, float out[3]) {
    using L = Lattice<D>;
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        const long long a = shifted<D>(g, x, y, z, i, +1), b = shifted<D>(g, x, y, z, i + 1, +1);
        const float d = local_density(ph, phi[a], c1[a]) - local_density(ph, phi[b], c1[b]);
        gx += L::w[i] * L::cx[i] * d;
        gy += L::w[i] * L::cy[i] * d;
        gz += L::w[i] * L::cz[i] * d;
    }
    out[0] = 3.f * gx;
    out[1] = 3.f * gy;
    out[2] = 3.f * gz;
}

// Wall fraction of the link from fluid node n along direction k, from the
// tanh profile of the diffuse solid (Sec. II.B).  FP64: it is evaluated only
// on links that cross the solid boundary.
template <int D>
__device__ double link_fraction(const double gc[3], double gnorm, double xi, int k) {
    using L = Lattice<D>;
    if (gnorm < 1e-12) return 0.5;
    double len = sqrt((double)(L::cx[k] * L::cx[k] + L::cy[k] * L::cy[k] + L::cz[k] * L::cz[k]));
    double cosnc = (gc[0] * L::cx[k] + gc[1] * L::cy[k] + gc[2] * L::cz[k]) / (gnorm * len);
    if (cosnc <= 1e-6) return 0.5;
    double q = xi / cosnc / len;
    return q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
}

// Post-stream f at fluid node n = (x, y, z) from post-collision fsrc, with the
// linear interpolated bounce-back of Bouzidi et al. where the upstream node
// is solid (C1 > 1/2).
template <int D>
__device__ void pull_f(const Geom& g, Pop fsrc, const float* c1, float alpha, int x, int y,
                       int z, long long n, float fout[Lattice<D>::Q]) {
    using L = Lattice<D>;
    unsigned cut = 0;
    long long up[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        up[i] = shifted<D>(g, x, y, z, i, -1);
        if (i > 0 && c1[up[i]] > 0.5f) cut |= 1u << i;
    }
    if (!cut) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) fout[i] = fsrc.ld(pop_index(g, L::Q, i, up[i]));
        return;
    }
    double gc[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i < L::Q; ++i) {
        double v = (double)c1[shifted<D>(g, x, y, z, i, +1)];
        double wi = (L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i]) == 1
                        ? (D == 2 ? 1.0 / 9.0 : 1.0 / 18.0)
                        : 1.0 / 36.0;
        gc[0] += wi * L::cx[i] * v;
        gc[1] += wi * L::cy[i] * v;
        gc[2] += wi * L::cz[i] * v;
    }
    gc[0] *= 3.0;
    gc[1] *= 3.0;
    gc[2] *= 3.0;
    double gnorm = sqrt(gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2]);
    double t = 1.0 - 2.0 * (double)c1[n];
    t = t < 0.0 ? 0.0 : (t > 1.0 - 1e-12 ? 1.0 - 1e-12 : t);
    double xi = 2.0 * (double)alpha * atanh(t);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        if (!((cut >> i) & 1u)) {
            fout[i] = fsrc.ld(pop_index(g, L::Q, i, up[i]));
            continue;
        }
        const int k = opp(i);
        double q = link_fraction<D>(gc, gnorm, xi, k);
        long long dn = shifted<D>(g, x, y, z, i, +1);
        bool down_solid = c1[dn] > 0.5f;
        double fk = (double)fsrc.ld(pop_index(g, L::Q, k, n));
        double v;
        if (q < 0.5 && !down_solid) {
            v = 2.0 * q * fk + (1.0 - 2.0 * q) * (double)fsrc.ld(pop_index(g, L::Q, k, dn));
        } else {
            if (q < 0.5) q = 0.5;
            v = fk / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * (double)fsrc.ld(pop_index(g, L::Q, i, n));
        }
        fout[i] = (float)v;
    }
}

// ----------------------------------------------------------------------------

__global__ void k_c1_from_mask(const uint8_t* __restrict__ mask, float* __restrict__ c1, long long N) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) c1[n] = mask[n] ? 1.f : 0.f;
}

__global__ void k_remask(const float* __restrict__ c1, uint8_t* __restrict__ mask, long long N) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) mask[n] = c1[n] > 0.5f ? 1 : 0;
}

__global__ void k_copy(const float* __restrict__ src, float* __restrict__ dst, long long N) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) dst[n] = src[n];
}

// C = sum_i g_i (post-stream g)
template <int D>
__global__ void k_moment(Geom g, Pop gsrc, float* __restrict__ phi, int pull) {
    using L = Lattice<D>;
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    decode(g, n, x, y, z);
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        long long src = pull ? shifted<D>(g, x, y, z, i, -1) : n;
        acc += (double)gsrc.ld(pop_index(g, L::Q, i, src));
    }
    phi[n] = (float)(gsrc.rest(L::Q, g.NP)[rest_index(g, n)] + acc);
}

// chemical potential of the fluid stage (mu = dPsi/dC2) or of the solid stage
// (mu_1 = dPsi/dC1 with confinement and range penalty)
template <int D>
__global__ void k_mu(Geom g, Phys ph, const float* __restrict__ phi, const float* __restrict__ c1,
                     const uint8_t* __restrict__ mask, float* __restrict__ mu) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    decode(g, n, x, y, z);
    float p0 = phi[n];
    float lp = laplacian<D>(g, phi, x, y, z, p0);
    float m;
    if (ph.stage == 2) {
        float C1 = c1[n];
        float lc1 = laplacian<D>(g, c1, x, y, z, C1);
        float S = C1 + p0;
        m = ph.k2 * p0 * (1.f - p0) * (1.f - 2.f * p0) + ph.k3 * S * (1.f - S) * (1.f - 2.f * S) -
            ph.a2 * ph.k2 * lp - ph.a2 * ph.k3 * (lc1 + lp);
    } else {
        float k13 = ph.k1 + ph.k3;
        m = k13 * p0 * (1.f - p0) * (1.f - 2.f * p0);
        bool inS = mask[n] != 0;
        if ((p0 < 0.5f && inS) || (p0 > 0.5f && !inS)) m += 2.f * ph.beta * (p0 - 0.5f);
        m -= ph.a2 * k13 * lp;
        if (p0 < 0.f) m += 2.f * ph.omega * p0;
        if (p0 > 1.f) m -= 2.f * ph.omega * (1.f - p0);
    }
    mu[n] = m;
}

// velocity, pressure, collision and streaming-in-place of one node.
// Mode 0: write post-collision populations to fdst/gdst.
// Mode 1: write u (dim planes) and the pressure P = p~/3 to aux.
template <int D, int MODE>
__global__ void k_collide(Geom g, Phys ph, Pop fsrc, Pop gsrc,
                          Pop fdst, Pop gdst, const float* __restrict__ c1,
                          const float* __restrict__ phi, const float* __restrict__ mu, int pull,
                          int* __restrict__ flag, float* __restrict__ aux) {
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const long long N = g.N;
    int x, y, z;
    decode(g, n, x, y, z);
    const float C = phi[n];
    const bool solid = ph.stage == 2 && c1[n] > 0.5f;
    float ux = 0.f, uy = 0.f, uz = 0.f, pt = 0.f;
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    float rho = 1.f, gr[3] = {0.f, 0.f, 0.f};
    float f[Q];
    if (!solid) {
        // surface tension in the potential form mu grad C, plus the body force
        float gp[3];
        gradient<D>(g, phi, x, y, z, gp);
        const float m0 = mu[n];
        Fx = m0 * gp[0];
        Fy = m0 * gp[1];
        Fz = m0 * gp[2];
        if (ph.stage == 2) {
            Fx += C * ph.grav[0];
            Fy += C * ph.grav[1];
            Fz += C * ph.grav[2];
        }
        if (pull) {
            if (ph.stage == 2) {
                pull_f<D>(g, fsrc, c1, ph.alpha, x, y, z, n, f);
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) f[i] = fsrc.ld(pop_index(g, L::Q, i, shifted<D>(g, x, y, z, i, -1)));
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fsrc.ld(pop_index(g, L::Q, i, n));
        }
        float mx = 0.f, my = 0.f, mz = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            pt += f[i];
            mx += L::cx[i] * f[i];
            my += L::cy[i] * f[i];
            mz += L::cz[i] * f[i];
        }
        ux = mx + 0.5f * Fx;
        uy = my + 0.5f * Fy;
        uz = mz + 0.5f * Fz;
        if (ph.contrast) {
            // rho u = sum c_i f_i + F/2;  p~ = sum f_i + u . grad rho / 2
            rho = local_density(ph, C, c1[n]);
            density_gradient<D>(g, ph, phi, c1, x, y, z, gr);
            ux /= rho;
            uy /= rho;
            uz /= rho;
            pt += 0.5f * (ux * gr[0] + uy * gr[1] + uz * gr[2]);
        }
    }
    if (MODE == 1) {
        // stored axes -> user axes: 2D uses (x, z) as (x, y)
        aux[n] = ux;
        if (D == 2) {
            aux[N + n] = uz;
        } else {
            aux[N + n] = uy;
            aux[2 * N + n] = uz;
        }
        aux[3 * N + n] = pt * (1.f / 3.f);
        return;
    }
    const float uu = ux * ux + uy * uy + uz * uz;
    if (solid) {
#pragma unroll
        for (int i = 0; i < Q; ++i) fdst.st(pop_index(g, L::Q, i, n), 0.f);
    } else {
        // tau = tau_3 + (tau_2 - tau_3) H(C2 - C3) under contrast
        const bool gas = ph.contrast && !(C - (1.f - c1[n] - C) > 0.f);
        const float itau = gas ? ph.inv_tau3 : ph.inv_tau, fpref = gas ? ph.fpref_gas : ph.fpref;
        const float ug = ux * gr[0] + uy * gr[1] + uz * gr[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
            float cF = L::cx[i] * Fx + L::cy[i] * Fy + L::cz[i] * Fz;
            float si = s_i(cu, uu);
            float feq = L::w[i] * (pt + rho * si);
            float cg = L::cx[i] * gr[0] + L::cy[i] * gr[1] + L::cz[i] * gr[2] - ug;
            float Fi = fpref * L::w[i] * (3.f * cF + cg * si);
            fdst.st(pop_index(g, L::Q, i, n), f[i] - (f[i] - feq) * itau + Fi);
        }
    }
    const float m = mu[n];
    float gi[Q];
    double C64 = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        long long src = pull ? shifted<D>(g, x, y, z, i, -1) : n;
        gi[i] = gsrc.ld(pop_index(g, L::Q, i, src));
        C64 += (double)gi[i];
    }
    C64 += gsrc.rest(Q, g.NP)[rest_index(g, n)];
    // rest population (FP64) = C - sum of the moving post-collision populations
    double moved = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        float cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
        float geq = L::w[i] * m + L::w[i] * C * s_i(cu, uu);
        float gs = gi[i] - (gi[i] - geq) * ph.inv_taug;
        moved += (double)gdst.st(pop_index(g, L::Q, i, n), gs);
    }
    gdst.rest(Q, g.NP)[rest_index(g, n)] = C64 - moved;
    if (!isfinite(C) || !isfinite(uu)) flag[0] = 1;
}

// t = 0 state: f = 0, g = g_eq(phi, mu, u = 0), as post-stream populations
template <int D>
__global__ void k_init_populations(Geom g, const float* __restrict__ phi, const float* __restrict__ mu,
                                   Pop fdst, Pop gdst) {
    using L = Lattice<D>;
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const float C = phi[n], m = mu[n];
    double moved = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const float geq = L::w[i] * m;
        moved += (double)gdst.st(pop_index(g, L::Q, i, n), geq);
        fdst.st(pop_index(g, L::Q, i, n), 0.f);
    }
    gdst.st(pop_index(g, L::Q, 0, n), 0.f);  // unused slot: the rest population is FP64
    gdst.rest(L::Q, g.NP)[rest_index(g, n)] = (double)C - moved;
    fdst.st(pop_index(g, L::Q, 0, n), 0.f);
}

// post-collision -> post-stream (with bounce-back for f in the fluid stage)
template <int D>
__global__ void k_pull_state(Geom g, Phys ph, Pop fsrc, Pop gsrc,
                             const float* __restrict__ c1, Pop fdst, Pop gdst) {
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    decode(g, n, x, y, z);
#pragma unroll
    for (int i = 1; i < Q; ++i) gdst.st(pop_index(g, L::Q, i, n), gsrc.ld(pop_index(g, L::Q, i, shifted<D>(g, x, y, z, i, -1))));
    gdst.st(pop_index(g, L::Q, 0, n), 0.f);
    gdst.rest(Q, g.NP)[rest_index(g, n)] = gsrc.rest(Q, g.NP)[rest_index(g, n)];
    const bool solid = ph.stage == 2 && c1[n] > 0.5f;
    float f[Q];
    if (solid) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = 0.f;
    } else if (ph.stage == 2) {
        pull_f<D>(g, fsrc, c1, ph.alpha, x, y, z, n, f);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = fsrc.ld(pop_index(g, L::Q, i, shifted<D>(g, x, y, z, i, -1)));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) fdst.st(pop_index(g, L::Q, i, n), f[i]);
}

// --- FP64 reductions -------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// per-node contributions: masses, discrete free energy (link form), kinetic
// energy, max |u| and a count of non-finite values; one partial per block
template <int D>
__global__ void __launch_bounds__(kBlock) k_reduce(Geom g, Phys ph, const float* __restrict__ c1,
                                                   const float* __restrict__ phi,
                                                   const uint8_t* __restrict__ mask,
                                                   const float* __restrict__ aux,
                                                   Pop gsrc, int pull,
                                                   double* __restrict__ partials) {
    using L = Lattice<D>;
    const long long N = g.N;
    double acc[RED_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double a2 = ph.a2, link = 1.5 * a2;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        int x, y, z;
        decode(g, n, x, y, z);
        double C1, C2;
        if (ph.stage == 2) {
            C1 = c1[n];
            C2 = phi[n];
        } else {
            C1 = phi[n];
            C2 = 0.0;
        }
        double C3 = 1.0 - C1 - C2;
        // masses: the evolving component summed in FP64 from the stored
        // populations themselves, so that drift measures the stored state
        double cm = gsrc.rest(L::Q, g.NP)[rest_index(g, n)];
        for (int i = 1; i < L::Q; ++i) {
            const long long src = pull ? shifted<D>(g, x, y, z, i, -1) : n;
            cm += (double)gsrc.ld(pop_index(g, L::Q, i, src));
        }
        const double m1 = ph.stage == 2 ? C1 : cm, m2 = ph.stage == 2 ? cm : 0.0;
        acc[RED_C1] += m1;
        acc[RED_C2] += m2;
        acc[RED_C3] += 1.0 - m1 - m2;
        double e;
        if (ph.stage == 2) {
            e = 0.5 * ph.k2 * C2 * C2 * (1.0 - C2) * (1.0 - C2) + 0.5 * ph.k3 * C3 * C3 * (1.0 - C3) * (1.0 - C3);
            for (int i = 1; i < L::Q; ++i) {
                long long m = shifted<D>(g, x, y, z, i, +1);
                double d2 = (double)phi[m] - C2;
                double d3 = (1.0 - (double)c1[m] - (double)phi[m]) - C3;
                e += link * (double)L::w[i] * (ph.k2 * d2 * d2 + ph.k3 * d3 * d3);
            }
        } else {
            double k13 = (double)ph.k1 + (double)ph.k3;
            e = 0.5 * k13 * C1 * C1 * (1.0 - C1) * (1.0 - C1);
            bool inS = mask[n] != 0;
            if ((C1 < 0.5 && inS) || (C1 > 0.5 && !inS)) e += ph.beta * (C1 - 0.5) * (C1 - 0.5);
            if (C1 < 0.0) e += ph.omega * C1 * C1;
            if (C1 > 1.0) e += ph.omega * (1.0 - C1) * (1.0 - C1);
            for (int i = 1; i < L::Q; ++i) {
                double d = (double)phi[shifted<D>(g, x, y, z, i, +1)] - C1;
                e += link * (double)L::w[i] * k13 * d * d;
            }
        }
        acc[RED_FREE] += e;
        double ux = aux[n], uy = aux[N + n], uz = D == 3 ? (double)aux[2 * N + n] : 0.0;
        double uu = ux * ux + uy * uy + uz * uz;
        bool solid = ph.stage == 2 && c1[n] > 0.5f;
        const double rho = ph.contrast ? (double)local_density(ph, phi[n], c1[n]) : 1.0;
        if (!solid) acc[RED_EKIN] += 0.5 * rho * uu;
        double um = sqrt(uu);
        if (!(um <= acc[RED_UMAX])) acc[RED_UMAX] = isfinite(um) ? um : acc[RED_UMAX];
        if (!isfinite(C2) || !isfinite(C1) || !isfinite(uu)) acc[RED_NONFINITE] += 1.0;
    }
    __shared__ double sh[kBlock / 64][RED_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < RED_SLOTS; ++k) {
        double v = k == RED_UMAX ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) sh[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < RED_SLOTS) {
        int k = threadIdx.x;
        double v = sh[0][k];
        for (int j = 1; j < kBlock / 64; ++j) v = k == RED_UMAX ? fmax(v, sh[j][k]) : v + sh[j][k];
        partials[(long long)blockIdx.x * RED_SLOTS + k] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_reduce_final(const double* __restrict__ partials, int nparts,
                                                         double* __restrict__ out) {
    double acc[RED_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < RED_SLOTS; ++k) {
            double v = partials[(long long)b * RED_SLOTS + k];
            acc[k] = k == RED_UMAX ? fmax(acc[k], v) : acc[k] + v;
        }
    }
    __shared__ double sh[kBlock / 64][RED_SLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < RED_SLOTS; ++k) {
        double v = k == RED_UMAX ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) sh[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < RED_SLOTS) {
        int k = threadIdx.x;
        double v = sh[0][k];
        for (int j = 1; j < kBlock / 64; ++j) v = k == RED_UMAX ? fmax(v, sh[j][k]) : v + sh[j][k];
        out[k] = v;
    }
}

}  // namespace

// --- launchers --------------------------------------------------------------

#define DSM_DISPATCH(dim, KERNEL, ...)                                          \
    do {                                                                        \
        if ((dim) == 2)                                                         \
            hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__);                         \
        else                                                                    \
            hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__);                         \
    } while (0)

hipError_t launch_c1_from_mask(const uint8_t* mask, float* c1, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_c1_from_mask, dim3(grid_for(N)), dim3(kBlock), 0, st, mask, c1, N);
    return hipGetLastError();
}

hipError_t launch_remask(const float* c1, uint8_t* mask, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_remask, dim3(grid_for(N)), dim3(kBlock), 0, st, c1, mask, N);
    return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N)), dim3(kBlock), 0, st, src, dst, N);
    return hipGetLastError();
}

hipError_t launch_moment(int dim, const Geom& g, Pop gsrc, float* phi, int pull, hipStream_t st) {
    DSM_DISPATCH(dim, k_moment, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, gsrc, phi, pull);
    return hipGetLastError();
}

hipError_t launch_mu(int dim, const Geom& g, const Phys& ph, const float* phi, const float* c1,
                     const uint8_t* mask, float* mu, hipStream_t st) {
    DSM_DISPATCH(dim, k_mu, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, phi, c1, mask, mu);
    return hipGetLastError();
}

hipError_t launch_collide_split(int dim, const Geom& g, const Phys& ph, Pop fsrc,
                                Pop gsrc, Pop fdst, Pop gdst, const float* c1,
                                const float* phi, const float* mu, int pull, int* flag, hipStream_t st) {
    if (dim == 2)
        hipLaunchKernelGGL((k_collide<2, 0>), dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, fsrc, gsrc,
                           fdst, gdst, c1, phi, mu, pull, flag, (float*)nullptr);
    else
        hipLaunchKernelGGL((k_collide<3, 0>), dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, fsrc, gsrc,
                           fdst, gdst, c1, phi, mu, pull, flag, (float*)nullptr);
    return hipGetLastError();
}

hipError_t launch_observe(int dim, const Geom& g, const Phys& ph, Pop fsrc, const float* c1,
                          const float* phi, const float* mu, int pull, float* aux, hipStream_t st) {
    if (dim == 2)
        hipLaunchKernelGGL((k_collide<2, 1>), dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, fsrc,
                           Pop{nullptr, 0}, Pop{nullptr, 0}, Pop{nullptr, 0}, c1, phi, mu, pull,
                           (int*)nullptr, aux);
    else
        hipLaunchKernelGGL((k_collide<3, 1>), dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, fsrc,
                           Pop{nullptr, 0}, Pop{nullptr, 0}, Pop{nullptr, 0}, c1, phi, mu, pull,
                           (int*)nullptr, aux);
    return hipGetLastError();
}

hipError_t launch_init_populations(int dim, const Geom& g, const float* phi, const float* mu, Pop fdst,
                                   Pop gdst, hipStream_t st) {
    DSM_DISPATCH(dim, k_init_populations, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, phi, mu, fdst, gdst);
    return hipGetLastError();
}

hipError_t launch_pull_state(int dim, const Geom& g, const Phys& ph, Pop fsrc, Pop gsrc,
                             const float* c1, Pop fdst, Pop gdst, hipStream_t st) {
    DSM_DISPATCH(dim, k_pull_state, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, ph, fsrc, gsrc, c1, fdst,
                 gdst);
    return hipGetLastError();
}

hipError_t launch_reduce(int dim, const Geom& g, const Phys& ph, const float* c1, const float* phi,
                         const uint8_t* mask, const float* aux, Pop gsrc, int pull, double* partials,
                         double* red, hipStream_t st) {
    long long want = (g.N + kBlock - 1) / kBlock;
    int blocks = (int)(want < kReduceBlocks ? (want < 1 ? 1 : want) : kReduceBlocks);
    DSM_DISPATCH(dim, k_reduce, dim3(blocks), dim3(kBlock), 0, st, g, ph, c1, phi, mask, aux, gsrc, pull,
                 partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partials, blocks, red);
    return hipGetLastError();
}

}  // namespace dsm
