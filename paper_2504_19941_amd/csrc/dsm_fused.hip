// dsm_fused.hip -- the fused single-pass time step of libdsm.so (gfx950).
//
// One launch performs a whole step of Sec. II.B on every node: stream
// (pull) the Cahn-Hilliard populations g and take their zeroth moment C,
// the chemical potential from the isotropic Laplacians of C and C1, the
// force mu grad C (+ body force), stream the hydrodynamic populations f with
// interpolated bounce-back at the diffuse solid, velocity and pressure, and
// both BGK collisions.  Populations are read once and written once.
//
// Dependencies: the collision at node x needs mu(x) and grad C(x), i.e. C on
// the 1-ring of x, and every C is the sum of Q pulled g values.  Each
// workgroup owns a TX x TY block of columns and marches along the slowest
// axis through a chunk of TZ planes.  Per plane it
//   A  pulls g for the block plus a 1-column halo and writes C (and the
//      frozen C1) of that plane into 4-slot LDS rings; a column's own pulled
//      g stay in registers until its collision one plane later;
//   C  collides the plane behind, whose 1-ring of C and C1 is complete.
// One barrier per plane suffices: A of the next plane writes a ring slot that
// C of this plane does not read.  Only halo columns are recomputed (their
// loads hit in L2, where neighbouring workgroups of the same XCD read the
// same lines); along the march each chunk recomputes 1 + 1 warm-up planes.
//
// Workgroups are renumbered so that each XCD (hardware dispatch is
// round-robin over the 8 XCDs) receives a contiguous range of tiles, which
// keeps the halo columns of neighbouring tiles inside one L2.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

namespace {

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ float s_i(float cu, float uu) { return 3.f * cu + 4.5f * cu * cu - 1.5f * uu; }

// Wrapped x-1, x, x+1 and the row offsets X*(y-1, y, y+1) of a column.
struct Col {
    int xs[3];
    int ys[3];
};

__device__ __forceinline__ Col make_col(int px, int py, int X, int Y) {
    Col c;
    c.xs[0] = pmod(px - 1, X);
    c.xs[1] = pmod(px, X);
    c.xs[2] = pmod(px + 1, X);
    c.ys[0] = pmod(py - 1, Y) * X;
    c.ys[1] = pmod(py, Y) * X;
    c.ys[2] = pmod(py + 1, Y) * X;
    return c;
}

// Plane offsets XY*(z-1, z, z+1), z in [0, Z).
struct Pl {
    int zs[3];
};

__device__ __forceinline__ Pl make_pl(int z, int Z, int XY) {
    Pl p;
    p.zs[0] = (z == 0 ? Z - 1 : z - 1) * XY;
    p.zs[1] = z * XY;
    p.zs[2] = (z == Z - 1 ? 0 : z + 1) * XY;
    return p;
}

// node index of position + s * c_i
template <int D>
__device__ __forceinline__ int nidx(const Col& c, const Pl& p, int i, int s) {
    using L = Lattice<D>;
    return c.xs[1 + s * L::cx[i]] + c.ys[1 + s * L::cy[i]] + p.zs[1 + s * L::cz[i]];
}

// Wall fraction of the link along direction k (FP64, boundary links only):
// distance to the C1 = 1/2 level from the tanh profile, along the link.
template <int D>
__device__ double link_fraction(const double gc[3], double gnorm, double xi, int k) {
    using L = Lattice<D>;
    if (gnorm < 1e-12) return 0.5;
    const double len = (L::cx[k] * L::cx[k] + L::cy[k] * L::cy[k] + L::cz[k] * L::cz[k]) == 1
                           ? 1.0
                           : 1.4142135623730951;
    const double cosnc = (gc[0] * L::cx[k] + gc[1] * L::cy[k] + gc[2] * L::cz[k]) / (gnorm * len);
    if (cosnc <= 1e-6) return 0.5;
    const double q = xi / cosnc / len;
    return q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
}

template <int D, int TX, int TY>
struct Tile {
    static constexpr int NT = TX * TY;
    static constexpr int HY = D == 3 ? 1 : 0;  // halo rows along y (none in 2D)
    static constexpr int CRX = TX + 2;
    static constexpr int CRY = TY + 2 * HY;
    static constexpr int CR = CRX * CRY;
    static constexpr int NHALO = CR - NT;
    static constexpr int NA = 1 + (NHALO + NT - 1) / NT;  // C positions per thread

    // C-region coordinates of the k-th position (k < NT: interior column k)
    static __device__ __forceinline__ void cpos(int k, int& rx, int& ry) {
        if (k < NT) {
            rx = (k % TX) + 1;
            ry = (k / TX) + HY;
            return;
        }
        int h = k - NT;
        if (h < HY * CRX) {
            rx = h % CRX;
            ry = h / CRX;
            return;
        }
        h -= HY * CRX;
        if (h < HY * CRX) {
            rx = h % CRX;
            ry = HY + TY + h / CRX;
            return;
        }
        h -= HY * CRX;
        ry = HY + h / 2;
        rx = (h % 2) ? TX + 1 : 0;
    }
};

template <int D, int TX, int TY, int STAGE, bool PULL>
__global__ void __launch_bounds__(TX* TY)
    k_step_fused(Geom g, Phys ph, const float* __restrict__ fsrc, const float* __restrict__ gsrc,
                 float* __restrict__ fdst, float* __restrict__ gdst, const float* __restrict__ c1g,
                 const uint8_t* __restrict__ mask, int* __restrict__ flag, int TZ, int ntx, int nty) {
    using T = Tile<D, TX, TY>;
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    constexpr int NT = T::NT, CRX = T::CRX, CR = T::CR, HY = T::HY;
    __shared__ float s_c[4][CR];                       // C of planes l-3..l (ring)
    __shared__ float s_c1[STAGE == 2 ? 4 : 1][CR];     // frozen C1, same ring

    const int X = g.X, Y = g.Y, Z = g.Z, XY = X * Y;
    const long long N = g.N;

    // XCD-aware tile order: XCD k (= blockIdx % 8) gets a contiguous range
    const int nb = gridDim.x, b = blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int tile = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int tile_x = tile % ntx, rest = tile / ntx;
    const int tile_y = rest % nty, tile_z = rest / nty;
    const int x0 = tile_x * TX, y0 = tile_y * TY, z0 = tile_z * TZ;
    const int zlen = min(TZ, Z - z0);

    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    const bool active = (x0 + tx < X) && (y0 + ty < Y);

    // C positions of this thread: its own column, then halo columns
    Col ca[T::NA];
    int ra[T::NA];
    bool va[T::NA];
#pragma unroll
    for (int k = 0; k < T::NA; ++k) {
        const int pk = k == 0 ? t : NT + (k - 1) * NT + t;
        va[k] = pk < CR;
        int rx = 0, ry = 0;
        if (va[k]) T::cpos(pk, rx, ry);
        ra[k] = rx + CRX * ry;
        ca[k] = make_col(x0 - 1 + rx, y0 - HY + ry, X, Y);
    }
    const int rint = ra[0];

    const float fpref3 = 3.f * ph.fpref;
    const float k13 = ph.k1 + ph.k3;
    float gA[Q], gB[Q];

    // Iteration j: lead plane l = z0 - 1 + j goes into ring slot j & 3; the
    // plane c = l - 1 (slot (j+3)&3, neighbours (j+2)&3 and j&3) collides.
    auto iteration = [&](int j, float (&gload)[Q], float (&gcoll)[Q]) {
        const int l = z0 - 1 + j;
        // ---- A -----------------------------------------------------------
        {
            const Pl pl = make_pl(pmod(l, Z), Z, XY);
            const int sl = j & 3;
#pragma unroll
            for (int k = 0; k < T::NA; ++k) {
                if (!va[k]) continue;
                float acc = 0.f;
                if (k == 0) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int src = PULL ? nidx<D>(ca[0], pl, i, -1) : (ca[0].xs[1] + ca[0].ys[1] + pl.zs[1]);
                        gload[i] = gsrc[(size_t)i * N + src];
                    }
#pragma unroll
                    for (int i = 0; i < Q; ++i) acc += gload[i];
                } else {
                    float tmp[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const int src = PULL ? nidx<D>(ca[k], pl, i, -1) : (ca[k].xs[1] + ca[k].ys[1] + pl.zs[1]);
                        tmp[i] = gsrc[(size_t)i * N + src];
                    }
#pragma unroll
                    for (int i = 0; i < Q; ++i) acc += tmp[i];
                }
                s_c[sl][ra[k]] = acc;
                if (STAGE == 2) s_c1[sl][ra[k]] = c1g[ca[k].xs[1] + ca[k].ys[1] + pl.zs[1]];
            }
        }
        __syncthreads();
        // ---- C: plane c = l - 1 ------------------------------------------
        if (j >= 2 && active) {
            const int c = l - 1;  // inside [z0, z0 + zlen)
            const Pl pc = make_pl(c, Z, XY);
            const int sm_ = (j + 2) & 3, s0 = (j + 3) & 3, sp = j & 3;  // planes c-1, c, c+1
            const int self = ca[0].xs[1] + ca[0].ys[1] + pc.zs[1];
            const float C = s_c[s0][rint];
            // Laplacians and gradient of C; Laplacian of C1
            float lc = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);  // plane of x + c_i
                const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);  // plane of x - c_i
                const int o = L::cx[i] + CRX * L::cy[i];
                const float a = s_c[spl][rint + o], bm = s_c[smi][rint - o];
                lc += L::w[i] * ((a - C) + (bm - C));
                const float d = a - bm;
                gx += L::w[i] * L::cx[i] * d;
                gy += L::w[i] * L::cy[i] * d;
                gz += L::w[i] * L::cz[i] * d;
            }
            lc *= 6.f;
            float mu, C1 = 0.f;
            if (STAGE == 2) {
                C1 = s_c1[s0][rint];
                float l1 = 0.f;
#pragma unroll
                for (int i = 1; i < Q; i += 2) {
                    const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);
                    const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);
                    const int o = L::cx[i] + CRX * L::cy[i];
                    l1 += L::w[i] * ((s_c1[spl][rint + o] - C1) + (s_c1[smi][rint - o] - C1));
                }
                l1 *= 6.f;
                const float S = C1 + C;
                mu = ph.k2 * C * (1.f - C) * (1.f - 2.f * C) + ph.k3 * S * (1.f - S) * (1.f - 2.f * S) -
                     ph.a2 * ph.k2 * lc - ph.a2 * ph.k3 * (l1 + lc);
            } else {
                mu = k13 * C * (1.f - C) * (1.f - 2.f * C);
                const bool inS = mask[self] != 0;
                if ((C < 0.5f && inS) || (C > 0.5f && !inS)) mu += 2.f * ph.beta * (C - 0.5f);
                mu -= ph.a2 * k13 * lc;
                if (C < 0.f) mu += 2.f * ph.omega * C;
                if (C > 1.f) mu -= 2.f * ph.omega * (1.f - C);
            }
            const bool solid = STAGE == 2 && C1 > 0.5f;
            float ux = 0.f, uy = 0.f, uz = 0.f, pt = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
            float f[Q];
            if (!solid) {
                Fx = mu * 3.f * gx;
                Fy = mu * 3.f * gy;
                Fz = mu * 3.f * gz;
                if (STAGE == 2) {
                    Fx += C * ph.grav[0];
                    Fy += C * ph.grav[1];
                    Fz += C * ph.grav[2];
                }
                // pull f; links whose upstream node is solid are rebuilt below
                unsigned cut = 0;
                if (STAGE == 2 && PULL) {
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const int su = L::cz[i] > 0 ? sm_ : (L::cz[i] < 0 ? sp : s0);
                        if (s_c1[su][rint - L::cx[i] - CRX * L::cy[i]] > 0.5f) cut |= 1u << i;
                    }
                }
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int src = PULL ? nidx<D>(ca[0], pc, i, -1) : self;
                    f[i] = ((cut >> i) & 1u) ? 0.f : fsrc[(size_t)i * N + src];
                }
                if (cut) {
                    double gc[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const int sl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);
                        const double v = (double)s_c1[sl][rint + L::cx[i] + CRX * L::cy[i]];
                        const double wi = (L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i]) == 1
                                              ? (D == 2 ? 1.0 / 9.0 : 1.0 / 18.0)
                                              : 1.0 / 36.0;
                        gc[0] += wi * L::cx[i] * v;
                        gc[1] += wi * L::cy[i] * v;
                        gc[2] += wi * L::cz[i] * v;
                    }
                    gc[0] *= 3.0;
                    gc[1] *= 3.0;
                    gc[2] *= 3.0;
                    const double gn = sqrt(gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2]);
                    double tt = 1.0 - 2.0 * (double)C1;
                    tt = tt < 0.0 ? 0.0 : (tt > 1.0 - 1e-12 ? 1.0 - 1e-12 : tt);
                    const double xi = 2.0 * (double)ph.alpha * atanh(tt);
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        if (!((cut >> i) & 1u)) continue;
                        const int k = opp(i);
                        double q = link_fraction<D>(gc, gn, xi, k);
                        const int sd = L::cz[i] > 0 ? sp : (L::cz[i] < 0 ? sm_ : s0);
                        const bool down_solid = s_c1[sd][rint + L::cx[i] + CRX * L::cy[i]] > 0.5f;
                        const double fk = (double)fsrc[(size_t)k * N + self];
                        double v;
                        if (q < 0.5 && !down_solid) {
                            const int dn = nidx<D>(ca[0], pc, i, +1);
                            v = 2.0 * q * fk + (1.0 - 2.0 * q) * (double)fsrc[(size_t)k * N + dn];
                        } else {
                            if (q < 0.5) q = 0.5;
                            v = fk / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * (double)fsrc[(size_t)i * N + self];
                        }
                        f[i] = (float)v;
                    }
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
            }
            const float uu = ux * ux + uy * uy + uz * uz;
            if (solid) {
#pragma unroll
                for (int i = 0; i < Q; ++i) fdst[(size_t)i * N + self] = 0.f;
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const float cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
                    const float cF = L::cx[i] * Fx + L::cy[i] * Fy + L::cz[i] * Fz;
                    const float feq = L::w[i] * (pt + s_i(cu, uu));
                    fdst[(size_t)i * N + self] = f[i] - (f[i] - feq) * ph.inv_tau + fpref3 * L::w[i] * cF;
                }
            }
            float restg = C;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const float cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
                const float geq = L::w[i] * mu + L::w[i] * C * s_i(cu, uu);
                restg -= geq;
                gdst[(size_t)i * N + self] = gcoll[i] - (gcoll[i] - geq) * ph.inv_taug;
            }
            gdst[self] = gcoll[0] - (gcoll[0] - restg) * ph.inv_taug;
            if (!isfinite(C) || !isfinite(uu)) flag[0] = 1;
        }
    };

    const int J = zlen + 2;
    for (int j = 0; j < J; j += 2) {
        iteration(j, gA, gB);
        if (j + 1 < J) iteration(j + 1, gB, gA);
    }
}

template <int D, int TX, int TY, int STAGE, bool PULL>
hipError_t launch_cfg(const Geom& g, const Phys& ph, const float* fsrc, const float* gsrc, float* fdst,
                      float* gdst, const float* c1, const uint8_t* mask, int* flag, int TZ, hipStream_t st) {
    const int ntx = (g.X + TX - 1) / TX;
    const int nty = (g.Y + TY - 1) / TY;
    const int ntz = (g.Z + TZ - 1) / TZ;
    const long long nblocks = (long long)ntx * nty * ntz;
    hipLaunchKernelGGL((k_step_fused<D, TX, TY, STAGE, PULL>), dim3((unsigned)nblocks), dim3(TX * TY), 0, st, g,
                       ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, ntx, nty);
    return hipGetLastError();
}

template <int D, int TX, int TY>
hipError_t launch_tile(const Geom& g, const Phys& ph, const float* fsrc, const float* gsrc, float* fdst,
                       float* gdst, const float* c1, const uint8_t* mask, int pull, int* flag, int TZ,
                       hipStream_t st) {
    if (ph.stage == 2) {
        if (pull) return launch_cfg<D, TX, TY, 2, true>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, st);
        return launch_cfg<D, TX, TY, 2, false>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, st);
    }
    if (pull) return launch_cfg<D, TX, TY, 1, true>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, st);
    return launch_cfg<D, TX, TY, 1, false>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, st);
}

}  // namespace

int fused_tile_variants(int dim) { return dim == 2 ? 3 : 4; }

hipError_t launch_step_fused(int dim, const Geom& g, const Phys& ph, const float* fsrc, const float* gsrc,
                             float* fdst, float* gdst, const float* c1, const uint8_t* mask, int pull, int* flag,
                             int variant, int TZ, hipStream_t st) {
    if (TZ < 1) TZ = 1;
    if (dim == 2) {
        switch (variant) {
            case 1: return launch_tile<2, 256, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
            case 2: return launch_tile<2, 64, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
            default: return launch_tile<2, 128, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        }
    }
    switch (variant) {
        case 1: return launch_tile<3, 64, 4>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        case 2: return launch_tile<3, 64, 8>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        case 3: return launch_tile<3, 32, 16>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        default: return launch_tile<3, 32, 8>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
    }
}

}  // namespace dsm
