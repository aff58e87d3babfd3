// dsm_fused.hip -- the fused single-pass time step of libdsm.so (gfx950).
//
// One launch performs a whole step of Sec. II.B on every node: stream (pull)
// the Cahn-Hilliard populations g and take their zeroth moment C, the
// chemical potential from the isotropic Laplacians of C and C1, the force
// mu grad C (+ body force), stream the hydrodynamic populations f with
// interpolated bounce-back at the diffuse solid, velocity and pressure, and
// both BGK collisions.  Every population is read once and written once.
//
// Work decomposition.  The collision at node x needs mu(x) and grad C(x), so C
// on the 1-ring of x; every C is the sum of Q pulled g values.  A workgroup
// owns a tile of TY lattice rows x 64*TXW columns (one 64-lane wave per row
// segment, so every wave-wide load of one direction is a contiguous run of
// one row) and marches along the slowest axis through TZ planes.  Iteration j
// works on two planes:
//   phase 1: issue the f loads of the collision plane c = l - 1; pull g of the
//            lead plane l for the own columns (kept in registers until their
//            collision one iteration later) and for the 1-column halo; write
//            C (and the frozen C1) of plane l into 4-slot LDS rings;
//   barrier;
//   phase 2: collide plane c, whose 1-ring of C and C1 is complete, and store.
// The ring slots written by phase 1 of an iteration are never read by phase 2
// of the iteration before or of the same iteration, so one barrier per plane
// suffices.  Halo columns are the only recomputation (their loads hit in L2,
// where the neighbouring tile of the same XCD reads the same lines), plus one
// warm-up plane on each side of the march; a tile spanning its whole lattice
// row has no side halo (its end columns' neighbours are its own columns).  Two forms of the tile share this
// scheme: fused_tile (3D with FP16 elements, held g in LDS) issues each
// plane's loads in its own phase 1; fused_tile_pipe (every other lattice and
// storage) issues them one plane ahead, before the previous plane's stores
// (see there).
//
// Addressing.  Populations are stored row-interleaved: the Q values of the X
// nodes of one row are contiguous, direction-major, each direction row padded
// to a whole number of 128-byte lines (dsm_lattice.h).  A wave's row is
// uniform, so the 9 source rows of a pull are scalar base addresses and the
// lanes only add their (wrapped) x - 1, x, x + 1; the own-column stores fill
// whole lines.
//
// Mass.  BGK conserves sum_i g_i at each node and streaming only moves
// values, so the liquid mass is exact up to rounding.  The rest population
// g_0, which carries nearly all of C, is stored in FP64 (dsm_lattice.h); C is
// summed in FP64 and the post-collision rest population is written as
// C - sum_{i>0} g*_i, equal to g_0 - (g_0 - g_eq,0)/tau_g in real arithmetic.
// The stored populations of a node then keep its C to FP64 rounding: with
// g_0 in FP32, rounding at the scale of C (~1e-7 relative per node and step)
// is systematic wherever the moving populations are below half an ulp of C,
// and the liquid mass drifts by ~1e-3 over 10^5 steps.
//
// Interpolated bounce-back.  A fluid node x pulls f_i from x - c_i; when that
// node is solid, the slot holds no population of its own, and the link kernel
// (dsm_links.hip) has already written the bounce-back value for x into it
// before this step.  The pull is therefore the same for every link.
#include <math.h>

#include "dsm_internal.h"

namespace dsm {

namespace {

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Products with lattice vectors, whose components are -1, 0 or 1: the kept
// terms are +-v exactly, summed in x, y, z order, and the zero terms are left
// out.  The full product sum rounds the same way, since the terms it adds
// besides these are exact zeros (the sign of an exact-zero result aside).
template <typename L>
__device__ __forceinline__ float cdot(int i, float vx, float vy, float vz) {
    const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
    const float v[3] = {vx, vy, vz};
    float s = 0.f;
    bool any = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (c[k] == 0) continue;
        const float t = c[k] > 0 ? v[k] : -v[k];
        s = any ? s + t : t;
        any = true;
    }
    return s;
}
// a += c_i v, componentwise
template <typename L>
__device__ __forceinline__ void cacc(int i, float v, float& ax, float& ay, float& az) {
    if (L::cx[i]) ax = L::cx[i] > 0 ? ax + v : ax - v;
    if (L::cy[i]) ay = L::cy[i] > 0 ? ay + v : ay - v;
    if (L::cz[i]) az = L::cz[i] > 0 ? az + v : az - v;
}
// a += (w_i c_i) v, componentwise
template <typename L>
__device__ __forceinline__ void wacc(int i, float v, float& ax, float& ay, float& az) {
    if (L::cx[i]) ax += L::w[i] * L::cx[i] * v;
    if (L::cy[i]) ay += L::w[i] * L::cy[i] * v;
    if (L::cz[i]) az += L::w[i] * L::cz[i] * v;
}
// s_i(u) = 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u for the directions in order.
// Direction i + 1 (odd i) is the opposite of i, so its two c.u terms are
// those of i with the first negated: (4.5 (c.u)^2 - 3 c.u) - 1.5 u.u, rounded
// as computing it afresh would round it.
template <typename L>
struct SeqS {
    float t1 = 0.f, t3 = 0.f;  // 3 c.u and 4.5 (c.u)^2 of the last odd direction
    __device__ __forceinline__ float next(int i, float ux, float uy, float uz, float uu15) {
        if (i == 0 || (i & 1)) {
            const float cu = cdot<L>(i, ux, uy, uz);
            t1 = 3.f * cu;
            t3 = 4.5f * cu * cu;
            return t1 + t3 - uu15;
        }
        return t3 - t1 - uu15;
    }
};

template <int D, int TXW, int TY>
struct Tile {
    static constexpr int TX = 64 * TXW;
    static constexpr int NT = TX * TY;
    static constexpr int NW = TXW * TY;        // waves
    static constexpr int HY = D == 3 ? 1 : 0;  // halo rows along y (none in 2D)
    static constexpr int CRX = TX + 2;
    static constexpr int CRY = TY + 2 * HY;
    static constexpr int CR = CRX * CRY;
    // Halo of the C region: waves 0 .. NROWH-1 take the rows above and below
    // the tile (top: waves 0 .. TXW-1, bottom: TXW .. 2 TXW-1), over the same
    // columns as their own row segment; wave SIDE takes the NSIDE remaining
    // columns (the four corners, then the left and right end of each row).
    static constexpr int NROWH = 2 * HY * TXW;
    static constexpr int SIDE = NROWH;
    static constexpr int NSIDE = 4 * HY + 2 * TY;
    static_assert(SIDE < NW && NSIDE <= 64, "tile too small for its halo");

    // side lane s: the four corners first (3D), then the two end columns of
    // each own row; odd lanes take the right end (4 corners keep the parity)
    static __device__ __forceinline__ void side_pos(int s, int& rx, int& ry) {
        const bool corner = HY && s < 4;
        rx = (s & 1) ? CRX - 1 : 0;
        ry = corner ? ((s & 2) ? CRY - 1 : 0) : HY + ((s - 4 * HY) >> 1);
    }
};


// Position of a side-halo column (see Tile): region index, wrapped column
// and row, and their neighbours.
struct SidePos {
    int reg, xw, yw, xm, xp, ym, yp;
};

// Buffer resources.  Every plane of populations gets a descriptor (base =
// start of the plane, range = one plane), so the hot loads and stores address
// with a scalar offset (row and direction, uniform per wave) plus a 32-bit
// lane offset (x), and an access outside the plane returns 0 / is dropped
// instead of faulting.  Word 3 is the gfx9 raw-buffer format.
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kNonTemporal = 2;  // cache-policy bit of buffer stores: nt

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, long long plane_bytes, int z) {
    // the plane start is wave-uniform; saying so keeps the descriptor in SGPRs
    const unsigned long long a = (unsigned long long)base + (unsigned long long)(plane_bytes * z);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    void* p = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)plane_bytes, kRsrcWord3);
}

// Population element types: loads return the value (raw: the stored bits,
// value: their meaning), stores write it (non-temporal) and return the value
// as stored, after rounding.
//
// Occupancy.  The 3D tile holds the pulled g of its lead plane for one
// iteration, until that plane's collision; in registers that brings it to
// about 150 VGPRs (about 205 when pipelined), 2-3 waves per SIMD, one 8-wave tile
// per CU.  With FP16 elements the 3D tile holds them instead as their raw
// bits in a two-slot LDS buffer of per-thread cells (exact, 2 bytes each), and
// the 3D FP16 kernels request 4 waves per SIMD, so two tiles share a CU: the FP16
// step moves half the bytes per memory instruction and is latency-bound at
// one tile per CU (measured at 128^3: 7 % faster than the pipelined tile at
// one tile per CU).
// The FP32 step is bound by the memory system, gains nothing from a second
// tile, and keeps its registers (min_waves 1: no request).  The 2D tiles are
// small enough (about 120 VGPRs) to be pipelined in either storage.
struct F32 {
    using Raw = unsigned;
    static constexpr unsigned bytes = 4;
    static constexpr int min_waves = 1;
    static constexpr bool lds_hold = false;
    static __device__ __forceinline__ Raw load_raw(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
    }
    static __device__ __forceinline__ float value(Raw b) { return __uint_as_float(b); }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return value(load_raw(r, voff, soff));
    }
    static __device__ __forceinline__ float store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, kNonTemporal);
        return v;
    }
};
struct F16 {  // FP16 holding value * kHalfScale
    using Raw = unsigned short;
    static constexpr unsigned bytes = 2;
    static constexpr int min_waves = 4;
    static constexpr bool lds_hold = true;
    static __device__ __forceinline__ Raw load_raw(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
    }
    // h / kHalfScale as one mixed-precision FMA (convert, scale, add +0).  The
    // scale is a power of two, so the product is exact; the +0 turns a -0
    // into +0 and changes nothing else.  Stores return this same value, so
    // what a step counts as stored is what the next step reads.
    static __device__ __forceinline__ float value(Raw h) {
        return __builtin_fmaf(__half2float(__ushort_as_half(h)), 1.f / kHalfScale, 0.f);
    }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return value(load_raw(r, voff, soff));
    }
    static __device__ __forceinline__ float store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
        const __half h = __float2half(v * kHalfScale);
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(h), r, (int)voff, (int)soff, kNonTemporal);
        return value(__half_as_ushort(h));
    }
};

// Lane offset past every plane: a buffer load there returns 0 without memory
// traffic.
constexpr unsigned kOOBLoad = 0x80000000u;  // (the pipelined tile names it kOOB)

// One tile of the march: columns [x0, x0 + 64 TXW) x rows [y0, y0 + TY),
// planes [z0, z0 + TZ) of one lattice.
template <int D, int TXW, int TY, int STAGE, bool PULL, bool RHO, typename E>
__device__ __forceinline__ void fused_tile(const Geom& g, const Phys& ph, const void* __restrict__ fsrc,
                                           const void* __restrict__ gsrc, void* __restrict__ fdst,
                                           void* __restrict__ gdst, const float* __restrict__ c1g,
                                           const uint8_t* __restrict__ mask, int* __restrict__ flag, int x0,
                                           int y0, int z0, int TZ) {
    using T = Tile<D, TXW, TY>;
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    constexpr int CRX = T::CRX, CR = T::CR, HY = T::HY;
    __shared__ float s_c[4][CR];                                    // C of planes l-3..l (ring)
    __shared__ float s_c1[STAGE == 2 ? 4 : 1][STAGE == 2 ? CR : 1];  // frozen C1, same ring
    // held lead-plane g of the own column (FP16: raw bits, slot j & 1)
    constexpr int HOLD = E::lds_hold ? T::NT : 1;
    __shared__ typename E::Raw s_gh[E::lds_hold ? 2 : 1][E::lds_hold ? Q - 1 : 1][HOLD];

    const int X = g.X, Y = g.Y, Z = g.Z, XP = g.XP;
    const int QX = Q * XP;                              // elements per row of populations
    const long long PL = (long long)QX * Y * E::bytes;  // bytes per plane of populations
    constexpr unsigned ES = E::bytes;
    const int zlen = min(TZ, Z - z0);

    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index (uniform)
    const int lane = t & 63;
    const int xseg = wv % TXW, yrow = wv / TXW;
    const int x = x0 + xseg * 64 + lane;
    const int y = y0 + yrow;  // uniform
    const bool active = (x < X) && (y < Y);
    // Lanes past the lattice's last column or row pull no g, except the first
    // one (column X, row Y): it holds C of the wrapped column (row) that the
    // last real one's stencil reads.  The others' ring cells are read by no
    // lattice node; their g pulls go past the plane and return 0 without
    // memory traffic (their rest value and C1 are still read: 12 of 84 bytes,
    // through plain loads that stay unconditional).
    const bool pulls = x <= X && y <= Y;
    const int rint = (1 + xseg * 64 + lane) + CRX * (HY + yrow);  // own region index
    // Region indices of the columns x - 1, x, x + 1 in the own row.  A tile
    // that spans its whole lattice row (x0 == 0, X <= TX) wraps them onto its
    // own columns and needs no side halo (whose loads are uncoalesced: each
    // of its lanes reads another row); other tiles use the halo columns at
    // either end of the region.
    const bool full_row = x0 == 0 && X <= T::TX;  // uniform
    const int xl = xseg * 64 + lane;            // column within the tile
    const int rrow = CRX * (HY + yrow);
    const int rcol[3] = {full_row ? 1 + pmod(xl - 1, X) : xl, xl + 1, full_row ? 1 + pmod(xl + 1, X) : xl + 2};

    // Own column, wrapped (the first lane past the edge of a ragged tile
    // computes C of the wrapped column, which the last real column reads).
    const int xv[3] = {pmod(x - 1, X), pmod(x, X), pmod(x + 1, X)};   // x-1, x, x+1
    // as byte offsets; past the plane for a lane that pulls nothing (every
    // other access of such a lane is masked already: it stores nothing and
    // pulls no f)
    const unsigned xb[3] = {pulls ? ES * xv[0] : kOOBLoad, pulls ? ES * xv[1] : kOOBLoad,
                            pulls ? ES * xv[2] : kOOBLoad};
    const int yw = pmod(y, Y);
    const int yv[3] = {yw == 0 ? Y - 1 : yw - 1, yw, yw + 1 == Y ? 0 : yw + 1};

    // Halo columns of this wave (see Tile)
    const bool row_halo = wv < T::NROWH;  // uniform
    const int hbot = HY ? (wv / TXW) : 0;  // 0: row above the tile, 1: row below
    const int hyw = pmod(hbot ? y0 + TY : y0 - 1, Y);
    const int hyv[3] = {hyw == 0 ? Y - 1 : hyw - 1, hyw, hyw + 1 == Y ? 0 : hyw + 1};
    const int hreg = (1 + xseg * 64 + lane) + CRX * (hbot ? T::CRY - 1 : 0);
    const bool side = !full_row && wv == T::SIDE && lane < T::NSIDE;
    // Side column of this lane: computed where used (only the side wave of a
    // tile narrower than its row runs that code), so that its indices hold no
    // registers through the march (measured: 3.6 % faster at 128^3, where no
    // tile has a side halo, and no slower where they do).
    auto side_at = [&]() {
        SidePos p;
        int srx = 0, sry = 0, sl = lane;
        asm volatile("" : "+v"(sl));  // computed here: not hoisted out of the march
        T::side_pos(sl, srx, sry);
        p.reg = srx + CRX * sry;
        p.xw = pmod(x0 - 1 + srx, X);
        p.yw = pmod(y0 - HY + sry, Y);
        p.xm = p.xw == 0 ? X - 1 : p.xw - 1;
        p.xp = p.xw + 1 == X ? 0 : p.xw + 1;
        p.ym = p.yw == 0 ? Y - 1 : p.yw - 1;
        p.yp = p.yw + 1 == Y ? 0 : p.yw + 1;
        return p;
    };

    const float fpref3 = 3.f * ph.fpref;
    const float k13 = ph.k1 + ph.k3;
    const double* __restrict__ g0src = rest_plane(gsrc, Q, g.NP, ES);
    double* __restrict__ g0dst = rest_plane(gdst, Q, g.NP, ES);
    float gA[Q], gB[Q];

    auto iteration = [&](int j, float (&gload)[Q], float (&gcoll)[Q], double& cload, double& ccoll) {
        const int l = z0 - 1 + j;  // lead plane
        const int c = l - 1;       // collision plane (valid when j >= 2)
        const int lz = pmod(l, Z);
        const int zl[3] = {lz == 0 ? Z - 1 : lz - 1, lz, lz + 1 == Z ? 0 : lz + 1};
        const int sl = j & 3;
        const bool collide = j >= 2 && active;
        const int cz = j >= 2 ? c : 0;  // c is inside [0, Z) from j = 2 on (uniform)
        const int zc[3] = {cz == 0 ? Z - 1 : cz - 1, cz, cz + 1 == Z ? 0 : cz + 1};

        // ---- phase 1 --------------------------------------------------------
        const __amdgpu_buffer_rsrc_t gl[3] = {plane_rsrc(gsrc, PL, zl[0]), plane_rsrc(gsrc, PL, zl[1]),
                                              plane_rsrc(gsrc, PL, zl[2])};
        // lead plane: the pulled moving g and the (FP64) rest population of the
        // own column and of this wave's halo column, if it has one, all issued
        // before any is consumed; C = g_0 + sum_{i>0} g_i in FP64 (the halo
        // columns in the same summation order as the own column)
        const long long node = xv[1] + X * ((long long)yv[1] + (long long)Y * lz);
        const double r0 = g0src[xv[1] + XP * ((long long)yv[1] + (long long)Y * lz)];
        const float c1v = STAGE == 2 ? c1g[node] : 0.f;
        typename E::Raw raw[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
            raw[i] = E::load_raw(gl[sz], xb[sx], ES * (unsigned)(yv[sy] * QX + i * XP));
        }
        typename E::Raw h[Q];
        double hr0 = 0.0;
        float hc1 = 0.f;
        int hdst = 0;
        if (row_halo) {
            const long long hnode = xv[1] + X * ((long long)hyw + (long long)Y * lz);
            hr0 = g0src[xv[1] + XP * ((long long)hyw + (long long)Y * lz)];
            hc1 = STAGE == 2 ? c1g[hnode] : 0.f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
                h[i] = E::load_raw(gl[sz], xb[sx], ES * (unsigned)(hyv[sy] * QX + i * XP));
            }
            hdst = hreg;
        } else if (side) {
            const SidePos sp_ = side_at();
            const int sxw = sp_.xw, syw = sp_.yw;
            const int sxv[3] = {sp_.xm, sxw, sp_.xp}, syv[3] = {sp_.ym, syw, sp_.yp};
            const long long hnode = sxw + X * ((long long)syw + (long long)Y * lz);
            hr0 = g0src[sxw + XP * ((long long)syw + (long long)Y * lz)];
            hc1 = STAGE == 2 ? c1g[hnode] : 0.f;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
                h[i] = E::load_raw(gl[sz], ES * (unsigned)(syv[sy] * QX + i * XP + sxv[sx]), 0u);
            }
            hdst = sp_.reg;
        }
        __builtin_amdgcn_sched_barrier(0);  // every pull in flight before the first is used
        {
            double acc = 0.0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                gload[i] = E::value(raw[i]);
                acc += (double)gload[i];
            }
            if (E::lds_hold) {
#pragma unroll
                for (int i = 1; i < Q; ++i) s_gh[j & 1][i - 1][t] = raw[i];
            }
            cload = r0 + acc;
            s_c[sl][rint] = (float)cload;
            if (STAGE == 2) s_c1[sl][rint] = c1v;
        }
        if (row_halo || side) {
            double acc = 0.0;
#pragma unroll
            for (int i = 1; i < Q; ++i) acc += (double)E::value(h[i]);
            s_c[sl][hdst] = (float)(hr0 + acc);
            if (STAGE == 2) s_c1[sl][hdst] = hc1;
        }
        // collision plane: f, in flight across the barrier (raw until after it)
        bool solid = false;
        if (STAGE == 2 && collide) solid = s_c1[(j + 3) & 3][rint] > 0.5f;
        typename E::Raw fr[Q];
        if (collide && !solid) {
            const __amdgpu_buffer_rsrc_t fc[3] = {plane_rsrc(fsrc, PL, zc[0]), plane_rsrc(fsrc, PL, zc[1]),
                                                  plane_rsrc(fsrc, PL, zc[2])};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
                fr[i] = E::load_raw(fc[sz], xb[sx], ES * (unsigned)(yv[sy] * QX + i * XP));
            }
        }
        __syncthreads();

        // ---- phase 2: collide plane c --------------------------------------
        if (!collide) return;
        const int sm_ = (j + 2) & 3, s0 = (j + 3) & 3, sp = j & 3;  // planes c-1, c, c+1
        const float C = s_c[s0][rint];
        // Laplacian and gradient of C (pairs of opposite directions)
        float lc = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);  // plane of x + c_i
            const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);  // plane of x - c_i
            const int ip = rcol[1 + L::cx[i]] + rrow + CRX * L::cy[i];  // x + c_i
            const int im = rcol[1 - L::cx[i]] + rrow - CRX * L::cy[i];  // x - c_i
            const float a = s_c[spl][ip], bm = s_c[smi][im];
            lc += L::w[i] * ((a - C) + (bm - C));
            const float d = a - bm;
            wacc<L>(i, d, gx, gy, gz);
        }
        lc *= 6.f;
        float mu, C1 = 0.f;
        float rho = 1.f, grx = 0.f, gry = 0.f, grz = 0.f;  // local density and its gradient (contrast)
        if (STAGE == 2) {
            C1 = s_c1[s0][rint];
            float l1 = 0.f;
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);
                const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);
                const int ip = rcol[1 + L::cx[i]] + rrow + CRX * L::cy[i];
                const int im = rcol[1 - L::cx[i]] + rrow - CRX * L::cy[i];
                const float a1 = s_c1[spl][ip], b1 = s_c1[smi][im];
                l1 += L::w[i] * ((a1 - C1) + (b1 - C1));
                if (RHO) {
                    const float d = local_density(ph, s_c[spl][ip], a1) - local_density(ph, s_c[smi][im], b1);
                    wacc<L>(i, d, grx, gry, grz);
                }
            }
            l1 *= 6.f;
            if (RHO) {
                rho = local_density(ph, C, C1);
                grx *= 3.f;
                gry *= 3.f;
                grz *= 3.f;
            }
            const float S = C1 + C;
            mu = ph.k2 * C * (1.f - C) * (1.f - 2.f * C) + ph.k3 * S * (1.f - S) * (1.f - 2.f * S) -
                 ph.a2 * ph.k2 * lc - ph.a2 * ph.k3 * (l1 + lc);
        } else {
            mu = k13 * C * (1.f - C) * (1.f - 2.f * C);
            const bool inS = mask[xv[1] + X * ((long long)yv[1] + (long long)Y * c)] != 0;
            if ((C < 0.5f && inS) || (C > 0.5f && !inS)) mu += 2.f * ph.beta * (C - 0.5f);
            mu -= ph.a2 * k13 * lc;
            if (C < 0.f) mu += 2.f * ph.omega * C;
            if (C > 1.f) mu -= 2.f * ph.omega * (1.f - C);
        }
        float ux = 0.f, uy = 0.f, uz = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f, pt = 0.f;
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
            float mx = 0.f, my = 0.f, mz = 0.f;
            // The f pulls are consumed from here on.  The empty asm marks their
            // raw values as changed at this point, so that their conversion (and
            // the wait for them) cannot be hoisted above the barrier.  With a
            // density contrast the longer stencil leaves no registers for that.
            if (!RHO) {
#pragma unroll
                for (int i = 0; i < Q; ++i) asm volatile("" : "+v"(fr[i]));
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                f[i] = E::value(fr[i]);
                pt += f[i];
                cacc<L>(i, f[i], mx, my, mz);
            }
            ux = mx + 0.5f * Fx;
            uy = my + 0.5f * Fy;
            uz = mz + 0.5f * Fz;
            if (RHO) {
                // rho u = sum c_i f_i + F/2;  p~ = sum f_i + u . grad rho / 2
                ux /= rho;
                uy /= rho;
                uz /= rho;
                pt += 0.5f * (ux * grx + uy * gry + uz * grz);
            }
        }
        const float uu = ux * ux + uy * uy + uz * uz;
        const float uu15 = 1.5f * uu;
        const unsigned own_off = ES * (unsigned)(yv[1] * QX);
        if (!solid) {
            const __amdgpu_buffer_rsrc_t fo = plane_rsrc(fdst, PL, c);
            float itau = ph.inv_tau, fp3 = fpref3, ug = 0.f;
            if (RHO) {
                // tau = tau_3 + (tau_2 - tau_3) H(C2 - C3)
                const bool liquid = C - (1.f - C1 - C) > 0.f;
                itau = liquid ? ph.inv_tau : ph.inv_tau3;
                fp3 = liquid ? fpref3 : 3.f * ph.fpref_gas;
                ug = ux * grx + uy * gry + uz * grz;
            }
            SeqS<L> sq;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const float si = sq.next(i, ux, uy, uz, uu15);
                const float cF = cdot<L>(i, Fx, Fy, Fz);
                float feq, fi;
                if (RHO) {
                    // F_i = (1 - 1/2tau) w_i [((c_i - u) . grad rho) s_i + c_i . F / c_s^2]
                    const float cg = cdot<L>(i, grx, gry, grz) - ug;
                    feq = L::w[i] * (pt + rho * si);
                    fi = fp3 * L::w[i] * (cF + (1.f / 3.f) * cg * si);
                } else {
                    feq = L::w[i] * (pt + si);
                    fi = fp3 * L::w[i] * cF;
                }
                E::store(fo, xb[1], own_off + ES * (unsigned)(i * XP), f[i] - (f[i] - feq) * itau + fi);
            }
        }
        const __amdgpu_buffer_rsrc_t go = plane_rsrc(gdst, PL, c);
        // moving populations first; the rest population takes what is left of
        // C (FP64), so the stored populations of the node keep its C
        double moved = 0.0;
        // held g: every LDS read issued before the first is used
        typename E::Raw gh[Q];
        if (E::lds_hold) {
#pragma unroll
            for (int i = 1; i < Q; ++i) gh[i] = s_gh[(j + 1) & 1][i - 1][t];
            __builtin_amdgcn_sched_barrier(0);
        }
        SeqS<L> sg;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float geq = L::w[i] * mu + L::w[i] * C * sg.next(i, ux, uy, uz, uu15);
            const float gc = E::lds_hold ? E::value(gh[i]) : gcoll[i];
            const float gs = gc - (gc - geq) * ph.inv_taug;
            moved += (double)E::store(go, xb[1], own_off + ES * (unsigned)(i * XP), gs);
        }
        __builtin_nontemporal_store(ccoll - moved, g0dst + (xv[1] + XP * ((long long)yv[1] + (long long)Y * c)));
        if (!isfinite(C) || !isfinite(uu)) flag[0] = 1;
    };

    double cA = 0.0, cB = 0.0;  // FP64 C of the own column, lead and collision plane
    const int J = zlen + 2;
    for (int j = 0; j < J; j += 2) {
        iteration(j, gA, gB, cA, cB);
        if (j + 1 < J) iteration(j + 1, gB, gA, cB, cA);
    }
}


// ---------------------------------------------------------------------------
// Pipelined tile (register-held elements).  The same march and arithmetic as
// fused_tile, with the memory operations reordered: the loads of plane j + 1
// (its pulled g, rest population and C1, and the f of the next collision
// plane) are issued right after the barrier of plane j, before plane j's
// collision and stores.  A lane's vector-memory operations complete in
// order, loads and stores alike, so a wait for a load also waits for every
// store issued before it; issued ahead of the stores, the next plane's loads
// never wait for them, and each plane's loads have a whole collision to land.
// Every memory operation of the steady-state loop is issued unconditionally
// (lanes outside the lattice and, for f, solid nodes address past the plane:
// their loads return 0 and their stores are dropped; the last plane's
// prefetch uses an empty descriptor), so the compiler's wait counts are exact.
typedef unsigned v2u __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;  // lane offset past every plane

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_v(const void* base, long long plane_bytes, int z,
                                                              bool valid) {
    const unsigned long long a = (unsigned long long)base + (unsigned long long)(plane_bytes * z);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    void* p = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, valid ? (int)plane_bytes : 0, kRsrcWord3);
}

template <int D, int TXW, int TY, int STAGE, bool PULL, bool RHO, typename E>
__device__ __forceinline__ void fused_tile_pipe(const Geom& g, const Phys& ph, const void* __restrict__ fsrc,
                                                const void* __restrict__ gsrc, void* __restrict__ fdst,
                                                void* __restrict__ gdst, const float* __restrict__ c1g,
                                                const uint8_t* __restrict__ mask, int* __restrict__ flag, int x0,
                                                int y0, int z0, int TZ) {
    using T = Tile<D, TXW, TY>;
    using L = Lattice<D>;
    constexpr int Q = L::Q;
    constexpr int CRX = T::CRX, CR = T::CR, HY = T::HY;
    __shared__ float s_c[4][CR];                                    // C of planes l-3..l (ring)
    __shared__ float s_c1[STAGE == 2 ? 4 : 1][STAGE == 2 ? CR : 1];  // frozen C1, same ring

    const int X = g.X, Y = g.Y, Z = g.Z, XP = g.XP;
    const int QX = Q * XP;                              // elements per row of populations
    const long long PL = (long long)QX * Y * E::bytes;  // bytes per plane of populations
    const long long RPL = (long long)XP * Y * 8;        // bytes per plane of the rest plane
    constexpr unsigned ES = E::bytes;
    const int zlen = min(TZ, Z - z0);

    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index (uniform)
    const int lane = t & 63;
    const int xseg = wv % TXW, yrow = wv / TXW;
    const int x = x0 + xseg * 64 + lane;
    const int y = y0 + yrow;  // uniform
    const bool active = (x < X) && (y < Y);
    // Lanes past the lattice's last column or row pull no g, except the first
    // one (column X, row Y): it holds C of the wrapped column (row) that the
    // last real one's stencil reads.  The others' ring cells are read by no
    // lattice node; their g pulls go past the plane and return 0 without
    // memory traffic (their rest value and C1 are still read: 12 of 84 bytes,
    // through plain loads that stay unconditional).
    const bool pulls = x <= X && y <= Y;
    const int rint = (1 + xseg * 64 + lane) + CRX * (HY + yrow);  // own region index
    // Region indices of the columns x - 1, x, x + 1 in the own row.  A tile
    // that spans its whole lattice row (x0 == 0, X <= TX) wraps them onto its
    // own columns and needs no side halo (whose loads are uncoalesced: each
    // of its lanes reads another row); other tiles use the halo columns at
    // either end of the region.
    const bool full_row = x0 == 0 && X <= T::TX;  // uniform
    const int xl = xseg * 64 + lane;            // column within the tile
    const int rrow = CRX * (HY + yrow);
    const int rcol[3] = {full_row ? 1 + pmod(xl - 1, X) : xl, xl + 1, full_row ? 1 + pmod(xl + 1, X) : xl + 2};

    const int xv[3] = {pmod(x - 1, X), pmod(x, X), pmod(x + 1, X)};  // x-1, x, x+1
    // as byte offsets; past the plane for a lane that pulls nothing (every
    // other access of such a lane is masked already)
    const unsigned xb[3] = {pulls ? ES * xv[0] : kOOB, pulls ? ES * xv[1] : kOOB, pulls ? ES * xv[2] : kOOB};
    const int yw = pmod(y, Y);
    const int yv[3] = {yw == 0 ? Y - 1 : yw - 1, yw, yw + 1 == Y ? 0 : yw + 1};

    const bool row_halo = wv < T::NROWH;  // uniform
    const int hbot = HY ? (wv / TXW) : 0;  // 0: row above the tile, 1: row below
    const int hyw = pmod(hbot ? y0 + TY : y0 - 1, Y);
    const int hyv[3] = {hyw == 0 ? Y - 1 : hyw - 1, hyw, hyw + 1 == Y ? 0 : hyw + 1};
    const int hreg = (1 + xseg * 64 + lane) + CRX * (hbot ? T::CRY - 1 : 0);
    const bool side = !full_row && wv == T::SIDE && lane < T::NSIDE;
    int srx = 0, sry = 0;
    if (side) T::side_pos(lane, srx, sry);
    const int sreg = srx + CRX * sry;
    const int sxw = pmod(x0 - 1 + srx, X), syw = pmod(y0 - HY + sry, Y);
    const int sxv[3] = {sxw == 0 ? X - 1 : sxw - 1, sxw, sxw + 1 == X ? 0 : sxw + 1};
    const int syv[3] = {syw == 0 ? Y - 1 : syw - 1, syw, syw + 1 == Y ? 0 : syw + 1};

    const float fpref3 = 3.f * ph.fpref;
    const float k13 = ph.k1 + ph.k3;
    const double* __restrict__ g0src = rest_plane(gsrc, Q, g.NP, ES);
    double* __restrict__ g0dst = rest_plane(gdst, Q, g.NP, ES);
    const unsigned own_off = ES * (unsigned)(yv[1] * QX);
    const unsigned g0_off = active ? 8u * (unsigned)(xv[1] + XP * yv[1]) : kOOB;

    float gF[Q], hF[Q], fF[Q];  // issued for the next plane
    float gN[Q], gC[Q], fN[Q];  // lead plane's g, collision plane's g and f
    double r0F = 0.0, hr0F = 0.0, cN = 0.0, cC = 0.0;
    float c1F = 0.f, hc1F = 0.f;
    uint8_t mF = 0, mN = 0;
    bool bad = false;
    const int J = zlen + 2;

    // loads of the lead plane of iteration jn: own column and halo column
    auto issue_g = [&](int jn, bool valid) {
        const int lz = pmod(z0 - 1 + jn, Z);
        const int zl[3] = {lz == 0 ? Z - 1 : lz - 1, lz, lz + 1 == Z ? 0 : lz + 1};
        const __amdgpu_buffer_rsrc_t gl[3] = {plane_rsrc_v(gsrc, PL, zl[0], valid),
                                              plane_rsrc_v(gsrc, PL, zl[1], valid),
                                              plane_rsrc_v(gsrc, PL, zl[2], valid)};
        r0F = g0src[xv[1] + XP * ((long long)yv[1] + (long long)Y * lz)];
        if (STAGE == 2) c1F = c1g[xv[1] + X * ((long long)yv[1] + (long long)Y * lz)];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
            gF[i] = E::load(gl[sz], xb[sx], ES * (unsigned)(yv[sy] * QX + i * XP));
        }
        if (row_halo) {
            hr0F = g0src[xv[1] + XP * ((long long)hyw + (long long)Y * lz)];
            if (STAGE == 2) hc1F = c1g[xv[1] + X * ((long long)hyw + (long long)Y * lz)];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
                hF[i] = E::load(gl[sz], xb[sx], ES * (unsigned)(hyv[sy] * QX + i * XP));
            }
        } else if (side) {
            hr0F = g0src[sxw + XP * ((long long)syw + (long long)Y * lz)];
            if (STAGE == 2) hc1F = c1g[sxw + X * ((long long)syw + (long long)Y * lz)];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
                hF[i] = E::load(gl[sz], ES * (unsigned)(syv[sy] * QX + i * XP + sxv[sx]), 0u);
            }
        }
    };
    // f of the collision plane of iteration jn (the lead plane of jn - 1);
    // need: the lane is a fluid node of the lattice
    auto issue_f = [&](int jn, bool valid, bool need) {
        const int cz = pmod(z0 - 2 + jn, Z);
        const int zc[3] = {cz == 0 ? Z - 1 : cz - 1, cz, cz + 1 == Z ? 0 : cz + 1};
        const __amdgpu_buffer_rsrc_t fc[3] = {plane_rsrc_v(fsrc, PL, zc[0], valid),
                                              plane_rsrc_v(fsrc, PL, zc[1], valid),
                                              plane_rsrc_v(fsrc, PL, zc[2], valid)};
        const unsigned xf[3] = {need ? xb[0] : kOOB, need ? xb[1] : kOOB, need ? xb[2] : kOOB};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int sy = PULL ? 1 - L::cy[i] : 1, sz = PULL ? 1 - L::cz[i] : 1, sx = PULL ? 1 - L::cx[i] : 1;
            fF[i] = E::load(fc[sz], xf[sx], ES * (unsigned)(yv[sy] * QX + i * XP));
        }
        if (STAGE == 1) mF = mask[xv[1] + X * ((long long)yv[1] + (long long)Y * cz)];
    };
    // phase 1: C = g_0 + sum_{i>0} g_i in FP64 of the lead plane (own column,
    // then the halo column, same summation order) into ring slot j & 3
    auto consume_lead = [&](int j) {
        const int sl = j & 3;
#pragma unroll
        for (int i = 1; i < Q; ++i) gN[i] = gF[i];
        double acc = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) acc += (double)gN[i];
        cN = r0F + acc;
        s_c[sl][rint] = (float)cN;
        if (STAGE == 2) s_c1[sl][rint] = c1F;
        if (row_halo || side) {
            double a = 0.0;
#pragma unroll
            for (int i = 1; i < Q; ++i) a += (double)hF[i];
            const int hr = row_halo ? hreg : sreg;
            s_c[sl][hr] = (float)(hr0F + a);
            if (STAGE == 2) s_c1[sl][hr] = hc1F;
        }
    };
    auto lead_solid = [&](int j) { return STAGE == 2 && s_c1[j & 3][rint] > 0.5f; };

    // warm-up: the two planes before the first collision
    issue_g(0, true);
    consume_lead(0);
    __syncthreads();
    issue_g(1, true);
    cC = cN;
#pragma unroll
    for (int i = 1; i < Q; ++i) gC[i] = gN[i];
    consume_lead(1);
    __syncthreads();
    issue_g(2, true);
    issue_f(2, true, active && !lead_solid(1));
    {
        // the stores of a collision, to an empty descriptor (all dropped): the
        // loop is entered with the same memory operations in flight as when
        // it goes round, so the waits inside it need not be conservative
        const __amdgpu_buffer_rsrc_t none = plane_rsrc_v(fdst, PL, 0, false);
#pragma unroll
        for (int i = 0; i < Q; ++i) E::store(none, kOOB, own_off + ES * (unsigned)(i * XP), 0.f);
#pragma unroll
        for (int i = 1; i < Q; ++i) E::store(none, kOOB, own_off + ES * (unsigned)(i * XP), 0.f);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, 0.0), none, (int)kOOB, 0, kNonTemporal);
    }
    cC = cN;
#pragma unroll
    for (int i = 1; i < Q; ++i) gC[i] = gN[i];

    for (int j = 2; j < J; ++j) {
        const int c = z0 - 2 + j;  // collision plane, inside [0, Z)
        consume_lead(j);
        __syncthreads();
        const int sm_ = (j + 2) & 3, s0 = (j + 3) & 3, sp = j & 3;  // planes c-1, c, c+1
        const bool solid = STAGE == 2 && s_c1[s0][rint] > 0.5f;
        // f of plane c (issued one plane ago): its moments first, so that the
        // wait for it comes before the next plane's loads are issued
#pragma unroll
        for (int i = 0; i < Q; ++i) fN[i] = fF[i];
        if (STAGE == 1) mN = mF;
        float pt = 0.f, mx = 0.f, my = 0.f, mz = 0.f;
        if (!solid) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                pt += fN[i];
                cacc<L>(i, fN[i], mx, my, mz);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        const bool more = j + 1 < J;  // uniform
        issue_g(j + 1, more);
        issue_f(j + 1, more, active && !lead_solid(j));
        __builtin_amdgcn_sched_barrier(0);

        // ---- collide plane c ------------------------------------------------
        const float C = s_c[s0][rint];
        float lc = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);  // plane of x + c_i
            const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);  // plane of x - c_i
            const int ip = rcol[1 + L::cx[i]] + rrow + CRX * L::cy[i];  // x + c_i
            const int im = rcol[1 - L::cx[i]] + rrow - CRX * L::cy[i];  // x - c_i
            const float a = s_c[spl][ip], bm = s_c[smi][im];
            lc += L::w[i] * ((a - C) + (bm - C));
            const float d = a - bm;
            wacc<L>(i, d, gx, gy, gz);
        }
        lc *= 6.f;
        float mu, C1 = 0.f;
        float rho = 1.f, grx = 0.f, gry = 0.f, grz = 0.f;
        if (STAGE == 2) {
            C1 = s_c1[s0][rint];
            float l1 = 0.f;
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                const int spl = L::cz[i] < 0 ? sm_ : (L::cz[i] > 0 ? sp : s0);
                const int smi = L::cz[i] < 0 ? sp : (L::cz[i] > 0 ? sm_ : s0);
                const int ip = rcol[1 + L::cx[i]] + rrow + CRX * L::cy[i];
                const int im = rcol[1 - L::cx[i]] + rrow - CRX * L::cy[i];
                const float a1 = s_c1[spl][ip], b1 = s_c1[smi][im];
                l1 += L::w[i] * ((a1 - C1) + (b1 - C1));
                if (RHO) {
                    const float d = local_density(ph, s_c[spl][ip], a1) - local_density(ph, s_c[smi][im], b1);
                    wacc<L>(i, d, grx, gry, grz);
                }
            }
            l1 *= 6.f;
            if (RHO) {
                rho = local_density(ph, C, C1);
                grx *= 3.f;
                gry *= 3.f;
                grz *= 3.f;
            }
            const float S = C1 + C;
            mu = ph.k2 * C * (1.f - C) * (1.f - 2.f * C) + ph.k3 * S * (1.f - S) * (1.f - 2.f * S) -
                 ph.a2 * ph.k2 * lc - ph.a2 * ph.k3 * (l1 + lc);
        } else {
            mu = k13 * C * (1.f - C) * (1.f - 2.f * C);
            const bool inS = mN != 0;
            if ((C < 0.5f && inS) || (C > 0.5f && !inS)) mu += 2.f * ph.beta * (C - 0.5f);
            mu -= ph.a2 * k13 * lc;
            if (C < 0.f) mu += 2.f * ph.omega * C;
            if (C > 1.f) mu -= 2.f * ph.omega * (1.f - C);
        }
        float ux = 0.f, uy = 0.f, uz = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
        if (!solid) {
            Fx = mu * 3.f * gx;
            Fy = mu * 3.f * gy;
            Fz = mu * 3.f * gz;
            if (STAGE == 2) {
                Fx += C * ph.grav[0];
                Fy += C * ph.grav[1];
                Fz += C * ph.grav[2];
            }
            ux = mx + 0.5f * Fx;
            uy = my + 0.5f * Fy;
            uz = mz + 0.5f * Fz;
            if (RHO) {
                ux /= rho;
                uy /= rho;
                uz /= rho;
                pt += 0.5f * (ux * grx + uy * gry + uz * grz);
            }
        }
        const float uu = ux * ux + uy * uy + uz * uz;
        const float uu15 = 1.5f * uu;
        const bool fluid = active && !solid;
        const __amdgpu_buffer_rsrc_t fo = plane_rsrc(fdst, PL, c);
        float itau = ph.inv_tau, fp3 = fpref3, ug = 0.f;
        if (RHO) {
            const bool liquid = C - (1.f - C1 - C) > 0.f;
            itau = liquid ? ph.inv_tau : ph.inv_tau3;
            fp3 = liquid ? fpref3 : 3.f * ph.fpref_gas;
            ug = ux * grx + uy * gry + uz * grz;
        }
        const unsigned xo = fluid ? xb[1] : kOOB;
        SeqS<L> sq;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float si = sq.next(i, ux, uy, uz, uu15);
            const float cF = cdot<L>(i, Fx, Fy, Fz);
            float feq, fi;
            if (RHO) {
                const float cg = cdot<L>(i, grx, gry, grz) - ug;
                feq = L::w[i] * (pt + rho * si);
                fi = fp3 * L::w[i] * (cF + (1.f / 3.f) * cg * si);
            } else {
                feq = L::w[i] * (pt + si);
                fi = fp3 * L::w[i] * cF;
            }
            E::store(fo, xo, own_off + ES * (unsigned)(i * XP), fN[i] - (fN[i] - feq) * itau + fi);
        }
        const __amdgpu_buffer_rsrc_t go = plane_rsrc(gdst, PL, c);
        const unsigned xg = active ? xb[1] : kOOB;
        double moved = 0.0;
        SeqS<L> sg;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float geq = L::w[i] * mu + L::w[i] * C * sg.next(i, ux, uy, uz, uu15);
            const float gs = gC[i] - (gC[i] - geq) * ph.inv_taug;
            moved += (double)E::store(go, xg, own_off + ES * (unsigned)(i * XP), gs);
        }
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<char*>(g0dst) + RPL * c, (short)0, (int)RPL, kRsrcWord3);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, cC - moved), ro, (int)g0_off, 0, kNonTemporal);
        bad |= active && (!isfinite(C) || !isfinite(uu));
        // the lead plane becomes the next collision plane
        cC = cN;
#pragma unroll
        for (int i = 1; i < Q; ++i) gC[i] = gN[i];
    }
    if (bad) flag[0] = 1;
}

template <int D, int TXW, int TY, int STAGE, bool PULL, bool RHO, typename E>
__device__ __forceinline__ void tile_step(const Geom& g, const Phys& ph, const void* __restrict__ fsrc,
                                          const void* __restrict__ gsrc, void* __restrict__ fdst,
                                          void* __restrict__ gdst, const float* __restrict__ c1g,
                                          const uint8_t* __restrict__ mask, int* __restrict__ flag, int x0, int y0,
                                          int z0, int TZ) {
    if constexpr (E::lds_hold && D == 3)
        fused_tile<D, TXW, TY, STAGE, PULL, RHO, E>(g, ph, fsrc, gsrc, fdst, gdst, c1g, mask, flag, x0, y0, z0, TZ);
    else
        fused_tile_pipe<D, TXW, TY, STAGE, PULL, RHO, E>(g, ph, fsrc, gsrc, fdst, gdst, c1g, mask, flag, x0, y0, z0,
                                                         TZ);
}

template <int D, int TXW, int TY, int STAGE, bool PULL, bool RHO, typename E>
__global__ void __launch_bounds__(64 * TXW * TY) __attribute__((amdgpu_waves_per_eu(D == 3 ? E::min_waves : 1)))
    k_step_fused(Geom g, Phys ph, const void* __restrict__ fsrc, const void* __restrict__ gsrc,
                 void* __restrict__ fdst, void* __restrict__ gdst, const float* __restrict__ c1g,
                 const uint8_t* __restrict__ mask, int* __restrict__ flag, int TZ, int ntx, int nty) {
    constexpr int TX = 64 * TXW;
    // XCD-aware tile order: hardware dispatch is round-robin over the 8 XCDs,
    // so XCD k (= blockIdx % 8) is given a contiguous range of tiles
    const int nb = gridDim.x, b = blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
    const int tile = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int tile_x = tile % ntx, rest = tile / ntx;
    const int tile_y = rest % nty, tile_z = rest / nty;
    tile_step<D, TXW, TY, STAGE, PULL, RHO, E>(g, ph, fsrc, gsrc, fdst, gdst, c1g, mask, flag, tile_x * TX,
                                                tile_y * TY, tile_z * TZ, TZ);
}

// Batched step: many lattices (same lattice type, storage and contrast
// variant) advance in one
// persistent launch.  The work list holds (lattice, tile) items, costliest
// first; each workgroup takes the next item from a shared counter (reset to
// zero by the bounce kernel that precedes every batched step) until the list
// is drained, so uneven lattices balance over the chip.  Each lattice's
// geometry, parameters and buffers come from a descriptor table, with the
// two buffer pairs exchanged by the step parity.
template <int D, int TXW, int TY, bool RHO, typename E>
__global__ void __launch_bounds__(64 * TXW * TY) __attribute__((amdgpu_waves_per_eu(D == 3 ? E::min_waves : 1)))
    k_step_batch(const BatchInst* __restrict__ inst, const BatchItem* __restrict__ items, int nitems,
                 int* __restrict__ counter, int parity, int TZ) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();  // also: every wave has left the previous item
        const int it = s_item;
        if (it >= nitems) break;  // uniform over the workgroup
        const BatchItem w = items[it];
        const BatchInst& d = inst[w.inst];
        tile_step<D, TXW, TY, 2, true, RHO, E>(d.geom, d.phys, d.f[parity], d.g[parity], d.f[1 - parity],
                                                d.g[1 - parity], d.c1, d.mask, d.flag, w.x0, w.y0, w.z0, TZ);
        __syncthreads();  // s_item is rewritten only after every wave has read it
    }
}

template <int D, int TXW, int TY, int STAGE, bool PULL, bool RHO, typename E>
hipError_t launch_cfg(const Geom& g, const Phys& ph, const void* fsrc, const void* gsrc, void* fdst, void* gdst,
                      const float* c1, const uint8_t* mask, int* flag, int TZ, hipStream_t st) {
    constexpr int TX = 64 * TXW;
    const int ntx = (g.X + TX - 1) / TX;
    const int nty = (g.Y + TY - 1) / TY;
    const int ntz = (g.Z + TZ - 1) / TZ;
    const long long nblocks = (long long)ntx * nty * ntz;
    if (nblocks < 1 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_step_fused<D, TXW, TY, STAGE, PULL, RHO, E>), dim3((unsigned)nblocks), dim3(64 * TXW * TY), 0,
                       st, g, ph, fsrc, gsrc, fdst, gdst, c1, mask, flag, TZ, ntx, nty);
    return hipGetLastError();
}

template <int D, int TXW, int TY, typename E>
hipError_t launch_tile_e(const Geom& g, const Phys& ph, Pop fsrc, Pop gsrc, Pop fdst, Pop gdst, const float* c1,
                         const uint8_t* mask, int pull, int* flag, int TZ, hipStream_t st) {
    const void *fs = fsrc.p, *gs = gsrc.p;
    void *fd = fdst.p, *gd = gdst.p;
    if (ph.stage == 2 && ph.contrast) {
        if (pull) return launch_cfg<D, TXW, TY, 2, true, true, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
        return launch_cfg<D, TXW, TY, 2, false, true, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
    }
    if (ph.stage == 2) {
        if (pull) return launch_cfg<D, TXW, TY, 2, true, false, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
        return launch_cfg<D, TXW, TY, 2, false, false, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
    }
    if (pull) return launch_cfg<D, TXW, TY, 1, true, false, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
    return launch_cfg<D, TXW, TY, 1, false, false, E>(g, ph, fs, gs, fd, gd, c1, mask, flag, TZ, st);
}

template <int D, int TXW, int TY>
hipError_t launch_tile(const Geom& g, const Phys& ph, Pop fsrc, Pop gsrc, Pop fdst, Pop gdst, const float* c1,
                       const uint8_t* mask, int pull, int* flag, int TZ, hipStream_t st) {
    if (fsrc.half) return launch_tile_e<D, TXW, TY, F16>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
    return launch_tile_e<D, TXW, TY, F32>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
}

}  // namespace

template <int D, int TXW, int TY, bool RHO, typename E>
auto batch_kernel() {
    return k_step_batch<D, TXW, TY, RHO, E>;
}

template <int D, int TXW, int TY, bool RHO>
hipError_t launch_batch_rho(const BatchInst* inst, const BatchItem* items, int nitems, int* counter, int blocks,
                            int parity, int TZ, int half, hipStream_t st) {
    if (half)
        hipLaunchKernelGGL((k_step_batch<D, TXW, TY, RHO, F16>), dim3(blocks), dim3(64 * TXW * TY), 0, st, inst,
                           items, nitems, counter, parity, TZ);
    else
        hipLaunchKernelGGL((k_step_batch<D, TXW, TY, RHO, F32>), dim3(blocks), dim3(64 * TXW * TY), 0, st, inst,
                           items, nitems, counter, parity, TZ);
    return hipGetLastError();
}

template <int D, int TXW, int TY>
hipError_t launch_batch_tile(const BatchInst* inst, const BatchItem* items, int nitems, int* counter, int grid,
                             int parity, int TZ, int half, int rho, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = grid < nitems ? grid : nitems;
    if (rho) return launch_batch_rho<D, TXW, TY, true>(inst, items, nitems, counter, blocks, parity, TZ, half, st);
    return launch_batch_rho<D, TXW, TY, false>(inst, items, nitems, counter, blocks, parity, TZ, half, st);
}

template <int D, int TXW, int TY, bool RHO>
int batch_occupancy_rho(int half) {
    int n = 0;
    hipError_t e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<D, TXW, TY, RHO, F16>(),
                                                                      64 * TXW * TY, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<D, TXW, TY, RHO, F32>(),
                                                                      64 * TXW * TY, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int D, int TXW, int TY>
int batch_occupancy_tile(int half, int rho) {
    return rho ? batch_occupancy_rho<D, TXW, TY, true>(half) : batch_occupancy_rho<D, TXW, TY, false>(half);
}

int fused_tile_variants(int dim) { return 3; }

void fused_tile_shape(int dim, int variant, int* tx, int* ty) {
    static const int t2[3][2] = {{256, 1}, {128, 1}, {64, 1}};
    static const int t3[3][2] = {{64, 4}, {64, 8}, {128, 4}};
    const int v = variant < 0 || variant > 2 ? 0 : variant;
    *tx = dim == 2 ? t2[v][0] : t3[v][0];
    *ty = dim == 2 ? t2[v][1] : t3[v][1];
}

hipError_t launch_step_batch(int dim, int variant, int half, int rho, const BatchInst* inst, const BatchItem* items,
                             int nitems, int* counter, int grid, int parity, int TZ, hipStream_t st) {
    if (TZ < 1) TZ = 1;
    if (dim == 2) {
        switch (variant) {
            case 1: return launch_batch_tile<2, 2, 1>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
            case 2: return launch_batch_tile<2, 1, 1>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
            default: return launch_batch_tile<2, 4, 1>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
        }
    }
    switch (variant) {
        case 1: return launch_batch_tile<3, 1, 8>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
        case 2: return launch_batch_tile<3, 2, 4>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
        default: return launch_batch_tile<3, 1, 4>(inst, items, nitems, counter, grid, parity, TZ, half, rho, st);
    }
}

int batch_blocks_per_cu(int dim, int variant, int half, int rho) {
    if (dim == 2) {
        switch (variant) {
            case 1: return batch_occupancy_tile<2, 2, 1>(half, rho);
            case 2: return batch_occupancy_tile<2, 1, 1>(half, rho);
            default: return batch_occupancy_tile<2, 4, 1>(half, rho);
        }
    }
    switch (variant) {
        case 1: return batch_occupancy_tile<3, 1, 8>(half, rho);
        case 2: return batch_occupancy_tile<3, 2, 4>(half, rho);
        default: return batch_occupancy_tile<3, 1, 4>(half, rho);
    }
}

namespace {
template <int D, int TXW, int TY, bool RHO, typename E>
int fused_occupancy() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_fused<D, TXW, TY, 2, true, RHO, E>,
                                                                      64 * TXW * TY, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}
template <int D, int TXW, int TY>
int fused_occupancy_tile(int half, int rho) {
    if (rho) return half ? fused_occupancy<D, TXW, TY, true, F16>() : fused_occupancy<D, TXW, TY, true, F32>();
    return half ? fused_occupancy<D, TXW, TY, false, F16>() : fused_occupancy<D, TXW, TY, false, F32>();
}
}  // namespace

int fused_blocks_per_cu(int dim, int variant, int half, int rho) {
    if (dim == 2) {
        switch (variant) {
            case 1: return fused_occupancy_tile<2, 2, 1>(half, rho);
            case 2: return fused_occupancy_tile<2, 1, 1>(half, rho);
            default: return fused_occupancy_tile<2, 4, 1>(half, rho);
        }
    }
    switch (variant) {
        case 1: return fused_occupancy_tile<3, 1, 8>(half, rho);
        case 2: return fused_occupancy_tile<3, 2, 4>(half, rho);
        default: return fused_occupancy_tile<3, 1, 4>(half, rho);
    }
}

hipError_t launch_step_fused(int dim, const Geom& g, const Phys& ph, Pop fsrc, Pop gsrc, Pop fdst, Pop gdst,
                             const float* c1, const uint8_t* mask, int pull, int* flag,
                             int variant, int TZ, hipStream_t st) {
    if (TZ < 1) TZ = 1;
    if (dim == 2) {
        switch (variant) {
            case 1: return launch_tile<2, 2, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
            case 2: return launch_tile<2, 1, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
            default: return launch_tile<2, 4, 1>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        }
    }
    switch (variant) {
        case 1: return launch_tile<3, 1, 8>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        case 2: return launch_tile<3, 2, 4>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
        default: return launch_tile<3, 1, 4>(g, ph, fsrc, gsrc, fdst, gdst, c1, mask, pull, flag, TZ, st);
    }
}

}  // namespace dsm
