// dsm_api.hip -- host side of the libdsm.so C ABI (include/dsm.h).
//
// Validates arguments before any HIP call, carves the device arrays out of
// the caller's buffer, converts host FP64 fields to device FP32 and back, and
// enqueues the kernels on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dsm_host.h"

using namespace dsm;

namespace {

thread_local std::string g_last_error;

}  // namespace

int dsm::set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

namespace {

int fail(int code, const std::string& msg) { return set_error(code, msg); }

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(DSM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

constexpr size_t kAlign = 256;
constexpr uint32_t kStateMagic = 0x44534d31u;  // "DSM1"

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int lattice_q(int dim) { return dim == 2 ? 9 : 19; }

// Returns an error message for invalid parameters, or nullptr.
const char* validate(const dsm_params* p) {
    if (!p) return "params is NULL";
    if (p->dim != 2 && p->dim != 3) return "dim must be 2 or 3";
    if (p->nx < 4 || p->ny < 4) return "nx and ny must be >= 4";
    if (p->dim == 2 && p->nz != 1) return "nz must be 1 when dim == 2";
    if (p->dim == 3 && p->nz < 4) return "nz must be >= 4 when dim == 3";
    // population slots, rows padded to the row pitch (at most 63 elements more)
    const double slots = ((double)p->nx + 64.0) * (double)p->ny * (double)p->nz * lattice_q(p->dim);
    if (slots > 4294967295.0) return "lattice has more than 2^32 - 1 populations";
    if (((double)p->nx + 64.0) * (double)(p->dim == 3 ? p->ny : 1) * lattice_q(p->dim) * 4.0 > 2147483647.0)
        return "one lattice plane of populations exceeds 2 GiB";
    for (int k = 0; k < 3; ++k)
        if (!(p->kappa[k] >= 0.0) || !isfinite(p->kappa[k])) return "kappa must be finite and >= 0";
    if (!(p->kappa[1] + p->kappa[2] > 0.0)) return "kappa_2 + kappa_3 must be > 0";
    if (!(p->alpha > 0.0) || !isfinite(p->alpha)) return "alpha must be > 0";
    if (!(p->tau > 0.5) || !isfinite(p->tau)) return "tau must be > 1/2";
    if (!(p->mobility > 0.0) || !isfinite(p->mobility)) return "mobility must be > 0";
    for (int k = 0; k < 3; ++k)
        if (!isfinite(p->gravity[k])) return "gravity must be finite";
    if (p->dim == 2 && p->gravity[2] != 0.0) return "gravity[2] must be 0 when dim == 2";
    if (p->reduce_every < 0) return "reduce_every must be >= 0";
    if (p->kernel != DSM_KERNEL_FUSED && p->kernel != DSM_KERNEL_SPLIT) return "unknown kernel";
    if (p->storage != DSM_STORAGE_FP32 && p->storage != DSM_STORAGE_FP16) return "unknown storage";
    for (int k = 0; k < 2; ++k)
        if (!(p->rho[k] >= 0.0) || !isfinite(p->rho[k])) return "rho must be finite and > 0 (0 selects 1)";
    if (!(p->tau_gas == 0.0 || p->tau_gas > 0.5) || !isfinite(p->tau_gas))
        return "tau_gas must be > 1/2 (0 selects tau)";
    return nullptr;
}

struct Layout {
    size_t off_f[2], off_g[2], off_c1, off_mask, off_phi, off_mu, off_aux, off_part, off_red, off_flag, off_links,
        off_ent, off_nlinks;
    size_t total;
};

Layout make_layout(const dsm_params* p) {
    Layout L;
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t Q = (size_t)lattice_q(p->dim);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int es = p->storage == DSM_STORAGE_FP16 ? 2 : 4;
    const size_t NP = (size_t)row_pitch(p->nx, es) * (N / (size_t)p->nx);  // padded rows
    const size_t fbytes = (size_t)pop_bytes((int)Q, (long long)NP, es);
    L.off_f[0] = take(fbytes);
    const size_t gbytes = fbytes + NP * sizeof(double);
    L.off_g[0] = take(gbytes);
    L.off_f[1] = take(fbytes);
    L.off_g[1] = take(gbytes);
    L.off_c1 = take(N * sizeof(float));
    L.off_mask = take(N);
    L.off_phi = take(N * sizeof(float));
    L.off_mu = take(N * sizeof(float));
    L.off_aux = take(4 * N * sizeof(float));
    L.off_part = take((size_t)kReduceBlocks * RED_SLOTS * sizeof(double));
    L.off_red = take(RED_SLOTS * sizeof(double));
    L.off_flag = take(4 * sizeof(int));
    L.off_ent = take(N * sizeof(int2));
    L.off_links = take((size_t)kLinksPerNode * N * sizeof(LinkRec));
    L.off_nlinks = take(4 * sizeof(int));
    L.total = o;
    return L;
}

struct StateHeader {
    uint32_t magic, version;
    int32_t dim, nx, ny, nz, stage, pull;
    int64_t steps;
    double gravity[3];
    double beta, omega, tau_s, taug_s;
};

}  // namespace

Phys dsm::sim_phys(const dsm_sim* s, int stage) {
    Phys ph;
    ph.k1 = (float)s->p.kappa[0];
    ph.k2 = (float)s->p.kappa[1];
    ph.k3 = (float)s->p.kappa[2];
    ph.a2 = (float)(s->p.alpha * s->p.alpha);
    ph.alpha = (float)s->p.alpha;
    double tau = stage == 1 ? s->tau_s : s->p.tau;
    double taug = stage == 1 ? s->taug_s : 0.5 + 3.0 * s->p.mobility;
    ph.inv_tau = (float)(1.0 / tau);
    ph.inv_taug = (float)(1.0 / taug);
    ph.fpref = (float)(1.0 - 0.5 / tau);
    // user axes -> stored axes (2D stores y along the slow axis)
    if (s->p.dim == 2) {
        ph.grav[0] = (float)s->p.gravity[0];
        ph.grav[1] = 0.f;
        ph.grav[2] = (float)s->p.gravity[1];
    } else {
        for (int k = 0; k < 3; ++k) ph.grav[k] = (float)s->p.gravity[k];
    }
    ph.beta = (float)s->beta;
    ph.omega = (float)s->omega;
    ph.stage = stage;
    // density and viscosity contrast (fluid stage only)
    const double r2 = s->p.rho[0] > 0.0 ? s->p.rho[0] : 1.0, r3 = s->p.rho[1] > 0.0 ? s->p.rho[1] : 1.0;
    const double tau3 = s->p.tau_gas > 0.0 ? s->p.tau_gas : s->p.tau;
    ph.rho2 = (float)r2;
    ph.rho3 = (float)r3;
    ph.inv_tau3 = (float)(1.0 / tau3);
    ph.fpref_gas = (float)(1.0 - 0.5 / tau3);
    ph.contrast = stage == 2 && (r2 != 1.0 || r3 != 1.0 || tau3 != s->p.tau) ? 1 : 0;
    return ph;
}

namespace {

Phys make_phys(const dsm_sim* s, int stage) { return sim_phys(s, stage); }

int upload_field(dsm_sim* s, const double* host, float* dev) {
    const size_t N = (size_t)s->N;
    s->stage_buf.resize(N);
    for (size_t n = 0; n < N; ++n) s->stage_buf[n] = (float)host[n];
    HIP_TRY(hipMemcpyAsync(dev, s->stage_buf.data(), N * sizeof(float), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return DSM_OK;
}

int download_field(dsm_sim* s, const float* dev, double* host, size_t count) {
    s->stage_buf.resize(count);
    HIP_TRY(hipMemcpyAsync(s->stage_buf.data(), dev, count * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t n = 0; n < count; ++n) host[n] = (double)s->stage_buf[n];
    return DSM_OK;
}

// Population buffers as the kernels take them.
Pop PF(const dsm_sim* s, int k) { return Pop{s->d.f[k], s->half}; }
Pop PG(const dsm_sim* s, int k) { return Pop{s->d.g[k], s->half}; }
size_t f_bytes(const dsm_sim* s) { return (size_t)pop_bytes(s->Q, s->geom.NP, s->es); }
size_t g_bytes(const dsm_sim* s) { return f_bytes(s) + (size_t)s->geom.NP * sizeof(double); }

// Element copies between the device layout and FP32 host staging (FP16
// elements hold value * kHalfScale).
int fetch_elems(dsm_sim* s, const void* dev, size_t count) {
    s->stage_buf.resize(count);
    if (!s->half) {
        HIP_TRY(hipMemcpyAsync(s->stage_buf.data(), dev, count * 4, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return DSM_OK;
    }
    s->stage16.resize(count);
    HIP_TRY(hipMemcpyAsync(s->stage16.data(), dev, count * 2, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t k = 0; k < count; ++k)
        s->stage_buf[k] = __half2float(__ushort_as_half(s->stage16[k])) * (1.f / kHalfScale);
    return DSM_OK;
}

int send_elems(dsm_sim* s, void* dev, size_t count) {
    if (!s->half) {
        HIP_TRY(hipMemcpyAsync(dev, s->stage_buf.data(), count * 4, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return DSM_OK;
    }
    s->stage16.resize(count);
    for (size_t k = 0; k < count; ++k) s->stage16[k] = __half_as_ushort(__float2half(s->stage_buf[k] * kHalfScale));
    HIP_TRY(hipMemcpyAsync(dev, s->stage16.data(), count * 2, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return DSM_OK;
}

// Populations: host arrays are [Q][N] (direction-major planes of nodes); the
// device stores them row-interleaved with row pitch XP, (row*Q + i)*XP + x
// with n = x + X*row (pop_index), and the FP64 rest plane with the same pitch.
// For g the rest population (direction 0) lives in the FP64 rest plane.
int download_pops(dsm_sim* s, const void* dev, double* host, bool is_g) {
    const size_t X = (size_t)s->geom.X, XP = (size_t)s->geom.XP, N = (size_t)s->N, Q = (size_t)s->Q,
                 rows = N / X;
    int rc = fetch_elems(s, dev, Q * rows * XP);
    if (rc) return rc;
    for (size_t r = 0; r < rows; ++r)
        for (size_t i = 0; i < Q; ++i)
            for (size_t x = 0; x < X; ++x) host[i * N + r * X + x] = (double)s->stage_buf[(r * Q + i) * XP + x];
    if (is_g) {
        HIP_TRY(hipMemcpy2DAsync(host, X * sizeof(double), rest_plane(dev, (int)Q, s->geom.NP, s->es),
                                 XP * sizeof(double), X * sizeof(double), rows, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return DSM_OK;
}

int upload_pops_one(dsm_sim* s, const double* host, void* dev, bool is_g) {
    const size_t X = (size_t)s->geom.X, XP = (size_t)s->geom.XP, N = (size_t)s->N, Q = (size_t)s->Q,
                 rows = N / X;
    s->stage_buf.assign(Q * rows * XP, 0.f);  // padding stays zero
    for (size_t r = 0; r < rows; ++r)
        for (size_t i = 0; i < Q; ++i)
            for (size_t x = 0; x < X; ++x)
                s->stage_buf[(r * Q + i) * XP + x] = (is_g && i == 0) ? 0.f : (float)host[i * N + r * X + x];
    int rc = send_elems(s, dev, Q * rows * XP);
    if (rc) return rc;
    if (is_g) {
        HIP_TRY(hipMemcpy2DAsync(rest_plane(dev, (int)Q, s->geom.NP, s->es), XP * sizeof(double), host,
                                 X * sizeof(double), X * sizeof(double), rows, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return DSM_OK;
}

// The fused step leaves f of solid nodes untouched (it is never read), so the
// spare buffer pair is cleared whenever a new state is installed: every byte of
// the state then depends only on the inputs.
int clear_spare_f(dsm_sim* s, int spare) {
    HIP_TRY(hipMemsetAsync(s->d.f[spare], 0, f_bytes(s), s->stream));
    return DSM_OK;
}

// Observables of the live state into phi, mu and aux.
int observe(dsm_sim* s) {
    const Phys ph = make_phys(s, s->stage);
    const int c = s->cur;
    HIP_TRY(launch_moment(s->p.dim, s->geom, PG(s, c), s->d.phi, s->pull, s->stream));
    HIP_TRY(launch_mu(s->p.dim, s->geom, ph, s->d.phi, s->d.c1, s->d.mask, s->d.mu, s->stream));
    HIP_TRY(launch_observe(s->p.dim, s->geom, ph, PF(s, c), s->d.c1, s->d.phi, s->d.mu, s->pull, s->d.aux,
                           s->stream));
    return DSM_OK;
}

int reduce(dsm_sim* s, double out[RED_SLOTS]) {
    int rc = observe(s);
    if (rc) return rc;
    const Phys ph = make_phys(s, s->stage);
    HIP_TRY(launch_reduce(s->p.dim, s->geom, ph, s->d.c1, s->d.phi, s->d.mask, s->d.aux, PG(s, s->cur), s->pull,
                          s->d.partials, s->d.red, s->stream));
    HIP_TRY(hipMemcpyAsync(out, s->d.red, RED_SLOTS * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return DSM_OK;
}

// Cut-link table of the fluid stage for the current C1.
int build_links(dsm_sim* s) {
    HIP_TRY(launch_find_links(s->p.dim, s->geom, s->d.c1, s->d.ent, s->d.nlinks, s->stream));
    int count[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(count, s->d.nlinks, sizeof(count), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const long long cap = (long long)kLinksPerNode * s->N;
    HIP_TRY(launch_build_links(s->p.dim, s->geom, s->p.alpha, s->d.c1, s->d.ent, count[0], s->d.links, cap,
                               s->d.nlinks, s->stream));
    HIP_TRY(hipMemcpyAsync(count, s->d.nlinks, sizeof(count), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->nlinks = 0;
    if (count[1] > cap)
        return fail(DSM_EINVAL, "solid surface has more cut links than the table holds (" +
                                    std::to_string(count[1]) + " > " + std::to_string(cap) + ")");
    // Order the records by the slot they write.  A slot index runs along x
    // within one direction row of one lattice row, so consecutive threads of
    // the link kernel then read and write neighbouring elements (the records
    // come out of the search in the order its atomics happened to run, which
    // scatters every wave's accesses over the lattice).  Each slot has one
    // record, so the order changes no result.
    if (count[1] > 1) {
        std::vector<LinkRec> h((size_t)count[1]);
        const size_t bytes = h.size() * sizeof(LinkRec);
        HIP_TRY(hipMemcpyAsync(h.data(), s->d.links, bytes, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        std::sort(h.begin(), h.end(), [](const LinkRec& a, const LinkRec& b) { return a.dst < b.dst; });
        HIP_TRY(hipMemcpyAsync(s->d.links, h.data(), bytes, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    s->nlinks = count[1];
    return DSM_OK;
}

// One time step of the live stage: reads buffer pair cur, writes 1 - cur.
int one_step(dsm_sim* s) {
    const Phys ph = make_phys(s, s->stage);
    const int c = s->cur, n = 1 - s->cur;
    if (s->p.kernel == DSM_KERNEL_FUSED) {
        if (s->stage == 2 && s->pull)
            HIP_TRY(launch_bounce(PF(s, c), s->d.links, s->nlinks, s->stream));
        HIP_TRY(launch_step_fused(s->p.dim, s->geom, ph, PF(s, c), PG(s, c), PF(s, n), PG(s, n), s->d.c1,
                                  s->d.mask, s->pull, s->d.flag, s->tile_variant, s->tile_planes, s->stream));
    } else {
        HIP_TRY(launch_moment(s->p.dim, s->geom, PG(s, c), s->d.phi, s->pull, s->stream));
        HIP_TRY(launch_mu(s->p.dim, s->geom, ph, s->d.phi, s->d.c1, s->d.mask, s->d.mu, s->stream));
        HIP_TRY(launch_collide_split(s->p.dim, s->geom, ph, PF(s, c), PG(s, c), PF(s, n), PG(s, n),
                                     s->d.c1, s->d.phi, s->d.mu, s->pull, s->d.flag, s->stream));
    }
    s->cur = n;
    s->pull = 1;
    return DSM_OK;
}

// Sets f = 0, g = g_eq(phi, mu(phi), 0) from the field already in d.phi.
int init_populations(dsm_sim* s, int stage) {
    const Phys ph = make_phys(s, stage);
    HIP_TRY(launch_mu(s->p.dim, s->geom, ph, s->d.phi, s->d.c1, s->d.mask, s->d.mu, s->stream));
    HIP_TRY(launch_init_populations(s->p.dim, s->geom, s->d.phi, s->d.mu, PF(s, 0), PG(s, 0), s->stream));
    s->cur = 0;
    s->pull = 0;
    return clear_spare_f(s, 1);
}

int check_flag(dsm_sim* s) {
    int h[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, s->d.flag, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (h[0]) return fail(DSM_EUNSTABLE, "non-finite values in the lattice state");
    return DSM_OK;
}

}  // namespace

// Default march of the default tile (3D variant 2, 2D variant 0), for a chip
// of `slots` tile slots (CUs x tiles resident per CU).
//
// 3D: of marches of 8 to 128 planes, the one that takes the fewest whole
// rounds of tiles times planes, each march's two fill planes counted as 0.36
// of a plane (ties go to the longer march, which re-reads fewer fill planes).
// Measured on MI355X: 128 x 256 x 128 FP32 at 17.5 GLUPS with 32 planes
// against 16.9 with 16; 80^3 FP32 at 9.8 with 8 against 6.5 with 16; the
// 256 x 256 x 192 pillar lattice with 96 planes in FP32 (one round of 256
// tiles: 736.9 us against 771.1 with 32) and 48 in FP16 (one round at two
// tiles per CU: 481.2 us against 489.4 with 16); 128^3 keeps 16 (FP32) and 8
// (FP16).
//
// 2D: 16 rows when the grid fills every slot in whole rounds, the last at
// least 80 % busy, else 8: rows of 1000 columns keep 16, narrower ones gain
// from 8, e.g. D2Q9 200 x 4096 at 25.1 GLUPS against 23.4 (FP16 30.9
// against 24.4).
int default_planes(const Geom& g, int dim, int slots) {
    int tx = 0, ty = 0;
    fused_tile_shape(dim, dim == 3 ? 2 : 0, &tx, &ty);
    const long long tiles = (long long)((g.X + tx - 1) / tx) * ((g.Y + ty - 1) / ty);
    if (slots < 1) return 16;
    if (dim == 2) {
        const long long n = tiles * ((g.Z + 15) / 16);
        const long long rounds = (n + slots - 1) / slots;
        return n >= slots && (double)n >= 0.8 * (double)(rounds * slots) ? 16 : 8;
    }
    double best = 0.0;
    int planes = 16;
    for (int p : {128, 96, 64, 48, 32, 16, 8}) {
        const long long n = tiles * ((g.Z + p - 1) / p);
        const double t = (double)((n + slots - 1) / slots) * ((p < g.Z ? p : g.Z) + 0.72);
        if (p == 128 || t < best - 1e-9) best = t, planes = p;
    }
    return planes;
}

// Tilings of lattices unlike the measured ones above (narrow 2D rows, small
// cubes, rows just wider than a tile) take the schedule model of the batched
// step, applied to the lattice alone: every tile variant with a march of 8,
// 16 or 32 planes, against the fixed default, which is kept unless the model
// predicts another at least 10 % faster.  Over 32 measured lattices (2D
// widths 100-1000, cubes 64-160) that never chose a slower tiling and gained
// 10 % on average, e.g. D2Q9 300 x 8192 at 29.6 GLUPS against 26.0 and
// D3Q19 64^3 at 6.8 against 3.5.  Every tiling gives bit-identical results.
// A 2D lattice whose 8-row marches of a variant make less than one round of
// resident workgroups is bound by the latency of its marches, and that
// variant also gets 4-row marches: D2Q9 128 x 64, 256^2 and 512 x 128 step in
// 11.9-13.2 us against 18.2-19.7, D2Q9 100 x 4096 in 21.0 against 22.6 (FP16
// 18.1 against 23.3); grids of a round or more keep 8 rows or longer (300 x
// 8192: 85.0 us with 8, 87.7 with 4).
//
// A lattice whose default grid fills at most half a round is latency-bound
// as a whole: its marches all run at once, so the step lasts the longest
// march (whole rounds of it), and short marches beat the default's despite
// their fill planes.  For those the latency form of the model
// (lattice_latency_cost) picks among every variant and marches of 2-32
// planes (1-32 rows in 2D), again only when it predicts 10 % or more.
// Measured (fused kernel): 48^3 22.7 us against 37.9 with the 8-plane
// default (FP16 20.1 against 38.1), 64^3 23.8 against 38.4 (FP16 21.1
// against 39.1), 128 x 64 x 64 39.7 against 53.4 (FP16 29.7 against 47.2),
// 80^3 FP16 46.0 against 48.0; D2Q9 128 x 64 7.4 against 12.4 with 4-row
// marches, 256^2 8.4 against 12.9, 64 x 2048 9.8 against 12.4, 512^2 FP16
// 13.1 against 14.6.  Over 26 3D and 22 2D lattices none was slower.  In 3D
// with FP16 elements, whose rounds overlap (two tiles per CU), the form also
// covers grids of up to 0.75 of a round: 96^3 66.6 against 77.8 us, 104^3
// 68.7 against 80.0, 96 x 96 x 192 116.0 against 142.1.
static void default_tiling_by_model(dsm_sim* s, int cus) {
    const int dim = s->p.dim, rho = make_phys(s, 2).contrast;
    auto bpc = [&](int v) { return fused_blocks_per_cu(dim, v, s->half, rho); };
    auto items_of = [&](int v, int planes) {
        int tx = 0, ty = 0;
        fused_tile_shape(dim, v, &tx, &ty);
        return (long long)((s->geom.X + tx - 1) / tx) * ((s->geom.Y + ty - 1) / ty) *
               ((s->geom.Z + planes - 1) / planes);
    };
    const double bound = dim == 3 && s->half ? 0.75 : 0.5;  // share of a round
    if ((double)items_of(s->tile_variant, s->tile_planes) <= bound * cus * bpc(s->tile_variant)) {
        auto lcost = [&](int v, int planes) {
            return lattice_latency_cost(s->geom, dim, v, planes, bpc(v), cus, s->half);
        };
        const double l0 = lcost(s->tile_variant, s->tile_planes);
        double best = l0;
        int bv = s->tile_variant, bp = s->tile_planes;
        for (int v = 0; v < fused_tile_variants(dim); ++v)
            for (int planes : {1, 2, 4, 8, 16, 32}) {
                if (planes == 1 && dim == 3) continue;  // 3D marches were measured from 2 planes
                const double c = lcost(v, planes);
                if (c < best) best = c, bv = v, bp = planes;
            }
        if (best < 0.9 * l0) {
            s->tile_variant = bv;
            s->tile_planes = bp;
        }
        return;
    }
    auto cost = [&](int v, int planes) { return lattice_schedule_cost(s->geom, dim, v, planes, bpc(v), cus); };
    auto under_one_round = [&](int v, int planes) { return items_of(v, planes) < (long long)cus * bpc(v); };
    const double c0 = cost(s->tile_variant, s->tile_planes);
    double best = c0;
    int bv = s->tile_variant, bp = s->tile_planes;
    for (int v = 0; v < fused_tile_variants(dim); ++v)
        for (int planes : {4, 8, 16, 32}) {
            if (planes == 4 && !(dim == 2 && under_one_round(v, 8))) continue;
            const double c = cost(v, planes);
            if (c < best) best = c, bv = v, bp = planes;
        }
    if (best < 0.9 * c0) {
        s->tile_variant = bv;
        s->tile_planes = bp;
    }
}

extern "C" {

size_t dsm_required_bytes(const dsm_params* p) {
    if (validate(p)) return 0;
    return make_layout(p).total;
}

int dsm_create(const dsm_params* p, const uint8_t* mask, void* dev_buf, size_t dev_bytes, void* stream,
               dsm_sim** out) {
    if (!out) return fail(DSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* msg = validate(p)) return fail(DSM_EINVAL, msg);
    if (!dev_buf) return fail(DSM_EINVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf) % kAlign) return fail(DSM_EINVAL, "dev_buf must be 256-byte aligned");
    const Layout L = make_layout(p);
    if (dev_bytes < L.total)
        return fail(DSM_ENOMEM, "device buffer too small: need " + std::to_string(L.total) + " bytes");
    dsm_sim* s = new (std::nothrow) dsm_sim();
    if (!s) return fail(DSM_EINVAL, "host allocation failed");
    s->p = *p;
    s->Q = lattice_q(p->dim);
    s->N = (long long)p->nx * p->ny * p->nz;
    s->stream = (hipStream_t)stream;
    s->half = p->storage == DSM_STORAGE_FP16 ? 1 : 0;
    s->es = s->half ? 2 : 4;
    {
        const int XP = row_pitch(p->nx, s->es);
        const long long NP = (long long)XP * (s->N / p->nx);
        if (p->dim == 2)
            s->geom = Geom{p->nx, 1, p->ny, s->N, XP, NP};
        else
            s->geom = Geom{p->nx, p->ny, p->nz, s->N, XP, NP};
    }
    char* base = (char*)dev_buf;
    for (int k = 0; k < 2; ++k) {
        s->d.f[k] = base + L.off_f[k];
        s->d.g[k] = base + L.off_g[k];
    }
    s->d.c1 = (float*)(base + L.off_c1);
    s->d.mask = (uint8_t*)(base + L.off_mask);
    s->d.phi = (float*)(base + L.off_phi);
    s->d.mu = (float*)(base + L.off_mu);
    s->d.aux = (float*)(base + L.off_aux);
    s->d.partials = (double*)(base + L.off_part);
    s->d.red = (double*)(base + L.off_red);
    s->d.flag = (int*)(base + L.off_flag);
    s->d.ent = (int2*)(base + L.off_ent);
    s->d.links = (LinkRec*)(base + L.off_links);
    s->d.nlinks = (int*)(base + L.off_nlinks);
    s->nlinks = 0;
    s->cur = 0;
    s->pull = 0;
    s->stage = 0;
    s->steps = 0;
    s->beta = s->omega = 0.0;
    s->tau_s = 1.0;
    s->taug_s = 1.0;
    s->tile_variant = p->dim == 3 ? 2 : 0;
    // FP16 3D tiles run two per CU (see the tile kernels' occupancy), so
    // shorter marches keep twice as many tiles in flight
    s->tile_planes = p->dim == 3 && s->half ? 8 : 16;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    if (cus > 0) {
        const int slots = cus * fused_blocks_per_cu(p->dim, s->tile_variant, s->half, make_phys(s, 2).contrast);
        s->tile_planes = default_planes(s->geom, p->dim, slots);
        default_tiling_by_model(s, cus);
    }
    auto cleanup = [&](int rc) {
        delete s;
        return rc;
    };
    const size_t N = (size_t)s->N;
    // every byte of the buffer starts at zero (padding and unused slots are
    // never written later, so state images depend only on the inputs); with
    // no mask that is already S empty and C1 = 0
    hipError_t e = hipMemsetAsync(dev_buf, 0, L.total, s->stream);
    std::vector<uint8_t> m;
    if (mask) {
        m.resize(N);
        for (size_t n = 0; n < N; ++n) m[n] = mask[n] ? 1 : 0;
        if (e == hipSuccess) e = hipMemcpyAsync(s->d.mask, m.data(), N, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = launch_c1_from_mask(s->d.mask, s->d.c1, s->N, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return cleanup(fail(DSM_EDEVICE, std::string("dsm_create: ") + hipGetErrorString(e)));
    // The sharp solid is a solid of the fluid stage like any other: a liquid
    // may be set on it at once, and its cut links (wall fractions from
    // C1 = 1[S]) are then those the split kernels evaluate on the fly.  A
    // mask with more cut links than the table holds needs a solid stage (or
    // a solid field) before a liquid.
    if (mask) {
        const int rc = build_links(s);
        if (rc == DSM_EDEVICE) return cleanup(rc);
        s->solid_failed = rc != DSM_OK;
    }
    *out = s;
    return DSM_OK;
}

int dsm_init_solid(dsm_sim* s, int n_steps, double beta, double omega, double tau_s, double mobility_s,
                   int flags) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (n_steps < 0) return fail(DSM_EINVAL, "n_steps must be >= 0");
    if (!(beta >= 0.0) || !(omega >= 0.0) || !isfinite(beta) || !isfinite(omega))
        return fail(DSM_EINVAL, "beta and omega must be finite and >= 0");
    if (!(tau_s > 0.5) || !(mobility_s > 0.0)) return fail(DSM_EINVAL, "tau_s must be > 1/2, mobility_s > 0");
    if (flags & ~(DSM_SOLID_RESET | DSM_SOLID_REMASK)) return fail(DSM_EINVAL, "unknown flags");
    s->beta = beta;
    s->omega = omega;
    s->tau_s = tau_s;
    s->taug_s = 0.5 + 3.0 * mobility_s;
    // The cut links of the previous C1 must not outlive it, and a stability
    // flag left by an earlier run must not be taken for this run's.
    s->nlinks = 0;
    s->solid_failed = 1;
    HIP_TRY(hipMemsetAsync(s->d.flag, 0, 4 * sizeof(int), s->stream));
    if ((flags & DSM_SOLID_RESET) || s->stage != 1) {
        s->stage = 1;
        HIP_TRY(launch_c1_from_mask(s->d.mask, s->d.phi, s->N, s->stream));
        int rc = init_populations(s, 1);
        if (rc) return rc;
    }
    for (int t = 0; t < n_steps; ++t) {
        int rc = one_step(s);
        if (rc) return rc;
    }
    // freeze C1 = sum of the solid-stage g
    HIP_TRY(launch_moment(s->p.dim, s->geom, PG(s, s->cur), s->d.c1, s->pull, s->stream));
    if (flags & DSM_SOLID_REMASK) HIP_TRY(launch_remask(s->d.c1, s->d.mask, s->N, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    int rc = check_flag(s);
    if (!rc) rc = build_links(s);
    if (!rc) s->solid_failed = 0;
    return rc;
}

int dsm_set_solid_field(dsm_sim* s, const double* C1) {
    if (!s || !C1) return fail(DSM_EINVAL, "NULL argument");
    s->nlinks = 0;
    s->solid_failed = 1;
    int rc = upload_field(s, C1, s->d.c1);
    if (rc) return rc;
    s->stage = 0;
    rc = build_links(s);
    if (!rc) s->solid_failed = 0;
    return rc;
}

int dsm_set_liquid(dsm_sim* s, const double* C2) {
    if (!s || !C2) return fail(DSM_EINVAL, "NULL argument");
    if (s->solid_failed)
        return fail(DSM_ESTATE, "the last solid stage or solid field failed; set the solid again first");
    int rc = upload_field(s, C2, s->d.phi);
    if (rc) return rc;
    s->stage = 2;
    s->steps = 0;
    HIP_TRY(hipMemsetAsync(s->d.flag, 0, 4 * sizeof(int), s->stream));
    return init_populations(s, 2);
}

int dsm_set_gravity(dsm_sim* s, const double g[3]) {
    if (!s || !g) return fail(DSM_EINVAL, "NULL argument");
    for (int k = 0; k < 3; ++k)
        if (!isfinite(g[k])) return fail(DSM_EINVAL, "gravity must be finite");
    if (s->p.dim == 2 && g[2] != 0.0) return fail(DSM_EINVAL, "gravity[2] must be 0 when dim == 2");
    for (int k = 0; k < 3; ++k) s->p.gravity[k] = g[k];
    return DSM_OK;
}

int dsm_step(dsm_sim* s, int n) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (n < 0) return fail(DSM_EINVAL, "n must be >= 0");
    if (s->stage != 2) return fail(DSM_ESTATE, "dsm_step needs a liquid (dsm_set_liquid) first");
    for (int t = 0; t < n; ++t) {
        int rc = one_step(s);
        if (rc) return rc;
        ++s->steps;
        if (s->p.reduce_every > 0 && s->steps % s->p.reduce_every == 0) {
            rc = check_flag(s);
            if (rc) return rc;
        }
    }
    return DSM_OK;
}

int dsm_step_timed(dsm_sim* s, int n, double* step_ms, double* links_ms) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (n < 1) return fail(DSM_EINVAL, "n must be >= 1");
    if (s->stage != 2) return fail(DSM_ESTATE, "dsm_step_timed needs a liquid (dsm_set_liquid) first");
    if (s->p.kernel != DSM_KERNEL_FUSED) return fail(DSM_EINVAL, "dsm_step_timed times the fused kernel only");
    std::vector<hipEvent_t> ev((size_t)4 * n, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto& e : ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            destroy();
            return fail(DSM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(r));
        }
    }
    int rc = DSM_OK;
    for (int t = 0; t < n && !rc; ++t) {
        const Phys ph = make_phys(s, s->stage);
        const int c = s->cur, o = 1 - s->cur;
        hipError_t r = hipEventRecord(ev[4 * t], s->stream);
        if (r == hipSuccess && s->pull) r = launch_bounce(PF(s, c), s->d.links, s->nlinks, s->stream);
        if (r == hipSuccess) r = hipEventRecord(ev[4 * t + 1], s->stream);
        if (r == hipSuccess) r = hipEventRecord(ev[4 * t + 2], s->stream);
        if (r == hipSuccess)
            r = launch_step_fused(s->p.dim, s->geom, ph, PF(s, c), PG(s, c), PF(s, o), PG(s, o), s->d.c1,
                                  s->d.mask, s->pull, s->d.flag, s->tile_variant, s->tile_planes, s->stream);
        if (r == hipSuccess) r = hipEventRecord(ev[4 * t + 3], s->stream);
        if (r != hipSuccess) {
            rc = fail(DSM_EDEVICE, std::string("dsm_step_timed: ") + hipGetErrorString(r));
            break;
        }
        s->cur = o;
        s->pull = 1;
        ++s->steps;
    }
    double sum_step = 0.0, sum_links = 0.0;
    if (!rc) {
        hipError_t r = hipStreamSynchronize(s->stream);
        for (int t = 0; t < n && r == hipSuccess; ++t) {
            float a = 0.f, b = 0.f;
            r = hipEventElapsedTime(&a, ev[4 * t], ev[4 * t + 1]);
            if (r == hipSuccess) r = hipEventElapsedTime(&b, ev[4 * t + 2], ev[4 * t + 3]);
            sum_links += a;
            sum_step += b;
        }
        if (r != hipSuccess) rc = fail(DSM_EDEVICE, std::string("dsm_step_timed: ") + hipGetErrorString(r));
    }
    destroy();
    if (rc) return rc;
    if (step_ms) *step_ms = sum_step / n;
    if (links_ms) *links_ms = sum_links / n;
    return check_flag(s);
}

int dsm_free_energy(dsm_sim* s, double* F, double* E_kin) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    double r[RED_SLOTS];
    int rc = reduce(s, r);
    if (rc) return rc;
    if (F) *F = r[RED_FREE];
    if (E_kin) *E_kin = r[RED_EKIN];
    return DSM_OK;
}

int dsm_mass(dsm_sim* s, double m[3]) {
    if (!s || !m) return fail(DSM_EINVAL, "NULL argument");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    double r[RED_SLOTS];
    int rc = reduce(s, r);
    if (rc) return rc;
    m[0] = r[RED_C1];
    m[1] = r[RED_C2];
    m[2] = r[RED_C3];
    return DSM_OK;
}

int dsm_solid_region(dsm_sim* s, uint8_t* mask) {
    if (!s || !mask) return fail(DSM_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(mask, s->d.mask, (size_t)s->N, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return DSM_OK;
}

int dsm_diagnostics(dsm_sim* s, dsm_diag* out) {
    if (!s || !out) return fail(DSM_EINVAL, "NULL argument");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    double r[RED_SLOTS];
    int rc = reduce(s, r);
    if (rc) return rc;
    out->mass[0] = r[RED_C1];
    out->mass[1] = r[RED_C2];
    out->mass[2] = r[RED_C3];
    out->free_energy = r[RED_FREE];
    out->kinetic_energy = r[RED_EKIN];
    out->max_speed = r[RED_UMAX];
    out->nonfinite_nodes = r[RED_NONFINITE];
    return DSM_OK;
}

int dsm_fields(dsm_sim* s, double* C1, double* C2, double* C3, double* u, double* p) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    // only what is asked for: the velocity and pressure kernels run when u or
    // p is requested, and each concentration plane is copied when an output
    // needs it (C3 needs both)
    int rc = DSM_OK;
    if (u || p) {
        rc = observe(s);
    } else {
        const hipError_t e = launch_moment(s->p.dim, s->geom, PG(s, s->cur), s->d.phi, s->pull, s->stream);
        if (e != hipSuccess) rc = fail(DSM_EDEVICE, std::string("dsm_fields: ") + hipGetErrorString(e));
    }
    if (rc) return rc;
    const size_t N = (size_t)s->N;
    const bool fluid = s->stage == 2;
    const bool need_c1 = C1 || C3, need_phi = fluid && (C2 || C3);
    std::vector<double> c1(need_c1 ? N : 0), phi(need_phi ? N : 0);
    if (need_c1) {
        rc = download_field(s, fluid ? s->d.c1 : s->d.phi, c1.data(), N);
        if (rc) return rc;
    }
    if (need_phi) {
        rc = download_field(s, s->d.phi, phi.data(), N);
        if (rc) return rc;
    }
    for (size_t n = 0; n < N; ++n) {
        const double a = need_c1 ? c1[n] : 0.0, b = need_phi ? phi[n] : 0.0;
        if (C1) C1[n] = a;
        if (C2) C2[n] = b;
        if (C3) C3[n] = 1.0 - a - b;
    }
    if (u) {
        rc = download_field(s, s->d.aux, u, (size_t)s->p.dim * N);
        if (rc) return rc;
    }
    if (p) {
        rc = download_field(s, s->d.aux + 3 * N, p, N);
        if (rc) return rc;
    }
    return DSM_OK;
}

int dsm_chemical_potential(dsm_sim* s, double* mu) {
    if (!s || !mu) return fail(DSM_EINVAL, "NULL argument");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    int rc = observe(s);
    if (rc) return rc;
    return download_field(s, s->d.mu, mu, (size_t)s->N);
}

int dsm_get_populations(dsm_sim* s, double* f, double* g) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    const void* fs = s->d.f[s->cur];
    const void* gs = s->d.g[s->cur];
    if (s->pull) {
        const Phys ph = make_phys(s, s->stage);
        const int o = 1 - s->cur;  // the spare pair is free between steps
        HIP_TRY(launch_pull_state(s->p.dim, s->geom, ph, PF(s, s->cur), PG(s, s->cur), s->d.c1, PF(s, o),
                                  PG(s, o), s->stream));
        fs = s->d.f[o];
        gs = s->d.g[o];
    }
    int rc = DSM_OK;
    if (f) rc = download_pops(s, fs, f, false);
    if (!rc && g) rc = download_pops(s, gs, g, true);
    return rc;
}

static int upload_pops(dsm_sim* s, const double* f, const double* g, int pair) {
    // a fluid state needs the cut links of a solid that was set successfully
    // (a failed solid stage leaves the handle in the solid stage)
    if (s->solid_failed && s->stage != 1)
        return fail(DSM_ESTATE, "the last solid stage or solid field failed; set the solid again first");
    int rc = upload_pops_one(s, f, s->d.f[pair], false);
    if (!rc) rc = upload_pops_one(s, g, s->d.g[pair], true);
    if (!rc) rc = clear_spare_f(s, 1 - pair);
    return rc;
}

int dsm_set_populations(dsm_sim* s, const double* f, const double* g) {
    if (!s || !f || !g) return fail(DSM_EINVAL, "NULL argument");
    int rc = upload_pops(s, f, g, 0);
    if (rc) return rc;
    if (s->stage == 0) s->stage = 2;
    s->cur = 0;
    s->pull = 0;
    return DSM_OK;
}

int dsm_set_postcollision(dsm_sim* s, const double* fs, const double* gs) {
    if (!s || !fs || !gs) return fail(DSM_EINVAL, "NULL argument");
    int rc = upload_pops(s, fs, gs, 0);
    if (rc) return rc;
    if (s->stage == 0) s->stage = 2;
    s->cur = 0;
    s->pull = 1;
    return DSM_OK;
}

size_t dsm_state_bytes(const dsm_sim* s) {
    if (!s) return 0;
    const size_t N = (size_t)s->N;
    return sizeof(StateHeader) + f_bytes(s) + g_bytes(s) + N * sizeof(float) + N;
}

int dsm_get_state(dsm_sim* s, void* host, size_t bytes) {
    if (!s || !host) return fail(DSM_EINVAL, "NULL argument");
    if (bytes != dsm_state_bytes(s)) return fail(DSM_EINVAL, "state size mismatch");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    StateHeader h;
    memset(&h, 0, sizeof(h));
    h.magic = kStateMagic;
    h.version = 3;  // 3: population and rest-plane rows padded to the row pitch
    h.dim = s->p.dim;
    h.nx = s->p.nx;
    h.ny = s->p.ny;
    h.nz = s->p.nz;
    h.stage = s->stage;
    h.pull = s->pull;
    h.steps = s->steps;
    for (int k = 0; k < 3; ++k) h.gravity[k] = s->p.gravity[k];
    h.beta = s->beta;
    h.omega = s->omega;
    h.tau_s = s->tau_s;
    h.taug_s = s->taug_s;
    char* o = (char*)host;
    memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    const size_t N = (size_t)s->N;
    HIP_TRY(hipMemcpyAsync(o, s->d.f[s->cur], f_bytes(s), hipMemcpyDeviceToHost, s->stream));
    o += f_bytes(s);
    HIP_TRY(hipMemcpyAsync(o, s->d.g[s->cur], g_bytes(s), hipMemcpyDeviceToHost, s->stream));
    o += g_bytes(s);
    HIP_TRY(hipMemcpyAsync(o, s->d.c1, N * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    o += N * sizeof(float);
    HIP_TRY(hipMemcpyAsync(o, s->d.mask, N, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return DSM_OK;
}

int dsm_set_state(dsm_sim* s, const void* host, size_t bytes) {
    if (!s || !host) return fail(DSM_EINVAL, "NULL argument");
    if (bytes != dsm_state_bytes(s)) return fail(DSM_EINVAL, "state size mismatch");
    StateHeader h;
    memcpy(&h, host, sizeof(h));
    if (h.magic != kStateMagic || h.version != 3) return fail(DSM_EINVAL, "not a dsm state image (or an older format)");
    if (h.dim != s->p.dim || h.nx != s->p.nx || h.ny != s->p.ny || h.nz != s->p.nz)
        return fail(DSM_EINVAL, "state image is for another lattice");
    if (h.stage != 1 && h.stage != 2) return fail(DSM_EINVAL, "state image has no live stage");
    const char* o = (const char*)host + sizeof(h);
    const size_t N = (size_t)s->N;
    HIP_TRY(hipMemcpyAsync(s->d.f[0], o, f_bytes(s), hipMemcpyHostToDevice, s->stream));
    o += f_bytes(s);
    HIP_TRY(hipMemcpyAsync(s->d.g[0], o, g_bytes(s), hipMemcpyHostToDevice, s->stream));
    o += g_bytes(s);
    HIP_TRY(hipMemcpyAsync(s->d.c1, o, N * sizeof(float), hipMemcpyHostToDevice, s->stream));
    o += N * sizeof(float);
    HIP_TRY(hipMemcpyAsync(s->d.mask, o, N, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemsetAsync(s->d.flag, 0, 4 * sizeof(int), s->stream));
    HIP_TRY(hipMemsetAsync(s->d.f[1], 0, f_bytes(s), s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->cur = 0;
    s->pull = h.pull;
    s->stage = h.stage;
    s->steps = h.steps;
    for (int k = 0; k < 3; ++k) s->p.gravity[k] = h.gravity[k];
    s->beta = h.beta;
    s->omega = h.omega;
    s->tau_s = h.tau_s;
    s->taug_s = h.taug_s;
    s->solid_failed = 1;
    int rc = build_links(s);
    if (!rc) s->solid_failed = 0;
    return rc;
}

long long dsm_step_count(const dsm_sim* s) { return s ? s->steps : -1; }

int dsm_set_tiling(dsm_sim* s, int variant, int planes) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (variant < 0 || variant >= fused_tile_variants(s->p.dim))
        return fail(DSM_EINVAL, "unknown tile variant");
    if (planes < 1 || planes > 4096) return fail(DSM_EINVAL, "planes must be in [1, 4096]");
    s->tile_variant = variant;
    s->tile_planes = planes;
    return DSM_OK;
}

int dsm_get_tiling(const dsm_sim* s, int* variant, int* planes) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (variant) *variant = s->tile_variant;
    if (planes) *planes = s->tile_planes;
    return DSM_OK;
}

int dsm_tiling_variants(int dim) { return (dim == 2 || dim == 3) ? fused_tile_variants(dim) : 0; }

int dsm_tune_tiling(dsm_sim* s, int reps, double* ms_per_step) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    if (reps < 1 || reps > 1000) return fail(DSM_EINVAL, "reps must be in [1, 1000]");
    if (s->stage != 2) return fail(DSM_ESTATE, "dsm_tune_tiling needs a liquid (dsm_set_liquid) first");
    if (s->p.kernel != DSM_KERNEL_FUSED) return fail(DSM_EINVAL, "dsm_tune_tiling tunes the fused kernel only");
    static const int kPlanes3[] = {2, 4, 8, 16, 32, 48, 64, 96, 128};
    static const int kPlanes2[] = {1, 2, 4, 8, 16, 32, 64, 128};
    const int dim = s->p.dim, Z = s->geom.Z;
    const int* list = dim == 3 ? kPlanes3 : kPlanes2;
    const int count = dim == 3 ? (int)(sizeof(kPlanes3) / sizeof(int)) : (int)(sizeof(kPlanes2) / sizeof(int));
    const int v0 = s->tile_variant, p0 = s->tile_planes;
    int bv = v0, bp = p0;
    double best = 1e300;
    for (int v = 0; v < fused_tile_variants(dim); ++v)
        for (int k = 0; k < count; ++k) {
            // marches of at least Z planes are one and the same launch: time the first only
            if (k > 0 && list[k - 1] >= Z) break;
            s->tile_variant = v;
            s->tile_planes = list[k];
            int rc = dsm_step(s, 1);
            double ms = 0.0;
            if (!rc) rc = dsm_step_timed(s, reps, &ms, nullptr);
            if (rc) {
                s->tile_variant = v0;
                s->tile_planes = p0;
                return rc;
            }
            if (ms < best) {
                best = ms;
                bv = v;
                bp = list[k];
            }
        }
    s->tile_variant = bv;
    s->tile_planes = bp;
    if (ms_per_step) *ms_per_step = best;
    return DSM_OK;
}

int dsm_destroy(dsm_sim* s) {
    if (!s) return fail(DSM_EINVAL, "sim is NULL");
    hipError_t e = hipStreamSynchronize(s->stream);
    delete s;
    if (e != hipSuccess) return fail(DSM_EDEVICE, std::string("dsm_destroy: ") + hipGetErrorString(e));
    return DSM_OK;
}

const char* dsm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---- Diagnostics without device allocation --------------------------------
//
// dsm_diagnostics_noalloc runs the same two reduction kernels as
// dsm_diagnostics, with the same grid, so its sums are bit-identical, but
// takes their workspace (one row of RED_SLOTS FP64 partial sums per reduction
// block, then the RED_SLOTS final values) from `scratch` below instead of the
// handle's buffer.  `scratch` is a file-scope device array: each GPU the
// library runs on holds its own copy, with the code object, until the process
// ends.  Host code never uses the array's name as an address; it uses the
// device address hipGetSymbolAddress returns, looked up once per device with
// that device current.  Every block writes its whole row and the final kernel
// reads only the rows of this call, so nothing has to start at zero; two calls
// that overlap on one GPU share the array and race.

namespace {

// The reduction grid never exceeds kReduceBlocks blocks, whatever the
// lattice, so this fixed workspace (65 600 bytes) fits every handle.
constexpr int kNoAllocPartials = kReduceBlocks;
constexpr size_t kNoAllocDoubles = (size_t)(kNoAllocPartials + 1) * RED_SLOTS;
constexpr int kMaxDevices = 64;
static_assert(kNoAllocPartials >= kReduceBlocks, "workspace must hold a partial row per reduction block");

}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device that runs `stream`.
int scratch_address(hipStream_t stream, double** out) {
    int dev = 0;
    if (stream) {
        hipDevice_t d = 0;
        HIP_TRY(hipStreamGetDevice(stream, &d));
        dev = (int)d;
    } else {
        HIP_TRY(hipGetDevice(&dev));
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(DSM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess)
            return fail(DSM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return DSM_OK;
}

}  // namespace

int dsm_diagnostics_noalloc(dsm_sim* s, dsm_diag* out) {
    if (!s || !out) return fail(DSM_EINVAL, "NULL argument");
    if (s->stage == 0) return fail(DSM_ESTATE, "no live state");
    double* ws = nullptr;
    int rc = scratch_address(s->stream, &ws);
    if (rc) return rc;
    rc = observe(s);
    if (rc) return rc;
    double* partials = ws;
    double* red = ws + (size_t)kNoAllocPartials * RED_SLOTS;
    const Phys ph = make_phys(s, s->stage);
    HIP_TRY(launch_reduce(s->p.dim, s->geom, ph, s->d.c1, s->d.phi, s->d.mask, s->d.aux, PG(s, s->cur), s->pull,
                          partials, red, s->stream));
    double r[RED_SLOTS];
    HIP_TRY(hipMemcpyAsync(r, red, sizeof(r), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    out->mass[0] = r[RED_C1];
    out->mass[1] = r[RED_C2];
    out->mass[2] = r[RED_C3];
    out->free_energy = r[RED_FREE];
    out->kinetic_energy = r[RED_EKIN];
    out->max_speed = r[RED_UMAX];
    out->nonfinite_nodes = r[RED_NONFINITE];
    return DSM_OK;
}
