// dsm_batch.hip -- batched form of the fluid-stage step (include/dsm.h).
//
// Many independent lattices advance together.  One step of the batch is
//   1. k_bounce_batch: the interpolated bounce-back of every member (runs of
//      kBatchChunk cut links), which also resets the work counters;
//   2. per lattice type present (2D, 3D): one persistent k_step_batch launch
//      whose workgroups take (member, tile) items from a counter.
// The launches of one and of two steps are captured in HIP graphs on a
// private stream and replayed on the caller's stream.  Member descriptors are
// rebuilt on the host before every batch call, with buffer pair 0 of each
// descriptor the member's live pair, so a member may also be used on its own
// between batch calls.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "dsm_host.h"

using namespace dsm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxPlanes = 4096;
constexpr int kGroups = 4;        // (2D, 3D) x (uniform fluid, density/viscosity contrast)
constexpr int kNumCounters = kGroups;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(DSM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int type_index(int dim) { return dim == 2 ? 0 : 1; }
int contrast_of(const dsm_sim* s) { return sim_phys(s, 2).contrast; }
// Work group of a member: lattice type and contrast variant of the kernel.
int group_of(const dsm_sim* s) { return 2 * type_index(s->p.dim) + contrast_of(s); }
int group_dim(int t) { return t < 2 ? 2 : 3; }

// Smallest tile of each lattice type (bounds the work list for any schedule).
void min_tile(int dim, int* tx, int* ty) {
    int bx = 1 << 30, by = 1 << 30;
    for (int v = 0; v < fused_tile_variants(dim); ++v) {
        int x = 0, y = 0;
        fused_tile_shape(dim, v, &x, &y);
        bx = std::min(bx, x);
        by = std::min(by, y);
    }
    *tx = bx;
    *ty = by;
}

struct Caps {
    size_t items[kGroups];
    size_t chunks;
};

// Checks the members; returns an error message or nullptr.
const char* check_members(dsm_sim* const* sims, int count) {
    if (!sims) return "sims is NULL";
    if (count < 1) return "count must be >= 1";
    for (int k = 0; k < count; ++k)
        if (!sims[k]) return "a member is NULL";
    std::vector<dsm_sim*> v(sims, sims + count);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end()) return "a lattice appears twice";
    for (int k = 1; k < count; ++k)
        if (sims[k]->half != sims[0]->half) return "members must share one population storage";
    return nullptr;
}

Caps member_caps(dsm_sim* const* sims, int count) {
    Caps c{{0, 0, 0, 0}, 0};
    for (int k = 0; k < count; ++k) {
        const dsm_sim* s = sims[k];
        int tx = 0, ty = 0;
        min_tile(s->p.dim, &tx, &ty);
        const Geom& g = s->geom;
        c.items[group_of(s)] +=
            (size_t)((g.X + tx - 1) / tx) * (size_t)((g.Y + ty - 1) / ty) * (size_t)g.Z;
        c.chunks += (size_t)((kLinksPerNode * s->N + kBatchChunk - 1) / kBatchChunk);
    }
    return c;
}

struct Offsets {
    size_t inst, items[kGroups], chunks, counters, flags, total;
};

Offsets make_offsets(int count, const Caps& c) {
    Offsets o;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at = align_up(at + bytes);
        return r;
    };
    o.inst = take((size_t)count * sizeof(BatchInst));
    for (int k = 0; k < kGroups; ++k) o.items[k] = take(c.items[k] * sizeof(BatchItem));
    o.chunks = take(c.chunks * sizeof(BatchChunk));
    o.counters = take(kNumCounters * sizeof(int));
    o.flags = take((size_t)count * sizeof(int));
    o.total = at;
    return o;
}

}  // namespace

struct dsm_batch {
    std::vector<dsm_sim*> sims;
    hipStream_t stream = nullptr;  // the caller's stream
    hipStream_t cap = nullptr;     // private stream for graph capture
    int half = 0;
    int cus = 1;
    Caps caps{};
    BatchInst* inst_dev = nullptr;
    BatchItem* items_dev[kGroups] = {nullptr, nullptr, nullptr, nullptr};
    BatchChunk* chunks_dev = nullptr;
    int* counters = nullptr;
    int* flags_dev = nullptr;
    bool present[kGroups] = {false, false, false, false};
    dsm_batch_schedule sched[2]{};  // by lattice type (2D, 3D)
    int nitems[kGroups] = {0, 0, 0, 0};
    int nchunks = 0;
    std::vector<BatchInst> inst_host, inst_sent;
    std::vector<BatchChunk> chunks_host, chunks_sent;
    std::vector<BatchItem> items_host;
    std::vector<int> flags_host;
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // one step, two steps
};

namespace {

void drop_graphs(dsm_batch* b) {
    for (auto& e : b->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

int grid_of(const dsm_batch* b, int t) {
    const dsm_batch_schedule& s = b->sched[t >> 1];
    const int per_cu =
        s.blocks_per_cu > 0 ? s.blocks_per_cu : batch_blocks_per_cu(group_dim(t), s.variant, b->half, t & 1);
    return std::max(1, per_cu) * b->cus;
}

// Work list of group t for its schedule: every tile of every member of the
// group, costliest (most planes) first, members in order otherwise.
int build_items(dsm_batch* b, int t) {
    const int dim = group_dim(t);
    const dsm_batch_schedule& s = b->sched[t >> 1];
    int tx = 0, ty = 0;
    fused_tile_shape(dim, s.variant, &tx, &ty);
    auto& it = b->items_host;
    it.clear();
    for (int k = 0; k < (int)b->sims.size(); ++k) {
        const dsm_sim* m = b->sims[k];
        if (group_of(m) != t) continue;
        const Geom& g = m->geom;
        for (int z0 = 0; z0 < g.Z; z0 += s.planes)
            for (int y0 = 0; y0 < g.Y; y0 += ty)
                for (int x0 = 0; x0 < g.X; x0 += tx) it.push_back(BatchItem{k, x0, y0, z0});
    }
    std::stable_sort(it.begin(), it.end(), [&](const BatchItem& a, const BatchItem& c) {
        const int za = std::min(s.planes, b->sims[a.inst]->geom.Z - a.z0);
        const int zc = std::min(s.planes, b->sims[c.inst]->geom.Z - c.z0);
        return za > zc;
    });
    if (it.size() > b->caps.items[t] || it.size() > (size_t)0x7fffffff)
        return set_error(DSM_EINVAL, "work list exceeds its table");
    b->nitems[t] = (int)it.size();
    if (!it.empty())
        HIP_TRY(hipMemcpyAsync(b->items_dev[t], it.data(), it.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                               b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return DSM_OK;
}

// Descriptors and link runs from the members' current state; uploads what
// changed.  Fails if a member is not stepping the fluid stage.
int refresh(dsm_batch* b) {
    const int count = (int)b->sims.size();
    b->inst_host.resize(count);
    b->chunks_host.clear();
    for (int k = 0; k < count; ++k) {
        dsm_sim* s = b->sims[k];
        if (s->stage != 2 || !s->pull)
            return set_error(DSM_ESTATE, "batch member " + std::to_string(k) +
                                             " must be in the fluid stage with at least one step taken");
        // field by field over a zeroed record, so that padding bytes compare
        // equal between calls
        BatchInst& d = b->inst_host[k];
        memset(&d, 0, sizeof(d));
        d.geom.X = s->geom.X;
        d.geom.Y = s->geom.Y;
        d.geom.Z = s->geom.Z;
        d.geom.N = s->geom.N;
        d.geom.XP = s->geom.XP;
        d.geom.NP = s->geom.NP;
        d.phys = sim_phys(s, 2);
        d.f[0] = s->d.f[s->cur];
        d.f[1] = s->d.f[1 - s->cur];
        d.g[0] = s->d.g[s->cur];
        d.g[1] = s->d.g[1 - s->cur];
        d.c1 = s->d.c1;
        d.mask = s->d.mask;
        d.flag = s->d.flag;
        d.links = s->d.links;
        d.nlinks = s->nlinks;
        d.half = s->half;
        for (int r = 0; r < s->nlinks; r += kBatchChunk) b->chunks_host.push_back(BatchChunk{k, r});
    }
    if (b->chunks_host.size() > b->caps.chunks) return set_error(DSM_EINVAL, "link runs exceed their table");
    const bool inst_same = b->inst_sent.size() == b->inst_host.size() &&
                           !memcmp(b->inst_sent.data(), b->inst_host.data(), count * sizeof(BatchInst));
    const bool chunks_same = b->chunks_sent.size() == b->chunks_host.size() &&
                             (b->chunks_host.empty() || !memcmp(b->chunks_sent.data(), b->chunks_host.data(),
                                                                b->chunks_host.size() * sizeof(BatchChunk)));
    if (!inst_same)
        HIP_TRY(hipMemcpyAsync(b->inst_dev, b->inst_host.data(), count * sizeof(BatchInst), hipMemcpyHostToDevice,
                               b->stream));
    if (!chunks_same) {
        if (!b->chunks_host.empty())
            HIP_TRY(hipMemcpyAsync(b->chunks_dev, b->chunks_host.data(), b->chunks_host.size() * sizeof(BatchChunk),
                                   hipMemcpyHostToDevice, b->stream));
        if ((int)b->chunks_host.size() != b->nchunks) drop_graphs(b);  // the bounce grid changes
        b->nchunks = (int)b->chunks_host.size();
    }
    if (!inst_same || !chunks_same) HIP_TRY(hipStreamSynchronize(b->stream));
    b->inst_sent = b->inst_host;
    b->chunks_sent = b->chunks_host;
    return DSM_OK;
}

// Launches of one step with the given parity on stream st.
hipError_t enqueue_step(dsm_batch* b, int parity, hipStream_t st) {
    hipError_t e = launch_bounce_batch(b->inst_dev, b->chunks_dev, b->nchunks, parity, b->counters, kNumCounters, st);
    for (int t = 0; t < kGroups && e == hipSuccess; ++t)
        if (b->present[t])
            e = launch_step_batch(group_dim(t), b->sched[t >> 1].variant, b->half, t & 1, b->inst_dev,
                                  b->items_dev[t], b->nitems[t], b->counters + t, grid_of(b, t), parity,
                                  b->sched[t >> 1].planes, st);
    return e;
}

int capture(dsm_batch* b) {
    if (b->exec[0] && b->exec[1]) return DSM_OK;
    drop_graphs(b);
    for (int k = 0; k < 2; ++k) {
        HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_step(b, 0, b->cap);
        if (e == hipSuccess && k == 1) e = enqueue_step(b, 1, b->cap);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[k], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            drop_graphs(b);
            return set_error(DSM_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
        }
    }
    return DSM_OK;
}

// n steps as graph replays; members' bookkeeping follows.
int run(dsm_batch* b, int n) {
    for (int k = 0; k + 2 <= n; k += 2) HIP_TRY(hipGraphLaunch(b->exec[1], b->stream));
    if (n & 1) HIP_TRY(hipGraphLaunch(b->exec[0], b->stream));
    for (dsm_sim* s : b->sims) {
        s->cur ^= (n & 1);
        s->steps += n;
    }
    return DSM_OK;
}

int check_flags(dsm_batch* b) {
    const int count = (int)b->sims.size();
    HIP_TRY(launch_batch_flags(b->inst_dev, count, b->flags_dev, b->stream));
    b->flags_host.assign(count, 0);
    HIP_TRY(hipMemcpyAsync(b->flags_host.data(), b->flags_dev, count * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int k = 0; k < count; ++k)
        if (b->flags_host[k])
            return set_error(DSM_EUNSTABLE, "batch member " + std::to_string(k) + " holds non-finite values");
    return DSM_OK;
}

int check_sched(int dim, const dsm_batch_schedule* s) {
    if (!s) return set_error(DSM_EINVAL, "schedule is NULL");
    if (s->variant < 0 || s->variant >= fused_tile_variants(dim)) return set_error(DSM_EINVAL, "unknown tile variant");
    if (s->planes < 1 || s->planes > kMaxPlanes) return set_error(DSM_EINVAL, "planes must be in [1, 4096]");
    if (s->blocks_per_cu < 0 || s->blocks_per_cu > 64) return set_error(DSM_EINVAL, "blocks_per_cu must be in [0, 64]");
    return DSM_OK;
}

// Plane counts the tuner considers.  Four-plane marches pay off in 2D, whose
// fill rows cost nothing measurable: the 512-lattice D2Q9 set steps at 29.4
// GLUPS with 4 against 28.8 with 8; in 3D their fill planes rule them out.
constexpr int kTunePlanes[] = {4, 8, 16, 32, 64, 128};

// Model constants per lattice type (index 0: 2D, 1: 3D), fitted to the
// batched kernel's measured step times on MI355X over every schedule (3 tile
// variants x 5 plane counts) of a 512-lattice D2Q9 set and of a 24-job set of
// the served form's 3D lattices.
// Relative cost of one wave marching one plane, per tile variant (2D:
// 256/128/64 columns; 3D: 64x4/64x8/128x4 columns).
constexpr double kWaveCost[2][3] = {{1.0, 1.16, 1.30}, {1.0, 1.02, 0.89}};
// Cost of each of the two planes an item marches beyond its own (to fill the
// C ring before its first collision), as a share of a full plane: they pull g
// only, mostly from L2, where the neighbouring items of the same lattice have
// just read them; in 3D they also pull the halo rows and columns.
constexpr double kFillShare[2] = {0.0, 0.36};
// Tail of a step: the share of the longest item that outlasts the drained
// queue.
constexpr double kTailShare[2] = {0.0625, 0.095};

// Modelled duration of one batched step of the members of one lattice type
// under a schedule, in units of one wave marching one plane.  A wave costs
// the same whether or not all of its lanes hold lattice columns; each item's
// two fill planes cost kFillShare of a plane each.  The dynamic queue, fed
// costliest item first, keeps every resident wave busy until the list is
// drained, so the step lasts the total work over the resident waves plus a
// tail of kTailShare of the longest item.
// One member's work (wave-planes) and its longest item under a tiling.
void member_work(const Geom& g, int dim, int tx, int ty, int planes, double* total, double* longest) {
    const double waves_per_item = (double)(tx / 64) * ty;
    const double tiles = (double)((g.X + tx - 1) / tx) * (double)((g.Y + ty - 1) / ty);
    const int full = g.Z / planes, tail = g.Z % planes;
    const double fill = 2.0 * kFillShare[dim - 2];
    *total += tiles * waves_per_item * ((double)full * (planes + fill) + (tail ? tail + fill : 0.0));
    *longest = std::max(*longest, (full ? planes : tail) + fill);
}

double schedule_cost(const dsm_batch* b, int dim, int variant, int planes) {
    int tx = 0, ty = 0;
    fused_tile_shape(dim, variant, &tx, &ty);
    const double waves_per_item = (double)(tx / 64) * ty;
    double cost = 0.0;
    for (int t = 2 * type_index(dim); t < 2 * type_index(dim) + 2; ++t) {
        if (!b->present[t]) continue;
        double total = 0.0, longest = 0.0;
        for (const dsm_sim* m : b->sims)
            if (group_of(m) == t) member_work(m->geom, dim, tx, ty, planes, &total, &longest);
        const int per_cu = batch_blocks_per_cu(dim, variant, b->half, t & 1);
        const double resident_waves = (double)b->cus * per_cu * waves_per_item;
        cost += kWaveCost[dim - 2][variant] * (total / resident_waves + kTailShare[dim - 2] * longest);
    }
    return cost;
}

}  // namespace

// Latency-bound form for one lattice whose grid makes a fraction of a round:
// every item marches at once, so the step lasts whole rounds of the longest
// march plus its fill planes.  Rounds are counted against a share of the
// resident workgroups (a full round of 2D items already contends), and tiles
// wider than the lattice row, rounded to whole waves, are charged their idle
// waves.  Constants fitted to small lattices timed over every tile variant
// and march: 22 in 3D (48^3 to 128^3 and two oblong ones, marches of 2 to 32
// planes) and 22 in 2D (128 x 64 to 2048^2, marches of 1 to 32 rows), FP32
// and FP16 each.  With FP16 elements two 3D tiles share a CU and the marches
// of consecutive rounds overlap, so a round holds 1.5 times the resident
// workgroups.
constexpr double kLatencyFill[2] = {0.5, 0.75};   // fill plane, as a share of a plane
constexpr double kLatencySlots[2][2] = {{0.5, 0.5}, {1.0, 1.5}};  // [2D, 3D][FP32, FP16]: workgroups per round
double dsm::lattice_latency_cost(const Geom& g, int dim, int variant, int planes, int blocks_per_cu, int cus,
                                 int half) {
    int tx = 0, ty = 0;
    fused_tile_shape(dim, variant, &tx, &ty);
    const long long tiles_x = (g.X + tx - 1) / tx;
    const long long items = tiles_x * ((g.Y + ty - 1) / ty) * ((g.Z + planes - 1) / planes);
    const double share = kLatencySlots[dim - 2][half ? 1 : 0];
    const double slots = std::max(1.0, share * (double)cus * blocks_per_cu);
    const double rounds = std::ceil((double)items / slots);
    const double idle = (double)(tiles_x * tx) / (double)((g.X + 63) / 64 * 64);
    return kWaveCost[dim - 2][variant] * idle * rounds * (std::min(planes, g.Z) + 2.0 * kLatencyFill[dim - 2]);
}

double dsm::lattice_schedule_cost(const Geom& g, int dim, int variant, int planes, int blocks_per_cu, int cus) {
    int tx = 0, ty = 0;
    fused_tile_shape(dim, variant, &tx, &ty);
    double total = 0.0, longest = 0.0;
    member_work(g, dim, tx, ty, planes, &total, &longest);
    const double resident_waves = (double)cus * blocks_per_cu * (double)(tx / 64) * ty;
    return kWaveCost[dim - 2][variant] * (total / resident_waves + kTailShare[dim - 2] * longest);
}

// Measured tuning: every candidate schedule of each lattice type present
// (tile variant x march planes x resident workgroups per CU) is installed
// and timed on the batch itself through the public calls: one untimed step,
// then reps steps as graph replays between two events, the stream
// synchronised before the next candidate.  The fastest is kept.  Workgroups
// per CU: 0 (as many as fit) and each smaller count up to 4.
static int tune_measured(dsm_batch* b, int reps, double cost[2]) {
    for (int d = 0; d < 2; ++d) {
        if (!b->present[2 * d] && !b->present[2 * d + 1]) continue;
        const int dim = d == 0 ? 2 : 3;
        dsm_batch_schedule best = b->sched[d];
        double best_ms = 1e300;
        for (int v = 0; v < fused_tile_variants(dim); ++v) {
            int fit = 1;  // workgroups per CU the kernels of this type allow
            for (int t = 2 * d; t < 2 * d + 2; ++t)
                if (b->present[t]) fit = std::max(fit, batch_blocks_per_cu(dim, v, b->half, t & 1));
            for (int planes : kTunePlanes)
                for (int per_cu = 0; per_cu <= std::min(fit - 1, 4); ++per_cu) {
                    const dsm_batch_schedule cand{v, planes, per_cu};
                    int rc = dsm_batch_set_schedule(b, dim, &cand);
                    if (!rc) rc = dsm_batch_step(b, 1);
                    double ms = 0.0;
                    if (!rc) rc = dsm_batch_step_timed(b, reps, &ms);
                    if (rc) return rc;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = cand;
                    }
                }
        }
        const int rc = dsm_batch_set_schedule(b, dim, &best);
        if (rc) return rc;
        if (cost) cost[d] = best_ms;
    }
    return DSM_OK;
}

extern "C" {

size_t dsm_batch_required_bytes(dsm_sim* const* sims, int count) {
    if (check_members(sims, count)) return 0;
    return make_offsets(count, member_caps(sims, count)).total;
}

int dsm_batch_create(dsm_sim* const* sims, int count, void* dev_buf, size_t dev_bytes, void* stream,
                     dsm_batch** out) {
    if (!out) return set_error(DSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char* msg = check_members(sims, count)) return set_error(DSM_EINVAL, msg);
    if (!dev_buf) return set_error(DSM_EINVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf) % kAlign) return set_error(DSM_EINVAL, "dev_buf must be 256-byte aligned");
    const Caps caps = member_caps(sims, count);
    const Offsets o = make_offsets(count, caps);
    if (dev_bytes < o.total)
        return set_error(DSM_ENOMEM, "device buffer too small: need " + std::to_string(o.total) + " bytes");
    dsm_batch* b = new (std::nothrow) dsm_batch();
    if (!b) return set_error(DSM_EINVAL, "host allocation failed");
    auto cleanup = [&](int rc) {
        drop_graphs(b);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return rc;
    };
    b->sims.assign(sims, sims + count);
    b->stream = (hipStream_t)stream;
    b->half = sims[0]->half;
    b->caps = caps;
    char* base = (char*)dev_buf;
    b->inst_dev = (BatchInst*)(base + o.inst);
    for (int k = 0; k < kGroups; ++k) b->items_dev[k] = (BatchItem*)(base + o.items[k]);
    b->chunks_dev = (BatchChunk*)(base + o.chunks);
    b->counters = (int*)(base + o.counters);
    b->flags_dev = (int*)(base + o.flags);
    for (dsm_sim* s : b->sims) b->present[group_of(s)] = true;
    b->sched[0] = dsm_batch_schedule{0, 32, 0};
    b->sched[1] = dsm_batch_schedule{2, 16, 0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(dev_buf, 0, o.total, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return cleanup(set_error(DSM_EDEVICE, std::string("dsm_batch_create: ") + hipGetErrorString(e)));
    for (int t = 0; t < kGroups; ++t)
        if (b->present[t]) {
            int rc = build_items(b, t);
            if (rc) return cleanup(rc);
        }
    int rc = refresh(b);
    if (rc) return cleanup(rc);
    *out = b;
    return DSM_OK;
}

int dsm_batch_set_schedule(dsm_batch* b, int dim, const dsm_batch_schedule* sched) {
    if (!b) return set_error(DSM_EINVAL, "batch is NULL");
    if (dim != 2 && dim != 3) return set_error(DSM_EINVAL, "dim must be 2 or 3");
    int rc = check_sched(dim, sched);
    if (rc) return rc;
    const int d = type_index(dim);
    b->sched[d] = *sched;
    for (int t = 2 * d; t < 2 * d + 2; ++t)
        if (b->present[t]) {
            rc = build_items(b, t);
            if (rc) return rc;
        }
    return DSM_OK;
}

int dsm_batch_get_schedule(const dsm_batch* b, int dim, dsm_batch_schedule* sched) {
    if (!b || !sched) return set_error(DSM_EINVAL, "NULL argument");
    if (dim != 2 && dim != 3) return set_error(DSM_EINVAL, "dim must be 2 or 3");
    *sched = b->sched[type_index(dim)];
    return DSM_OK;
}

int dsm_batch_tune(dsm_batch* b, int reps, double cost[2]) {
    if (!b) return set_error(DSM_EINVAL, "batch is NULL");
    if (reps < 0 || reps > 1000) return set_error(DSM_EINVAL, "reps must be in [0, 1000]");
    if (cost) cost[0] = cost[1] = 0.0;
    int rc = refresh(b);
    if (rc) return rc;
    if (reps > 0) return tune_measured(b, reps, cost);
    for (int d = 0; d < 2; ++d) {
        if (!b->present[2 * d] && !b->present[2 * d + 1]) continue;
        const int dim = d == 0 ? 2 : 3;
        dsm_batch_schedule best = b->sched[d];
        double best_cost = 1e300;
        for (int v = 0; v < fused_tile_variants(dim); ++v)
            for (int planes : kTunePlanes) {
                const double c = schedule_cost(b, dim, v, planes);
                if (c < best_cost) {
                    best_cost = c;
                    best = dsm_batch_schedule{v, planes, 0};
                }
            }
        b->sched[d] = best;
        for (int t = 2 * d; t < 2 * d + 2; ++t)
            if (b->present[t]) {
                rc = build_items(b, t);
                if (rc) return rc;
            }
        if (cost) cost[d] = best_cost;
    }
    return DSM_OK;
}

int dsm_batch_step(dsm_batch* b, int n) {
    if (!b) return set_error(DSM_EINVAL, "batch is NULL");
    if (n < 0) return set_error(DSM_EINVAL, "n must be >= 0");
    int rc = refresh(b);
    if (!rc) rc = capture(b);
    if (!rc) rc = run(b, n);
    if (!rc) rc = check_flags(b);
    return rc;
}

int dsm_batch_step_timed(dsm_batch* b, int n, double* ms_per_step) {
    if (!b) return set_error(DSM_EINVAL, "batch is NULL");
    if (n < 1) return set_error(DSM_EINVAL, "n must be >= 1");
    int rc = refresh(b);
    if (!rc) rc = capture(b);
    if (rc) return rc;
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    auto done = [&](int code) {
        for (auto& e : ev) (void)hipEventDestroy(e);
        return code;
    };
    hipError_t e = hipEventRecord(ev[0], b->stream);
    if (e != hipSuccess) return done(set_error(DSM_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e)));
    rc = run(b, n);
    if (rc) return done(rc);
    e = hipEventRecord(ev[1], b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e != hipSuccess) return done(set_error(DSM_EDEVICE, std::string("dsm_batch_step_timed: ") + hipGetErrorString(e)));
    if (ms_per_step) *ms_per_step = ms / n;
    return done(check_flags(b));
}

int dsm_batch_size(const dsm_batch* b) { return b ? (int)b->sims.size() : -1; }

int dsm_batch_items(const dsm_batch* b, int dim) {
    if (!b || (dim != 2 && dim != 3)) return -1;
    int n = 0;
    for (int t = 2 * type_index(dim); t < 2 * type_index(dim) + 2; ++t)
        if (b->present[t]) n += b->nitems[t];
    return n;
}

int dsm_batch_destroy(dsm_batch* b) {
    if (!b) return set_error(DSM_EINVAL, "batch is NULL");
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return DSM_OK;
}

}  // extern "C"
