// C ABI of the QED event generator: argument checks, context and scratch
// management, launch sizing.  All device work is in the kernels of qed_kernels.hip
// (the step), qed_train.hip (the networks and their tables) and qed_grid.hip (grid
// coupling).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/qed.h"
#include "qed_internal.hpp"

using qed::u64;

struct qed_ctx {
    qed_config cfg;
    hipStream_t stream;
    int num_cu;
    qed::DevState *st;        // device
    qed_tuning tune;
    uint8_t *alive;           // photon scratch, sized by photon_cap
    u64 *dead_idx, *hole_idx, *mover_idx;
    u64 photon_cap;
    uint32_t *nsub[2], *queue[2];  // binned-scheduler scratch, sized by lepton_cap
    u64 lepton_cap[2];
    u64 *last_n[3];           // count pointers of the last step (for qed_sync)
    bool prof;                // bracket launches with events
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> rec_id;  // kernel id of each recorded launch
    size_t rec_used;          // event pairs in use
    bool capturing;           // between qed_graph_begin and qed_graph_end
    qed::MlpModel *model;     // surrogate sampler's network (device)
    qed::MlpModel *pair_model;  // the photon path's network of the energy split (device)
    bool have_pair_model;
    uint64_t *gap_hist;       // event-gap diagnostic (caller's device array) and its bins
    uint32_t gap_bins;
    bool have_model;
    qed::CellDev cells;       // sub-steps per cell (cells.n[0] null: per particle)
    uint32_t *cell_buf;       // 2 * cell_cap counts (device)
    u64 cell_cap;
    uint32_t *cell_slot[3];   // per-slot cell of each species, sized by cell_slot_cap
    u64 cell_slot_cap[3];
    std::vector<void *> retired;  // replaced scratch: recorded graphs may still use it
    // tile-sorted deposition: per-slot ranks and records (dep_cap slots), tile counts (zero between calls) and offsets (dep_tiles tiles), the
    // parts' tiles and staged regions (dep_parts parts)
    uint32_t *dep_pos, *dep_count, *dep_off, *dep_part_off, *dep_part_tile;
    qed::DepRecord *dep_rec;
    double *dep_stage;
    u64 dep_cap, dep_tiles, dep_parts;
};

struct qed_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// ---------------------------------------------------------------------------
// Per-slot scratch of qed_step_static: one file-scope device array, resolved to
// a device address once per GPU (qed_init), never allocated at call time.  The
// step's kernels read every entry of these lists only after writing it in the
// same step, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticSlots = QED_STATIC_MAX_SLOTS;
constexpr size_t align256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kOffAlive = 0;                                            // uint8 per photon slot
constexpr size_t kOffDead = align256(kOffAlive + kStaticSlots);            // u64 per photon slot
constexpr size_t kOffHole = align256(kOffDead + 8 * kStaticSlots);
constexpr size_t kOffMover = align256(kOffHole + 8 * kStaticSlots);
constexpr size_t kOffNsub = align256(kOffMover + 8 * kStaticSlots);        // 2 x uint32 per lepton slot
constexpr size_t kOffQueue = align256(kOffNsub + 2 * 4 * kStaticSlots);    // 2 x uint32 per lepton slot
constexpr size_t kOffCell = align256(kOffQueue + 2 * 4 * kStaticSlots);    // 3 x uint32 per slot
constexpr size_t kStaticBytes = align256(kOffCell + 3 * 4 * kStaticSlots);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices];  // device address of scratch on each GPU

// With `dev` current: the device address of this GPU's copy of scratch.
qed_status resolve_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return QED_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return QED_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QED_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    return QED_OK;
}

// Per-slot scratch of one step: the context's buffers or the static array.
struct SlotScratch {
    uint8_t *alive;
    u64 *dead_idx, *hole_idx, *mover_idx;
    uint32_t *nsub[2], *queue[2];
    uint32_t *cell_slot[3];
};

SlotScratch static_scratch(unsigned char *base) {
    SlotScratch x;
    x.alive = base + kOffAlive;
    x.dead_idx = reinterpret_cast<u64 *>(base + kOffDead);
    x.hole_idx = reinterpret_cast<u64 *>(base + kOffHole);
    x.mover_idx = reinterpret_cast<u64 *>(base + kOffMover);
    for (int s = 0; s < 2; ++s) {
        x.nsub[s] = reinterpret_cast<uint32_t *>(base + kOffNsub) + s * kStaticSlots;
        x.queue[s] = reinterpret_cast<uint32_t *>(base + kOffQueue) + s * kStaticSlots;
    }
    for (int s = 0; s < 3; ++s) x.cell_slot[s] = reinterpret_cast<uint32_t *>(base + kOffCell) + s * kStaticSlots;
    return x;
}

}  // namespace

namespace {

#define HIP_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return QED_ERR_HIP;   \
    } while (0)

bool species_ok(const qed_species &s) {
    return s.n && s.x && s.y && s.z && s.ux && s.uy && s.uz && s.w && s.id;
}

bool field_ok(const qed_field &f) {
    return f.ex && f.ey && f.ez && f.bx && f.by && f.bz && (f.stride == 0 || f.stride == 1);
}

qed::SpeciesDev to_dev(const qed_species &s) {
    qed::SpeciesDev d;
    d.n = reinterpret_cast<u64 *>(s.n);
    d.cap = s.capacity;
    d.x = s.x;
    d.y = s.y;
    d.z = s.z;
    d.ux = s.ux;
    d.uy = s.uy;
    d.uz = s.uz;
    d.w = s.w;
    d.id = s.id;
    d.parent = s.parent;
    d.events = s.events;
    d.tau = s.tau;
    d.birth = nullptr;  // set by qed_step when cascades run
    return d;
}

qed::FieldDev to_dev(const qed_field &f) {
    qed::FieldDev d;
    d.ex = f.ex;
    d.ey = f.ey;
    d.ez = f.ez;
    d.bx = f.bx;
    d.by = f.by;
    d.bz = f.bz;
    d.stride = f.stride;
    return d;
}

int grid_for(u64 work, int max_blocks) {
    u64 b = (work + 255) / 256;
    if (b < 1) b = 1;
    if (b > (u64)max_blocks) b = (u64)max_blocks;
    return (int)b;
}

template <class T>
void release(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Scratch that is replaced by a larger buffer stays allocated until qed_finalize: a
// recorded graph keeps the addresses it was recorded with.
template <class T>
void retire(qed_ctx *c, T *&p) {
    if (p) c->retired.push_back(reinterpret_cast<void *>(p));
    p = nullptr;
}

qed_status ensure_photon_scratch(qed_ctx *c, u64 cap) {
    if (cap <= c->photon_cap) return QED_OK;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    retire(c, c->alive);
    retire(c, c->dead_idx);
    retire(c, c->hole_idx);
    retire(c, c->mover_idx);
    c->photon_cap = 0;
    HIP_TRY(hipMalloc(&c->alive, cap));
    HIP_TRY(hipMalloc(&c->dead_idx, cap * sizeof(u64)));
    HIP_TRY(hipMalloc(&c->hole_idx, cap * sizeof(u64)));
    HIP_TRY(hipMalloc(&c->mover_idx, cap * sizeof(u64)));
    c->photon_cap = cap;
    return QED_OK;
}

qed_status ensure_lepton_scratch(qed_ctx *c, int s, u64 cap) {
    if (cap <= c->lepton_cap[s]) return QED_OK;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    retire(c, c->nsub[s]);
    retire(c, c->queue[s]);
    c->lepton_cap[s] = 0;
    HIP_TRY(hipMalloc(&c->nsub[s], cap * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&c->queue[s], cap * sizeof(uint32_t)));
    c->lepton_cap[s] = cap;
    return QED_OK;
}

qed_status ensure_cell_slots(qed_ctx *c, int s, u64 cap) {
    if (cap <= c->cell_slot_cap[s]) return QED_OK;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    retire(c, c->cell_slot[s]);
    c->cell_slot_cap[s] = 0;
    HIP_TRY(hipMalloc(&c->cell_slot[s], cap * sizeof(uint32_t)));
    c->cell_slot_cap[s] = cap;
    return QED_OK;
}

// Scratch of the tile-sorted deposition; false if it cannot be had now (recording a
// graph, or out of memory: the caller then adds per wave).
bool ensure_deposit_scratch(qed_ctx *c, u64 cap, u64 tiles) {
    const u64 parts = qed::dep_max_parts(cap, tiles);
    if (cap <= c->dep_cap && tiles <= c->dep_tiles && parts <= c->dep_parts) return true;
    if (c->capturing) return false;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return false;
    bool ok = true;
    if (cap > c->dep_cap) {
        retire(c, c->dep_pos);
        retire(c, c->dep_rec);
        c->dep_cap = 0;
        ok = hipMalloc(&c->dep_pos, cap * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&c->dep_rec, cap * sizeof(qed::DepRecord)) == hipSuccess;
        if (ok) c->dep_cap = cap;
    }
    if (ok && tiles > c->dep_tiles) {
        retire(c, c->dep_count);
        retire(c, c->dep_off);
        retire(c, c->dep_part_off);
        c->dep_tiles = 0;
        ok = hipMalloc(&c->dep_count, tiles * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&c->dep_off, (tiles + 1) * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&c->dep_part_off, (tiles + 1) * sizeof(uint32_t)) == hipSuccess &&
             hipMemset(c->dep_count, 0, tiles * sizeof(uint32_t)) == hipSuccess;   // the scan keeps it zero
        if (ok) c->dep_tiles = tiles;
    }
    if (ok && parts > c->dep_parts) {
        retire(c, c->dep_part_tile);
        retire(c, c->dep_stage);
        c->dep_parts = 0;
        ok = hipMalloc(&c->dep_part_tile, parts * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&c->dep_stage, parts * qed::kDepStage * sizeof(double)) == hipSuccess;
        if (ok) c->dep_parts = parts;
    }
    if (!ok) (void)hipGetLastError();   // an allocation failure is not kept as the stream's error
    return ok;
}

bool tuning_ok(const qed_tuning &t) {
    return t.lepton_blocks_per_cu >= 1 && t.lepton_blocks_per_cu <= 1024 && t.heavy_blocks_per_cu >= 1 &&
           t.heavy_blocks_per_cu <= 64 && t.photon_blocks_per_cu >= 1 && t.photon_blocks_per_cu <= 1024 &&
           t.chunk >= 64 && t.chunk % 64 == 0 && t.chunk <= (1u << 20) &&
           t.resolve_batch >= 1 && t.resolve_batch <= 64 && t.prepass_finish <= 1 &&
           t.prepass_blocks_per_cu >= 1 && t.prepass_blocks_per_cu <= 1024 && t.scatter_blocks_per_cu >= 1 &&
           t.scatter_blocks_per_cu <= 1024 && t.bins_per_octave >= 4 &&
           t.bins_per_octave <= (uint32_t)qed::kMaxBinsPerOctave && t.light_tile >= 64 && t.light_tile <= 512 &&
           t.light_tile % 64 == 0 && t.tiled_slots >= 64 && t.tiled_slots <= 256 && t.tiled_slots % 64 == 0;
}

const char *kKernelName[qed::K_COUNT] = {"k_begin", "k_photon", "k_lepton", "k_prepass",
                                         "k_scan",  "k_scatter", "k_light", "k_heavy",
                                         "k_end",   "k_fill",   "k_move",  "k_synchrotron", "k_tiled",
                                         "k_gen", "k_photon_surr", "k_cell_clear", "k_cell_max"};

// Event pair for one profiled launch (grown on demand, reused after a read).
bool prof_pair(qed_ctx *c, int id, hipEvent_t *a, hipEvent_t *b) {
    if (2 * (c->rec_used + 1) > c->ev_pool.size()) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            c->ev_pool.push_back(e);
        }
    }
    *a = c->ev_pool[2 * c->rec_used];
    *b = c->ev_pool[2 * c->rec_used + 1];
    if (c->rec_id.size() <= c->rec_used) c->rec_id.resize(c->rec_used + 1);
    c->rec_id[c->rec_used] = id;
    c->rec_used++;
    return true;
}

hipError_t launch(qed_ctx *c, int id, const qed::StepArgs &a, int precision, int blocks) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof && !c->capturing && prof_pair(c, id, &e0, &e1)) {
        hipError_t r = hipEventRecord(e0, c->stream);
        if (r != hipSuccess) return r;
    }
    hipError_t r = qed::launch_kernel(id, a, precision, blocks, c->stream);
    if (r == hipSuccess && e1) r = hipEventRecord(e1, c->stream);
    return r;
}

}  // namespace

namespace {

// Device buffers of one table / training run, released on every exit path.
struct DevBufs {
    std::vector<void *> p;
    template <class T>
    bool alloc(T **out, size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return false;
        p.push_back(q);
        *out = static_cast<T *>(q);
        return true;
    }
    ~DevBufs() {
        for (void *q : p) (void)hipFree(q);
    }
};

bool table_args_ok(double lo, double hi, uint32_t nchi, uint32_t nx) {
    return isfinite(lo) && isfinite(hi) && hi > lo && nchi >= 2 && nchi <= 65536 && nx >= 256 && nx % 256 == 0 &&
           nx <= (1u << 20) && (u64)nchi * (nx + 1) <= (1ull << 31);
}

qed_status build_table(qed_ctx *c, DevBufs &B, double lo, double hi, uint32_t nchi, uint32_t nx,
                       qed::CdfTableDev &t, int kind = 0) {
    t.kind = kind;
    t.nchi = (int)nchi;
    t.nx = (int)nx;
    t.lo10 = lo;
    t.hi10 = hi;
    if (!B.alloc(&t.cdf, (size_t)nchi * (nx + 1) * sizeof(double)) || !B.alloc(&t.total, nchi * sizeof(double)))
        return QED_ERR_HIP;
    if (qed::launch_cdf_table(t, c->stream) != hipSuccess) return QED_ERR_HIP;
    return QED_OK;
}

// Seeded initial weights: uniform in +-sqrt(6 / (fan_in + fan_out)), zero biases.
void init_params(float *p, uint64_t seed) {
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0xD1B54A32D192ED03ull;
    auto next = [&x]() {  // splitmix64
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1p-53;
    };
    for (int k = 0; k < QED_MLP_NPARAMS; ++k) p[k] = 0.0f;
    auto fill = [&](int off, int n, int fin, int fout) {
        const double a = sqrt(6.0 / (fin + fout));
        for (int k = 0; k < n; ++k) p[off + k] = (float)((2.0 * next() - 1.0) * a);
    };
    fill(qed::kOffW1, 128, 2, 64);
    fill(qed::kOffW2, 4096, 64, 64);
    fill(qed::kOffW3, 4096, 64, 64);
    fill(qed::kOffW4, 64, 64, 1);
}

}  // namespace

namespace {

// fixed: nullptr to use (and grow) the context's scratch; else the static array's
// lists, within QED_STATIC_MAX_SLOTS per species (no allocation, no host wait).
qed_status step_impl(qed_ctx *c, qed_particles *p, const qed_field fields[3], double dt, uint64_t seed,
                     uint32_t step, uint32_t *step_dev, const SlotScratch *fixed = nullptr) {
    if (!c || !p || !fields) return QED_ERR_INVALID_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return QED_ERR_INVALID_ARG;
    const bool emission = c->cfg.emission != 0, pairs = c->cfg.pairs != 0;
    const qed_species *sp[3] = {&p->electrons, &p->positrons, &p->photons};
    // every species that can be read or appended to must be complete
    const bool need[3] = {emission || pairs, emission || pairs, emission || pairs};
    for (int s = 0; s < 3; ++s) {
        if (!need[s]) continue;
        if (!species_ok(*sp[s])) return QED_ERR_INVALID_ARG;
    }
    if (emission && (!field_ok(fields[0]) || !field_ok(fields[1]))) return QED_ERR_INVALID_ARG;
    const bool surrogate = c->cfg.sampler == QED_SAMPLER_SURROGATE;
    if (surrogate && emission && (!sp[0]->tau || !sp[1]->tau)) return QED_ERR_INVALID_ARG;
    if (pairs && !field_ok(fields[2])) return QED_ERR_INVALID_ARG;
    const bool pair_surr = pairs && c->cfg.pair_sampler == QED_SAMPLER_SURROGATE;
    if (pair_surr && !sp[2]->tau) return QED_ERR_INVALID_ARG;
    const uint32_t gens = c->cfg.cascade_generations;
    if (gens > 0) {
        for (int s = 0; s < 3; ++s)
            if (need[s] && !sp[s]->birth) return QED_ERR_INVALID_ARG;
        for (int s = 0; s < 3; ++s)
            if ((s < 2 ? emission : pairs) && fields[s].stride != 0) return QED_ERR_INVALID_ARG;
    }
    const bool binned = c->cfg.scheduler == QED_SCHED_BINNED && emission;
    if (binned && (sp[0]->capacity > 0xFFFFFFFFull || sp[1]->capacity > 0xFFFFFFFFull))
        return QED_ERR_INVALID_ARG;
    const bool cells = c->cells.n[0] != nullptr;
    if (fixed) {
        // every slot a kernel of this step can touch lies below a species' capacity
        if (pairs && sp[2]->capacity > kStaticSlots) return QED_ERR_SCRATCH;
        for (int s = 0; s < 2; ++s)
            if (binned && sp[s]->capacity > kStaticSlots) return QED_ERR_SCRATCH;
        for (int s = 0; s < 3; ++s)
            if (cells && need[s] && sp[s]->capacity > kStaticSlots) return QED_ERR_SCRATCH;
    }
    HIP_TRY(hipSetDevice(c->cfg.device));
    if (pairs && !fixed) {
        qed_status r = ensure_photon_scratch(c, sp[2]->capacity > 0 ? sp[2]->capacity : 1);
        if (r != QED_OK) return r;
    }
    if (binned && !fixed) {
        for (int s = 0; s < 2; ++s) {
            qed_status r = ensure_lepton_scratch(c, s, sp[s]->capacity > 0 ? sp[s]->capacity : 1);
            if (r != QED_OK) return r;
        }
    }
    if (cells && !fixed) {
        for (int s = 0; s < 3; ++s) {
            if (!need[s]) continue;
            qed_status r = ensure_cell_slots(c, s, sp[s]->capacity > 0 ? sp[s]->capacity : 1);
            if (r != QED_OK) return r;
        }
    }
    SlotScratch x;
    if (fixed) {
        x = *fixed;
    } else {
        x.alive = c->alive;
        x.dead_idx = c->dead_idx;
        x.hole_idx = c->hole_idx;
        x.mover_idx = c->mover_idx;
        for (int s = 0; s < 2; ++s) {
            x.nsub[s] = c->nsub[s];
            x.queue[s] = c->queue[s];
        }
        for (int s = 0; s < 3; ++s) x.cell_slot[s] = c->cell_slot[s];
    }
    qed::StepArgs a;
    memset(&a, 0, sizeof(a));
    for (int s = 0; s < 3; ++s) {
        a.sp[s] = to_dev(*sp[s]);
        if (gens > 0) a.sp[s].birth = sp[s]->birth;
        if (s == 2 && !pair_surr) a.sp[s].tau = nullptr;  // photons carry tau on that path only
        a.fl[s] = to_dev(fields[s]);
        c->last_n[s] = a.sp[s].n;
    }
    a.st = c->st;
    a.dt = dt;
    a.p_max = c->cfg.p_max;
    a.p_max_lep = surrogate ? c->cfg.surrogate_p_max : c->cfg.p_max;
    a.pair_coef = c->cfg.pair_bound_coef;
    a.seed = seed;
    a.step = step;
    a.step_dev = step_dev;
    a.max_sub = c->cfg.max_substeps;
    a.emission = emission;
    a.pairs = pairs;
    a.light_max = c->tune.light_max;
    a.chunk = c->tune.chunk;
    a.resolve_batch = c->tune.resolve_batch;
    a.prepass_finish = c->tune.prepass_finish;
    a.bins_per_octave = c->tune.bins_per_octave;
    a.light_tile = c->tune.light_tile;
    a.tiled_slots = c->tune.tiled_slots;
    a.alive = x.alive;
    a.dead_idx = x.dead_idx;
    a.hole_idx = x.hole_idx;
    a.mover_idx = x.mover_idx;
    for (int s = 0; s < 2; ++s) {
        a.nsub[s] = x.nsub[s];
        a.queue[s] = x.queue[s];
    }
    a.gap_hist = reinterpret_cast<u64 *>(c->gap_hist);
    a.gap_bins = c->gap_bins;
    a.sampler = surrogate ? 1 : 0;
    a.model = c->have_model ? c->model : nullptr;
    a.pair_model = c->have_pair_model ? c->pair_model : nullptr;
    a.cells = c->cells;
    for (int s = 0; s < 3; ++s) a.cells.slot[s] = x.cell_slot[s];
    const u64 lep_cap = sp[0]->capacity > sp[1]->capacity ? sp[0]->capacity : sp[1]->capacity;
    const int lepton_blocks = grid_for(lep_cap, c->num_cu * (int)c->tune.lepton_blocks_per_cu);
    const int heavy_blocks = c->num_cu * (int)c->tune.heavy_blocks_per_cu;
    const int photon_blocks = grid_for(sp[2]->capacity, c->num_cu * (int)c->tune.photon_blocks_per_cu);
    const int aux_blocks = grid_for(sp[2]->capacity, c->num_cu * 4);
    const int prec = c->cfg.precision == QED_PREC_F64 ? 0 : 1;
    hipError_t r = launch(c, qed::K_BEGIN, a, prec, 1);
    if (r == hipSuccess && a.cells.n[0]) {
        const u64 ncell = (u64)a.cells.nx * a.cells.ny * a.cells.nz;
        u64 cap = lep_cap > sp[2]->capacity ? lep_cap : sp[2]->capacity;
        r = launch(c, qed::K_CELL_CLEAR, a, prec, grid_for(ncell, c->num_cu * 4));
        if (r == hipSuccess) r = launch(c, qed::K_CELL_MAX, a, prec, grid_for(cap, c->num_cu * 8));
    }
    if (r == hipSuccess && pairs) r = launch(c, pair_surr ? qed::K_PHOTON_SURR : qed::K_PHOTON, a, prec, photon_blocks);
    const bool tiled = c->cfg.scheduler == QED_SCHED_TILED;
    if (r == hipSuccess && emission && !binned)
        r = launch(c, tiled ? qed::K_TILED : qed::K_LEPTON, a, prec, lepton_blocks);
    if (binned) {
        if (r == hipSuccess)
            r = launch(c, qed::K_PREPASS, a, prec, grid_for(lep_cap, c->num_cu * (int)c->tune.prepass_blocks_per_cu));
        if (r == hipSuccess) r = launch(c, qed::K_SCAN, a, prec, 1);
        if (r == hipSuccess)
            r = launch(c, qed::K_SCATTER, a, prec, grid_for(lep_cap, c->num_cu * (int)c->tune.scatter_blocks_per_cu));
        if (r == hipSuccess && a.light_max > 0) r = launch(c, qed::K_LIGHT, a, prec, lepton_blocks);
        if (r == hipSuccess) r = launch(c, qed::K_HEAVY, a, prec, heavy_blocks);
    }
    // cascade passes: the particles of the previous pass, from their birth time
    for (uint32_t g = 1; g <= gens && r == hipSuccess; ++g) {
        a.gen = g;
        r = launch(c, qed::K_GEN, a, prec, 1);
        if (r == hipSuccess && pairs) r = launch(c, qed::K_PHOTON, a, prec, photon_blocks);
        if (r == hipSuccess && emission) r = launch(c, qed::K_LEPTON, a, prec, lepton_blocks);
    }
    a.gen = 0;
    if (r == hipSuccess) r = launch(c, qed::K_END, a, prec, 1);
    if (r == hipSuccess && pairs) r = launch(c, qed::K_FILL, a, prec, aux_blocks);
    if (r == hipSuccess && pairs) r = launch(c, qed::K_MOVE, a, prec, aux_blocks);
    return r == hipSuccess ? QED_OK : QED_ERR_HIP;
}

}  // namespace

namespace {

qed_status set_model(qed_ctx *c, const qed_sampler_model *m, qed::MlpModel *dst, bool &have) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    if (!m) {
        HIP_TRY(hipSetDevice(c->cfg.device));
        HIP_TRY(hipStreamSynchronize(c->stream));
        have = false;
        return QED_OK;
    }
    if (!m->params || m->nbins < 1 || m->nbins > QED_MLP_MAX_BINS || !m->fallback) return QED_ERR_INVALID_ARG;
    if (!(m->log10_chi_hi > m->log10_chi_lo) || !isfinite(m->log10_chi_lo) || !isfinite(m->log10_chi_hi))
        return QED_ERR_INVALID_ARG;
    for (int k = 0; k < QED_MLP_NPARAMS; ++k)
        if (!isfinite(m->params[k])) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    float *dp = nullptr;
    HIP_TRY(hipMalloc(&dp, QED_MLP_NPARAMS * sizeof(float)));
    qed_status st = QED_OK;
    if (hipMemcpy(dp, m->params, QED_MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        qed::launch_mlp_pack(dp, dst, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        st = QED_ERR_HIP;
    (void)hipFree(dp);
    if (st != QED_OK) return st;
    // the range, bins and fallback flags
    struct {
        float lo, inv_span;
        int nbins;
    } head = {(float)m->log10_chi_lo, (float)(1.0 / (m->log10_chi_hi - m->log10_chi_lo)), m->nbins};
    uint8_t fb[QED_MLP_MAX_BINS];
    memset(fb, 1, sizeof(fb));
    for (int k = 0; k < m->nbins; ++k) fb[k] = m->fallback[k] ? 1 : 0;
    char *base = reinterpret_cast<char *>(dst);
    HIP_TRY(hipMemcpy(base + offsetof(qed::MlpModel, lo), &head, sizeof(head), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + offsetof(qed::MlpModel, fallback), fb, sizeof(fb), hipMemcpyHostToDevice));
    have = true;
    return QED_OK;
}

}  // namespace

extern "C" {

qed_status qed_config_default(qed_config *cfg) {
    if (!cfg) return QED_ERR_INVALID_ARG;
    memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->stream = nullptr;
    cfg->precision = QED_PREC_MIXED;
    cfg->p_max = 0.01;
    cfg->emission = 1;
    cfg->pairs = 1;
    cfg->scheduler = QED_SCHED_NAIVE;
    cfg->pair_bound_coef = 0.1;
    cfg->max_substeps = 1u << 24;
    cfg->sampler = QED_SAMPLER_REJECTION;
    cfg->cascade_generations = 0;
    cfg->surrogate_p_max = 0.1;
    cfg->pair_sampler = QED_SAMPLER_REJECTION;
    return QED_OK;
}

qed_status qed_init(qed_ctx **out, const qed_config *cfg) {
    if (!out || !cfg) return QED_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->precision != QED_PREC_F64 && cfg->precision != QED_PREC_MIXED) return QED_ERR_INVALID_ARG;
    if (!(cfg->p_max > 0.0 && cfg->p_max <= 1.0)) return QED_ERR_INVALID_ARG;
    if (!(cfg->pair_bound_coef > 0.0) || !isfinite(cfg->pair_bound_coef)) return QED_ERR_INVALID_ARG;
    if (cfg->max_substeps < 1) return QED_ERR_INVALID_ARG;
    if (cfg->scheduler != QED_SCHED_NAIVE && cfg->scheduler != QED_SCHED_BINNED && cfg->scheduler != QED_SCHED_TILED)
        return QED_ERR_INVALID_ARG;
    if (cfg->sampler != QED_SAMPLER_REJECTION && cfg->sampler != QED_SAMPLER_SURROGATE) return QED_ERR_INVALID_ARG;
    if (cfg->sampler == QED_SAMPLER_SURROGATE && cfg->precision != QED_PREC_MIXED) return QED_ERR_INVALID_ARG;
    if (cfg->cascade_generations > 64) return QED_ERR_INVALID_ARG;
    if (cfg->sampler == QED_SAMPLER_SURROGATE && !(cfg->surrogate_p_max > 0.0 && cfg->surrogate_p_max <= 1.0))
        return QED_ERR_INVALID_ARG;
    if (cfg->cascade_generations > 0 && cfg->sampler != QED_SAMPLER_REJECTION) return QED_ERR_INVALID_ARG;
    if (cfg->pair_sampler != QED_SAMPLER_REJECTION && cfg->pair_sampler != QED_SAMPLER_SURROGATE)
        return QED_ERR_INVALID_ARG;
    if (cfg->pair_sampler == QED_SAMPLER_SURROGATE &&
        (cfg->precision != QED_PREC_MIXED || cfg->cascade_generations > 0))
        return QED_ERR_INVALID_ARG;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(cfg->device));
    {
        const qed_status r = resolve_scratch(cfg->device);
        if (r != QED_OK) return r;
    }
    qed_ctx *c = new (std::nothrow) qed_ctx();
    if (!c) return QED_ERR_HIP;
    c->cfg = *cfg;
    c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) {
        delete c;
        return QED_ERR_HIP;
    }
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->tune.lepton_blocks_per_cu = 8;
    c->tune.heavy_blocks_per_cu = 4;
    c->tune.photon_blocks_per_cu = 8;
    c->tune.light_max = 48;
    c->tune.chunk = 256;
    c->tune.resolve_batch = 16;
    c->tune.prepass_finish = 1;
    c->tune.prepass_blocks_per_cu = 8;
    c->tune.scatter_blocks_per_cu = 2;
    c->tune.bins_per_octave = 16;
    c->tune.light_tile = 512;
    c->tune.tiled_slots = 256;
    c->tune.deposit_sort_min = 1u << 14;
    if (hipMalloc(&c->st, sizeof(qed::DevState)) != hipSuccess ||
        hipMemset(c->st, 0, sizeof(qed::DevState)) != hipSuccess ||
        hipMalloc(&c->model, sizeof(qed::MlpModel)) != hipSuccess ||
        hipMalloc(&c->pair_model, sizeof(qed::MlpModel)) != hipSuccess) {
        if (c->st) (void)hipFree(c->st);
        if (c->model) (void)hipFree(c->model);
        if (c->pair_model) (void)hipFree(c->pair_model);
        delete c;
        return QED_ERR_HIP;
    }
    *out = c;
    return QED_OK;
}

qed_status qed_step(qed_ctx *c, qed_particles *p, const qed_field fields[3], double dt, uint64_t seed,
                    uint32_t step) {
    return step_impl(c, p, fields, dt, seed, step, nullptr);
}

qed_status qed_step_counted(qed_ctx *c, qed_particles *p, const qed_field fields[3], double dt, uint64_t seed,
                            uint32_t *step) {
    if (!step) return QED_ERR_INVALID_ARG;
    return step_impl(c, p, fields, dt, seed, 0, step);
}

qed_status qed_step_static(qed_ctx *c, qed_particles *p, const qed_field fields[3], double dt, uint64_t seed,
                           uint32_t step) {
    if (!c) return QED_ERR_INVALID_ARG;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c->cfg.device >= 0 && c->cfg.device < kMaxDevices) base = g_scratch_ptr[c->cfg.device];
    }
    if (!base) return QED_ERR_STATE;  // qed_init resolves it for the context's device
    const SlotScratch x = static_scratch(base);
    return step_impl(c, p, fields, dt, seed, step, nullptr, &x);
}

qed_status qed_sync(qed_ctx *c, qed_report *rep) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    qed::DevState h;
    HIP_TRY(hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost));
    qed_status s = QED_OK;
    if (h.status_bits & 1ull)
        s = QED_ERR_CAPACITY;
    else if (h.status_bits & 2ull)
        s = QED_ERR_NONFINITE;
    if (rep) {
        memset(rep, 0, sizeof(*rep));
        rep->status = s;
        for (int k = 0; k < 3; ++k) {
            rep->required_capacity[k] = h.required[k];
            if (c->last_n[k]) HIP_TRY(hipMemcpy(&rep->n[k], c->last_n[k], sizeof(u64), hipMemcpyDeviceToHost));
        }
        rep->nonfinite = h.nonfinite;
    }
    // clear the sticky status
    h.status_bits = 0;
    h.nonfinite = 0;
    h.required[0] = h.required[1] = h.required[2] = 0;
    HIP_TRY(hipMemcpy(&c->st->status_bits, &h.status_bits, sizeof(u64), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&c->st->nonfinite, &h.nonfinite, sizeof(u64), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&c->st->required[0], &h.required[0], 3 * sizeof(u64), hipMemcpyHostToDevice));
    return s;
}

namespace {
bool grid_ok(const qed_grid &g, qed::GridDev &d) {
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return false;
    if ((u64)g.nx * g.ny * g.nz >= (1ull << 31)) return false;
    if (!(g.dx > 0.0 && g.dy > 0.0 && g.dz > 0.0) || !isfinite(g.dx) || !isfinite(g.dy) || !isfinite(g.dz))
        return false;
    if (!isfinite(g.x0) || !isfinite(g.y0) || !isfinite(g.z0)) return false;
    const void *f[6] = {g.ex, g.ey, g.ez, g.bx, g.by, g.bz};
    for (int k = 0; k < 6; ++k) d.f[k] = f[k];
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.x0 = g.x0;
    d.y0 = g.y0;
    d.z0 = g.z0;
    d.idx = 1.0 / g.dx;
    d.idy = 1.0 / g.dy;
    d.idz = 1.0 / g.dz;
    return true;
}
}  // namespace

qed_status qed_gather(qed_ctx *c, const qed_grid *grid, const qed_species *sp, void *const out[6]) {
    if (!c || !grid || !sp || !out) return QED_ERR_INVALID_ARG;
    qed::GridDev g;
    if (!grid_ok(*grid, g)) return QED_ERR_INVALID_ARG;
    for (int k = 0; k < 6; ++k)
        if (!g.f[k] || !out[k]) return QED_ERR_INVALID_ARG;
    if (!sp->n || !sp->x || !sp->y || !sp->z) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    qed::GatherArgs a;
    a.n = reinterpret_cast<const u64 *>(sp->n);
    a.cap = sp->capacity;
    a.x = sp->x;
    a.y = sp->y;
    a.z = sp->z;
    for (int k = 0; k < 6; ++k) a.out[k] = out[k];
    const int dtype = c->cfg.precision == QED_PREC_F64 ? 1 : 0;
    if (qed::launch_gather(g, a, dtype, grid_for(sp->capacity, c->num_cu * 8), c->stream) != hipSuccess)
        return QED_ERR_HIP;
    return QED_OK;
}

qed_status qed_deposit(qed_ctx *c, const qed_grid *grid, const qed_species *sp, double charge, double *jx,
                       double *jy, double *jz) {
    if (!c || !grid || !sp || !jx || !jy || !jz || !isfinite(charge)) return QED_ERR_INVALID_ARG;
    qed::GridDev g;
    if (!grid_ok(*grid, g)) return QED_ERR_INVALID_ARG;
    if (!sp->n || !sp->x || !sp->y || !sp->z || !sp->ux || !sp->uy || !sp->uz || !sp->w) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    qed::DepositArgs a;
    a.n = reinterpret_cast<const u64 *>(sp->n);
    a.cap = sp->capacity;
    a.x = sp->x;
    a.y = sp->y;
    a.z = sp->z;
    a.ux = sp->ux;
    a.uy = sp->uy;
    a.uz = sp->uz;
    a.w = sp->w;
    a.charge = charge;
    a.j[0] = jx;
    a.j[1] = jy;
    a.j[2] = jz;
    const int dtype = c->cfg.precision == QED_PREC_F64 ? 1 : 0;
    const uint32_t te = qed::kDepTileEdge;
    const u64 tiles[3] = {(grid->nx + te - 1) / te, (grid->ny + te - 1) / te, (grid->nz + te - 1) / te};
    const u64 ntiles = tiles[0] * tiles[1] * tiles[2];
    if (sp->capacity >= c->tune.deposit_sort_min && sp->capacity < (1ull << 32) && ntiles <= qed::kDepMaxTiles &&
        ensure_deposit_scratch(c, sp->capacity, ntiles)) {
        qed::DepSortArgs d;
        d.n = a.n;
        d.cap = sp->capacity;
        d.x = a.x;
        d.y = a.y;
        d.z = a.z;
        d.ux = a.ux;
        d.uy = a.uy;
        d.uz = a.uz;
        d.w = a.w;
        d.charge = charge;
        for (int k = 0; k < 3; ++k) {
            d.j[k] = a.j[k];
            d.tiles[k] = (uint32_t)tiles[k];
        }
        d.ntiles = (uint32_t)ntiles;
        d.max_parts = qed::dep_max_parts(sp->capacity, ntiles);
        d.count = c->dep_count;
        d.off = c->dep_off;
        d.part_off = c->dep_part_off;
        d.part_tile = c->dep_part_tile;
        d.pos = c->dep_pos;
        d.rec = c->dep_rec;
        d.stage = c->dep_stage;
        if (qed::launch_deposit_sorted(g, d, dtype, grid_for(sp->capacity, c->num_cu * 8), c->stream) != hipSuccess)
            return QED_ERR_HIP;
        return QED_OK;
    }
    if (qed::launch_deposit(g, a, dtype, grid_for(sp->capacity, c->num_cu * 8), c->stream) != hipSuccess)
        return QED_ERR_HIP;
    return QED_OK;
}

qed_status qed_synchrotron(qed_ctx *c, const void *x, void *F, void *G, uint64_t n, int dtype) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (dtype != QED_F32 && dtype != QED_F64) return QED_ERR_INVALID_ARG;
    if (n == 0) return QED_OK;
    if (!x || (!F && !G)) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    // grid-stride over 128 (float) or 64 (double) blocks per CU: measured fastest on
    // gfx950 for the 2^28-element benchmark (each block stages the fit table once)
    const int blocks = grid_for(n, c->num_cu * (dtype == QED_F32 ? 128 : 64));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof && prof_pair(c, qed::K_SYNCHROTRON, &e0, &e1)) HIP_TRY(hipEventRecord(e0, c->stream));
    if (qed::launch_synchrotron(x, F, G, n, dtype == QED_F32 ? 0 : 1, c->st, blocks, c->stream) != hipSuccess)
        return QED_ERR_HIP;
    if (e1) HIP_TRY(hipEventRecord(e1, c->stream));
    return QED_OK;
}

qed_status qed_get_stats(qed_ctx *c, qed_stats *out) {
    if (!c || !out) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    qed::DevState h;
    HIP_TRY(hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost));
    memset(out, 0, sizeof(*out));
    out->steps = h.steps;
    for (int k = 0; k < 3; ++k) {
        out->substeps[k] = h.substeps[k];
        out->particles[k] = h.particles[k];
    }
    out->heavy_particles = h.heavy_particles;
    out->heavy_substeps = h.heavy_substeps;
    out->sampled_photons = h.sampled_photons;
    out->sampled_substeps = h.sampled_substeps;
    out->emissions = h.emissions;
    out->pairs = h.pairs;
    out->clips = h.clips;
    out->capped = h.capped;
    out->learned_events = h.learned_events;
    out->fallback_events = h.fallback_events;
    out->fallback_draws = h.fallback_draws;
    out->envelope_clips = h.envelope_clips;
    out->pair_learned = h.pair_learned;
    out->pair_fallback = h.pair_fallback;
    out->pair_fallback_draws = h.pair_fallback_draws;
    out->pair_envelope_clips = h.pair_envelope_clips;
    out->chi_guard = h.chi_guard;
    double mp;
    memcpy(&mp, &h.max_p_bits, sizeof(mp));
    out->max_p = mp;
    return QED_OK;
}

qed_status qed_reset_stats(qed_ctx *c) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    qed::DevState h;
    HIP_TRY(hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost));
    h.steps = 0;
    h.substeps[0] = h.substeps[1] = h.substeps[2] = 0;
    h.particles[0] = h.particles[1] = h.particles[2] = 0;
    h.heavy_particles = h.heavy_substeps = 0;
    h.sampled_photons = h.sampled_substeps = 0;
    h.emissions = h.pairs = h.clips = h.capped = 0;
    h.learned_events = h.fallback_events = h.fallback_draws = h.envelope_clips = 0;
    h.pair_learned = h.pair_fallback = h.pair_fallback_draws = h.pair_envelope_clips = 0;
    h.chi_guard = 0;
    h.max_p_bits = 0;
    HIP_TRY(hipMemcpy(c->st, &h, sizeof(h), hipMemcpyHostToDevice));
    return QED_OK;
}

qed_status qed_graph_begin(qed_ctx *c) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (c->capturing || !c->stream) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    return QED_OK;
}

qed_status qed_graph_end(qed_ctx *c, qed_graph **out) {
    if (!c || !out) return QED_ERR_INVALID_ARG;
    *out = nullptr;
    if (!c->capturing) return QED_ERR_STATE;
    c->capturing = false;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return QED_ERR_HIP;
    }
    qed_graph *h = new (std::nothrow) qed_graph();
    if (!h) {
        (void)hipGraphExecDestroy(e);
        (void)hipGraphDestroy(g);
        return QED_ERR_HIP;
    }
    h->graph = g;
    h->exec = e;
    *out = h;
    return QED_OK;
}

qed_status qed_graph_launch(qed_ctx *c, qed_graph *g) {
    if (!c || !g) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipGraphLaunch(g->exec, c->stream));
    return QED_OK;
}

void qed_graph_destroy(qed_graph *g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

qed_status qed_get_tuning(qed_ctx *c, qed_tuning *out) {
    if (!c || !out) return QED_ERR_INVALID_ARG;
    *out = c->tune;
    return QED_OK;
}

qed_status qed_set_tuning(qed_ctx *c, const qed_tuning *t) {
    if (!c || !t || !tuning_ok(*t)) return QED_ERR_INVALID_ARG;
    c->tune = *t;
    return QED_OK;
}

qed_status qed_profile_enable(qed_ctx *c, int on) {
    if (!c) return QED_ERR_INVALID_ARG;
    c->prof = on != 0;
    return QED_OK;
}

qed_status qed_profile_read(qed_ctx *c, qed_kernel_time *out, int max, int *count) {
    if (!c || !count || max < 0 || (max > 0 && !out)) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double ms[qed::K_COUNT] = {0};
    u64 nl[qed::K_COUNT] = {0};
    for (size_t k = 0; k < c->rec_used; ++k) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
        ms[c->rec_id[k]] += t;
        nl[c->rec_id[k]] += 1;
    }
    c->rec_used = 0;
    int w = 0;
    for (int id = 0; id < qed::K_COUNT && w < max; ++id) {
        if (!nl[id]) continue;
        out[w].name = kKernelName[id];
        out[w].launches = nl[id];
        out[w].total_ms = ms[id];
        ++w;
    }
    *count = w;
    return QED_OK;
}

// ---------------------------------------------------------------------------
// Surrogate sampler: model installation, evaluation, training.
// ---------------------------------------------------------------------------
qed_status qed_sampler_set(qed_ctx *c, const qed_sampler_model *m) {
    if (!c) return QED_ERR_INVALID_ARG;
    return set_model(c, m, c->model, c->have_model);
}

qed_status qed_pair_sampler_set(qed_ctx *c, const qed_sampler_model *m) {
    if (!c) return QED_ERR_INVALID_ARG;
    return set_model(c, m, c->pair_model, c->have_pair_model);
}

qed_status qed_pair_sampler_infer(qed_ctx *c, const float *chi, const float *u, float *d, uint64_t n) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (n == 0) return QED_OK;
    if (!chi || !u || !d) return QED_ERR_INVALID_ARG;
    if (!c->have_pair_model) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    if (qed::launch_mlp_infer(c->pair_model, chi, u, d, n, grid_for(n, c->num_cu * 8), c->stream, 1) != hipSuccess)
        return QED_ERR_HIP;
    return QED_OK;
}

qed_status qed_sampler_infer(qed_ctx *c, const float *chi, const float *u, float *x, uint64_t n) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (n == 0) return QED_OK;
    if (!chi || !u || !x) return QED_ERR_INVALID_ARG;
    if (!c->have_model) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    if (qed::launch_mlp_infer(c->model, chi, u, x, n, grid_for(n, c->num_cu * 8), c->stream) != hipSuccess)
        return QED_ERR_HIP;
    return QED_OK;
}

qed_status qed_emission_rate(qed_ctx *c, const float *chi, float *chi_q, uint64_t n) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (n == 0) return QED_OK;
    if (!chi || !chi_q) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    if (qed::launch_rate(chi, chi_q, n, grid_for(n, c->num_cu * 8), c->stream) != hipSuccess) return QED_ERR_HIP;
    return QED_OK;
}


qed_status qed_substep_cells(qed_ctx *c, const qed_grid *g) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    if (!g) {
        c->cells.n[0] = c->cells.n[1] = nullptr;
        return QED_OK;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return QED_ERR_INVALID_ARG;
    const u64 ncell = (u64)g->nx * g->ny * g->nz;
    if (ncell > (1ull << 28)) return QED_ERR_INVALID_ARG;
    if (!(g->dx > 0.0 && g->dy > 0.0 && g->dz > 0.0) || !isfinite(g->dx) || !isfinite(g->dy) || !isfinite(g->dz))
        return QED_ERR_INVALID_ARG;
    if (!isfinite(g->x0) || !isfinite(g->y0) || !isfinite(g->z0)) return QED_ERR_INVALID_ARG;
    if (c->cfg.sampler != QED_SAMPLER_REJECTION || c->cfg.pair_sampler != QED_SAMPLER_REJECTION ||
        c->cfg.cascade_generations != 0)
        return QED_ERR_STATE;
    if (ncell > c->cell_cap) {
        HIP_TRY(hipSetDevice(c->cfg.device));
        uint32_t *buf = nullptr;
        HIP_TRY(hipMalloc(&buf, 2 * ncell * sizeof(uint32_t)));
        retire(c, c->cell_buf);
        c->cell_buf = buf;
        c->cell_cap = ncell;
    }
    c->cells.n[0] = c->cell_buf;
    c->cells.n[1] = c->cell_buf + ncell;
    c->cells.nx = g->nx;
    c->cells.ny = g->ny;
    c->cells.nz = g->nz;
    c->cells.x0 = g->x0;
    c->cells.y0 = g->y0;
    c->cells.z0 = g->z0;
    c->cells.dx = g->dx;
    c->cells.dy = g->dy;
    c->cells.dz = g->dz;
    return QED_OK;
}

qed_status qed_event_gaps(qed_ctx *c, uint64_t *hist, uint32_t nbins) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (hist && nbins < 2) return QED_ERR_INVALID_ARG;
    c->gap_hist = hist;
    c->gap_bins = hist ? nbins : 0;
    return QED_OK;
}

qed_status qed_pair_rate(qed_ctx *c, const float *chi, float *T, uint64_t n) {
    if (!c) return QED_ERR_INVALID_ARG;
    if (n == 0) return QED_OK;
    if (!chi || !T) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    if (qed::launch_pair_rate(chi, T, n, grid_for(n, c->num_cu * 8), c->stream) != hipSuccess) return QED_ERR_HIP;
    return QED_OK;
}

qed_status qed_emission_cdf(qed_ctx *c, double lo, double hi, uint32_t nchi, uint32_t nx, double *cdf_out,
                            double *total_out) {
    if (!c || !cdf_out || !table_args_ok(lo, hi, nchi, nx)) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    DevBufs B;
    qed::CdfTableDev t;
    qed_status st = build_table(c, B, lo, hi, nchi, nx, t);
    if (st != QED_OK) return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(cdf_out, t.cdf, (size_t)nchi * (nx + 1) * sizeof(double), hipMemcpyDeviceToHost));
    if (total_out) HIP_TRY(hipMemcpy(total_out, t.total, nchi * sizeof(double), hipMemcpyDeviceToHost));
    return QED_OK;
}

qed_status qed_train_config_default(qed_train_config *cfg) {
    if (!cfg) return QED_ERR_INVALID_ARG;
    memset(cfg, 0, sizeof(*cfg));
    cfg->log10_chi_lo = -3.0;
    cfg->log10_chi_hi = 2.0;
    cfg->table_chi = 1025;
    cfg->table_x = 8192;
    cfg->steps = 60000;
    cfg->blocks = 256;
    cfg->batch_tiles = 4;
    cfg->lr = 1e-2f;
    cfg->lr_final = 3e-5f;
    cfg->seed = 1;
    cfg->nbins = 50;
    cfg->per_bin = 5;
    cfg->tolerance = 1e-3;
    return QED_OK;
}

qed_status qed_train_sampler(qed_ctx *c, const qed_train_config *cfg, const float *init, float *params_out,
                             float *loss_out, float *bin_err_out, uint8_t *fallback_out) {
    if (!c || !cfg || !params_out) return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    if (!table_args_ok(cfg->log10_chi_lo, cfg->log10_chi_hi, cfg->table_chi, cfg->table_x)) return QED_ERR_INVALID_ARG;
    if (cfg->steps < 1 || cfg->blocks < 1 || cfg->blocks > 65536 || cfg->batch_tiles < 1 || cfg->batch_tiles > 1024)
        return QED_ERR_INVALID_ARG;
    if (cfg->nbins < 1 || cfg->nbins > QED_MLP_MAX_BINS || cfg->per_bin < 2 || cfg->per_bin > 64)
        return QED_ERR_INVALID_ARG;
    if (!(cfg->lr > 0.0f) || !(cfg->lr_final > 0.0f) || !(cfg->tolerance > 0.0)) return QED_ERR_INVALID_ARG;
    if (cfg->target != 0 && cfg->target != 1) return QED_ERR_INVALID_ARG;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    DevBufs B;
    qed::CdfTableDev t;
    qed_status st =
        build_table(c, B, cfg->log10_chi_lo, cfg->log10_chi_hi, cfg->table_chi, cfg->table_x, t, cfg->target);
    if (st != QED_OK) return st;
    const u64 batch = (u64)cfg->blocks * 64 * cfg->batch_tiles;
    float *params, *m, *v, *partials, *loss, *bin_err;
    qed::Sample *data;
    qed::MlpModel *model;
    if (!B.alloc(&params, QED_MLP_NPARAMS * sizeof(float)) || !B.alloc(&m, QED_MLP_NPARAMS * sizeof(float)) ||
        !B.alloc(&v, QED_MLP_NPARAMS * sizeof(float)) ||
        !B.alloc(&partials, (size_t)cfg->blocks * (QED_MLP_NPARAMS + 1) * sizeof(float)) ||
        !B.alloc(&loss, cfg->steps * sizeof(float)) || !B.alloc(&bin_err, cfg->nbins * sizeof(float)) ||
        !B.alloc(&data, batch * sizeof(qed::Sample)) || !B.alloc(&model, sizeof(qed::MlpModel)))
        return QED_ERR_HIP;
    std::vector<float> h(QED_MLP_NPARAMS);
    if (init)
        memcpy(h.data(), init, h.size() * sizeof(float));
    else
        init_params(h.data(), cfg->seed);
    HIP_TRY(hipMemcpy(params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(m, 0, QED_MLP_NPARAMS * sizeof(float), c->stream));
    HIP_TRY(hipMemsetAsync(v, 0, QED_MLP_NPARAMS * sizeof(float), c->stream));
    HIP_TRY(hipMemsetAsync(bin_err, 0, cfg->nbins * sizeof(float), c->stream));
    const double beta1 = 0.9, beta2 = 0.999;
    const int data_blocks = grid_for(batch, c->num_cu * 8);
    for (uint32_t k = 0; k < cfg->steps; ++k) {
        if (qed::launch_mlp_data(t, data, batch, cfg->seed, k, cfg->log10_chi_lo, cfg->log10_chi_hi, data_blocks,
                                 c->stream) != hipSuccess)
            return QED_ERR_HIP;
        qed::TrainArgs ta;
        ta.params = params;
        ta.batch = data;
        ta.partials = partials;
        ta.tiles = cfg->batch_tiles;
        ta.inv_batch = (float)(1.0 / (double)batch);
        if (qed::launch_mlp_train(ta, (int)cfg->blocks, c->stream) != hipSuccess) return QED_ERR_HIP;
        qed::ReduceArgs ra;
        memset(&ra, 0, sizeof(ra));
        ra.partials = partials;
        ra.blocks = (int)cfg->blocks;
        ra.params = params;
        ra.m = m;
        ra.v = v;
        ra.loss_out = loss + k;
        const double frac = cfg->steps > 1 ? (double)k / (double)(cfg->steps - 1) : 1.0;
        ra.lr = (float)(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + cos(M_PI * frac)));
        ra.beta1 = (float)beta1;
        ra.beta2 = (float)beta2;
        ra.eps = 1e-8f;
        ra.c1 = (float)(1.0 / (1.0 - pow(beta1, k + 1.0)));
        ra.c2 = (float)(1.0 / (1.0 - pow(beta2, k + 1.0)));
        if (qed::launch_mlp_reduce(ra, c->stream) != hipSuccess) return QED_ERR_HIP;
    }
    // validation of the packed network on the table
    if (qed::launch_mlp_pack(params, model, c->stream) != hipSuccess) return QED_ERR_HIP;
    struct {
        float lo, inv_span;
        int nbins;
    } head = {(float)cfg->log10_chi_lo, (float)(1.0 / (cfg->log10_chi_hi - cfg->log10_chi_lo)), cfg->nbins};
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(reinterpret_cast<char *>(model) + offsetof(qed::MlpModel, lo), &head, sizeof(head),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(reinterpret_cast<char *>(model) + offsetof(qed::MlpModel, fallback), 0, QED_MLP_MAX_BINS));
    if (qed::launch_mlp_validate(model, t, cfg->nbins, cfg->per_bin, bin_err, c->stream) != hipSuccess)
        return QED_ERR_HIP;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(params_out, params, QED_MLP_NPARAMS * sizeof(float), hipMemcpyDeviceToHost));
    if (loss_out) HIP_TRY(hipMemcpy(loss_out, loss, cfg->steps * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<float> be(cfg->nbins);
    HIP_TRY(hipMemcpy(be.data(), bin_err, cfg->nbins * sizeof(float), hipMemcpyDeviceToHost));
    for (int k = 0; k < cfg->nbins; ++k) {
        if (bin_err_out) bin_err_out[k] = be[k];
        if (fallback_out) fallback_out[k] = !(be[k] <= cfg->tolerance);
    }
    return QED_OK;
}

qed_status qed_mlp_gradient(qed_ctx *c, const float *params, const float *samples, uint64_t n, float *loss_out,
                            float *grad_out) {
    if (!c || !params || !samples || !grad_out || n == 0 || n % 64 != 0 || n > (1ull << 26))
        return QED_ERR_INVALID_ARG;
    if (c->capturing) return QED_ERR_STATE;
    HIP_TRY(hipSetDevice(c->cfg.device));
    HIP_TRY(hipStreamSynchronize(c->stream));
    DevBufs B;
    const int blocks = (int)(n / 64);
    float *dp, *partials, *grad, *loss;
    qed::Sample *data;
    if (!B.alloc(&dp, QED_MLP_NPARAMS * sizeof(float)) ||
        !B.alloc(&partials, (size_t)blocks * (QED_MLP_NPARAMS + 1) * sizeof(float)) ||
        !B.alloc(&grad, QED_MLP_NPARAMS * sizeof(float)) || !B.alloc(&loss, sizeof(float)) ||
        !B.alloc(&data, n * sizeof(qed::Sample)))
        return QED_ERR_HIP;
    HIP_TRY(hipMemcpy(dp, params, QED_MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(data, samples, n * sizeof(qed::Sample), hipMemcpyHostToDevice));
    qed::TrainArgs ta;
    ta.params = dp;
    ta.batch = data;
    ta.partials = partials;
    ta.tiles = 1;
    ta.inv_batch = (float)(1.0 / (double)n);
    if (qed::launch_mlp_train(ta, blocks, c->stream) != hipSuccess) return QED_ERR_HIP;
    qed::ReduceArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.partials = partials;
    ra.blocks = blocks;
    ra.grad_out = grad;
    ra.loss_out = loss;
    if (qed::launch_mlp_reduce(ra, c->stream) != hipSuccess) return QED_ERR_HIP;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(grad_out, grad, QED_MLP_NPARAMS * sizeof(float), hipMemcpyDeviceToHost));
    if (loss_out) HIP_TRY(hipMemcpy(loss_out, loss, sizeof(float), hipMemcpyDeviceToHost));
    return QED_OK;
}

void qed_finalize(qed_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    release(c->alive);
    release(c->dead_idx);
    release(c->hole_idx);
    release(c->mover_idx);
    for (int s = 0; s < 2; ++s) {
        release(c->nsub[s]);
        release(c->queue[s]);
    }
    release(c->st);
    release(c->model);
    release(c->pair_model);
    release(c->cell_buf);
    for (int s = 0; s < 3; ++s) release(c->cell_slot[s]);
    release(c->dep_pos);
    release(c->dep_rec);
    release(c->dep_count);
    release(c->dep_off);
    release(c->dep_part_off);
    release(c->dep_part_tile);
    release(c->dep_stage);
    for (void *b : c->retired) (void)hipFree(b);
    delete c;
}

const char *qed_status_string(qed_status s) {
    switch (s) {
        case QED_OK: return "ok";
        case QED_ERR_INVALID_ARG: return "invalid argument";
        case QED_ERR_CAPACITY: return "particle buffer capacity exceeded";
        case QED_ERR_NONFINITE: return "non-finite input";
        case QED_ERR_HIP: return "HIP runtime error";
        case QED_ERR_STATE: return "invalid state";
        case QED_ERR_SCRATCH: return "size beyond the static scratch of qed_step_static";
    }
    return "unknown status";
}

}  // extern "C"
