// Internal interface between the C ABI (qed_capi.hip) and the kernels
// (qed_kernels.hip, qed_train.hip, qed_grid.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "qed_mlp.hpp"

namespace qed {

typedef unsigned long long u64;

// Sub-step-count bins of the binned scheduler: bin 0 holds the light particles
// (N <= light_max), bin j >= 1 the heavy ones with floor(B log2 N) = j - 1, B bins per
// octave (the tuning's bins_per_octave, at most kMaxBinsPerOctave; at 16 the counts in
// one bin differ by less than 4.4%, so a wave of one bin idles little at the end of
// its loop).  kBins covers N up to 2^31 at the finest binning.
constexpr int kMaxBinsPerOctave = 32;
constexpr int kBins = 1024;
static_assert(1 + 31 * kMaxBinsPerOctave < kBins, "bins cover every sub-step count");

// Per-context device state: step bookkeeping and cumulative counters.
struct DevState {
    u64 n0[3];        // live counts at step start (clamped to capacity)
    u64 dead;         // photons that decayed in this step (= entries of the dead list)
    u64 ntot;         // photon count after appends (clamped), before compaction
    u64 S;            // photon count after compaction
    u64 holes;        // compaction: holes found in [0, S)
    u64 movers;       // compaction: survivors found in [S, ntot)
    u64 heavy[2];     // binned scheduler: heavy particles per lepton species
    u64 queue[2];     // binned scheduler: next unclaimed entry of each work queue
    u64 particles[3]; // cumulative particle-steps per species
    u64 steps;
    // Counters updated by atomics from every block sit on their own 128-byte lines
    // so that the L2 serves them in parallel.
    alignas(128) u64 substeps[3];  // cumulative particle-sub-steps per species
    alignas(128) u64 heavy_particles;  // cumulative work of the heavy-queue kernel
    alignas(128) u64 heavy_substeps;
    alignas(128) u64 sampled_photons;  // cumulative work of the photon sampling pass
    alignas(128) u64 sampled_substeps;
    alignas(128) u64 emissions;
    alignas(128) u64 pairs;
    alignas(128) u64 clips;
    alignas(128) u64 capped;
    alignas(128) u64 nonfinite;
    alignas(128) u64 learned_events;   // surrogate sampler
    alignas(128) u64 fallback_events;
    alignas(128) u64 fallback_draws;
    alignas(128) u64 envelope_clips;
    alignas(128) u64 pair_learned;     // photon optical-depth path: energy splits
    alignas(128) u64 pair_fallback;    // from the network / by rejection, the
    alignas(128) u64 pair_fallback_draws;  // candidates used and those above the
    alignas(128) u64 pair_envelope_clips;  // envelope
    alignas(128) u64 chi_guard;    // float chi sub-steps recomputed in double (cancellation)
    alignas(128) u64 max_p_bits;   // largest acceptance probability (bits of a non-negative double)
    alignas(128) u64 status_bits;  // bit 0: capacity exceeded, bit 1: non-finite input
    u64 required[3];  // largest count requested per species (capacity errors)
    u64 lo[3], hi[3]; // slots of the current pass: [0, n0) in the main pass; the
                      // particles appended by the previous pass in a cascade pass
    uint32_t hist[2][kBins];    // per-bin counts of the current step
    uint32_t offset[2][kBins];  // start of each heavy bin in the work queue
    uint32_t cursor[2][kBins];  // fill position inside each bin
};

struct SpeciesDev {
    u64 *n;
    u64 cap;
    double *x, *y, *z;
    void *ux, *uy, *uz, *w;
    uint64_t *id, *parent;
    uint32_t *events;
    double *tau;
    double *birth;  // cascades: time within the step at which each new particle was born
};

struct FieldDev {
    const void *ex, *ey, *ez, *bx, *by, *bz;
    u64 stride;
};

// Sub-steps chosen per cell: the node cells [x0 + i dx, x0 + (i + 1) dx) x ... of a
// periodic grid and one count per cell for each group (0: electrons and positrons,
// 1: photons), rebuilt at every step start.
struct CellDev {
    uint32_t *n[2];        // null: every particle takes its own count
    uint32_t *slot[3];     // per slot of each species: 1 + its cell's index, 0: none
    uint32_t nx, ny, nz;
    double x0, y0, z0, dx, dy, dz;
};

struct StepArgs {
    SpeciesDev sp[3];  // electrons, positrons, photons
    FieldDev fl[3];
    DevState *st;
    double dt, p_max, pair_coef;
    double p_max_lep;      // sub-step bound target of the leptons (p_max, or the surrogate's)
    uint64_t seed;
    uint32_t step, max_sub;
    int emission, pairs;   // which algorithms run in this step
    uint32_t light_max;    // binned scheduler: largest N handled by the light pass
    uint32_t chunk;        // binned scheduler: queue entries claimed per wave (multiple of 64)
    uint32_t resolve_batch;  // surrogate: waiting emissions that trigger a batched resolve (1..64)
    uint32_t prepass_finish; // binned: the pre-pass finishes particles of one quiet sub-step
    uint32_t bins_per_octave; // binned: sub-step-count bins per octave (4..kMaxBinsPerOctave)
    uint32_t light_tile;     // binned: slots per wave tile of the light pass (64..512, a multiple of 64)
    uint32_t tiled_slots;    // tiled: slots per wave tile (64..256, a multiple of 64)
    uint8_t *alive;        // photon flags, one per slot: 0 decayed, 1 alive
    u64 *dead_idx;         // slots of the photons that decayed this step
    u64 *hole_idx;         // compaction lists
    u64 *mover_idx;
    uint32_t *nsub[2];     // binned scheduler: sub-step count per lepton slot (0: skipped)
    uint32_t *queue[2];    // binned scheduler: heavy lepton slots sorted by bin, heaviest first
    int sampler;           // 0 rejection, 1 surrogate
    const MlpModel *model; // surrogate: installed network (nullptr: rejection for every chi)
    const MlpModel *pair_model;  // photon path: network of the energy split (nullptr: rejection)
    uint32_t gen;          // 0: main pass; g >= 1: cascade pass g over DevState's lo..hi,
                           // each particle starting at its birth time
    uint32_t *step_dev;    // non-null: the step number is *step_dev (k_end increments it)
    u64 *gap_hist;         // non-null: event-gap histograms [2][gap_bins] (emissions, pairs)
    uint32_t gap_bins;
    CellDev cells;         // sub-steps per cell (cells.n[0] null: per particle)
};

// Event-gap diagnostic: one more event whose particle had gap sub-steps since its
// previous event in the step (or since the step start); gaps >= bins go to the last bin.
__device__ __forceinline__ void count_gap(const StepArgs &a, int kind, uint32_t gap) {
    if (a.gap_hist) atomicAdd(&a.gap_hist[kind * a.gap_bins + (gap < a.gap_bins ? gap : a.gap_bins - 1)], 1ull);
}

// The step number of the random streams and child ids.
__device__ __forceinline__ uint32_t step_of(const StepArgs &a) { return a.step_dev ? *a.step_dev : a.step; }

// Kernels, in launch order, and the standalone synchrotron kernel.
enum KernelId {
    K_BEGIN = 0,
    K_PHOTON,   // Algorithm 2 for all photons
    K_LEPTON,   // naive scheduler: one lane per lepton
    K_PREPASS,  // binned scheduler: sub-step counts and histogram
    K_SCAN,
    K_SCATTER,
    K_LIGHT,
    K_HEAVY,
    K_END,
    K_FILL,
    K_MOVE,
    K_SYNCHROTRON,
    K_TILED,    // tile-sorted scheduler: the whole lepton pass
    K_GEN,      // cascades: advance the pass ranges to the particles of the previous pass
    K_PHOTON_SURR,  // photon optical-depth path
    K_CELL_CLEAR,   // sub-steps per cell: clear the per-cell counts
    K_CELL_MAX,     // sub-steps per cell: largest own count of each group in each cell
    K_COUNT
};

// Enqueue one kernel of a step (precision: 0 = F64, 1 = MIXED).  blocks is the
// grid size in x; lepton kernels add y = 2 (one row per lepton species).
hipError_t launch_kernel(int id, const StepArgs &a, int precision, int blocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Training of the surrogate sampler's network.
// ---------------------------------------------------------------------------
// CDF of the emitted energy over x in [0, 1] on a grid of chi: row c (chi =
// 10^(lo10 + c (hi10 - lo10) / (nchi - 1))) holds nx + 1 values at
// x = 1 - (1 - k/nx)^2; total[c] is the integral of eq. (1) over c b.
struct CdfTableDev {
    double *cdf;
    double *total;
    int nchi, nx;
    double lo10, hi10;
    int kind;  // 0: emission, rows over x = 1 - (1 - k/nx)^2; 1: pair creation, rows of
               // the half-distribution H(D) = P(|d - 1/2| <= D) over D = k / (2 nx)
};

struct Sample {
    float s, v, y, w;  // network inputs, target output, loss weight
};

struct TrainArgs {
    const float *params;   // float parameters (kMlpParams)
    const Sample *batch;   // blocks * 4 waves * tiles * 16 samples
    float *partials;       // [blocks][kMlpParams + 1]: gradient sums and the loss
    uint32_t tiles;        // 16-sample tiles per wave
    float inv_batch;       // 1 / batch size
};

struct ReduceArgs {
    const float *partials;
    int blocks;
    float *params, *m, *v;  // Adam state (unused when grad_out is set)
    float *grad_out;        // non-null: write the summed gradient, no update
    float *loss_out;        // optional: the summed loss
    float lr, beta1, beta2, eps, c1, c2;  // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
};

hipError_t launch_rate(const float *chi, float *out, u64 n, int blocks, hipStream_t s);
hipError_t launch_pair_rate(const float *chi, float *out, u64 n, int blocks, hipStream_t s);
hipError_t launch_cdf_table(const CdfTableDev &t, hipStream_t s);
hipError_t launch_mlp_data(const CdfTableDev &t, Sample *out, u64 n, uint64_t seed, uint32_t step,
                           double lo10, double hi10, int blocks, hipStream_t s);
hipError_t launch_mlp_train(const TrainArgs &ta, int blocks, hipStream_t s);
hipError_t launch_mlp_reduce(const ReduceArgs &ra, hipStream_t s);
hipError_t launch_mlp_pack(const float *params, MlpModel *out, hipStream_t s);
hipError_t launch_mlp_validate(const MlpModel *model, const CdfTableDev &t, int nbins, int per_bin,
                               float *bin_err, hipStream_t s);
hipError_t launch_mlp_infer(const MlpModel *model, const float *chi, const float *u, float *x, u64 n,
                            int blocks, hipStream_t s, int kind = 0);

// ---------------------------------------------------------------------------
// Grid coupling (qed_grid.hip).
// ---------------------------------------------------------------------------
struct GridDev {
    const void *f[6];               // Ex, Ey, Ez, Bx, By, Bz (gather only)
    uint32_t nx, ny, nz;
    double x0, y0, z0, idx, idy, idz;  // origin and inverse cell sizes
};

struct GatherArgs {
    const u64 *n;
    u64 cap;
    const double *x, *y, *z;
    void *out[6];                   // per-slot Ex .. Bz
};

struct DepositArgs {
    const u64 *n;
    u64 cap;
    const double *x, *y, *z;
    const void *ux, *uy, *uz, *w;
    double charge;
    double *j[3];                   // Jx, Jy, Jz on the E lattices
};

// Scratch and geometry of the tile-sorted deposition.
constexpr uint32_t kDepTileEdge = 4;            // node cells per tile edge
constexpr uint32_t kDepPart = 2048;             // particles of one tile summed by one block
constexpr uint32_t kDepStage = 3 * 6 * 6 * 6;   // doubles staged per part
constexpr uint32_t kBinLdsTiles = 4096;         // up to this many tiles counted in LDS
constexpr uint32_t kDepMaxTiles = 1u << 18;     // beyond: the wave-run kernel
// parts a deposit of cap slots over ntiles tiles can need
inline u64 dep_max_parts(u64 cap, u64 ntiles) { return ntiles + (cap + kDepPart - 1) / kDepPart; }
// One particle of the tile-sorted deposition: one cache line.
struct alignas(64) DepRecord {
    double ph[3];                   // fractions within the node cell along x, y, z
    double cur[3];                  // current density components x, y, z
    uint32_t local;                 // node within its tile (x + 4 y + 16 z)
    uint32_t pad[3];
};
static_assert(sizeof(DepRecord) == 64, "one record per cache line");

struct DepSortArgs {
    const u64 *n;
    u64 cap;                        // slots
    const double *x, *y, *z;
    const void *ux, *uy, *uz, *w;
    double charge;
    double *j[3];
    uint32_t tiles[3], ntiles;      // tiles per axis, their product
    u64 max_parts;                  // dep_max_parts(cap, ntiles): blocks of k_dep_accum
    uint32_t *count;                // ntiles, zero on entry and on exit
    uint32_t *off;                  // ntiles + 1: first record of each tile, total
    uint32_t *part_off;             // ntiles + 1: first part of each tile, total
    uint32_t *part_tile;            // max_parts: tile of each part
    uint32_t *pos;                  // per slot: rank in its tile (~0u: off the grid)
    DepRecord *rec;                 // cap records in tile order
    double *stage;                  // kDepStage per part: the part's summed region
};

// dtype: 0 = float, 1 = double (the context's momentum and field type).
hipError_t launch_gather(const GridDev &g, const GatherArgs &a, int dtype, int blocks, hipStream_t s);
hipError_t launch_deposit(const GridDev &g, const DepositArgs &a, int dtype, int blocks, hipStream_t s);
hipError_t launch_deposit_sorted(const GridDev &g, const DepSortArgs &a, int dtype, int blocks, hipStream_t s);

// Enqueue the elementwise synchrotron kernel (dtype: 0 = float, 1 = double).
hipError_t launch_synchrotron(const void *x, void *F, void *G, u64 n, int dtype, DevState *st,
                              int blocks, hipStream_t s);

}  // namespace qed
