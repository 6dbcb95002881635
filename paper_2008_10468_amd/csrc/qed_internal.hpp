// Internal interface between the C ABI (qed_capi.hip) and the kernels
// (qed_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qed {

typedef unsigned long long u64;

// Per-context device state: step bookkeeping and cumulative counters.
struct DevState {
    u64 n0[3];        // live counts at step start (clamped to capacity)
    u64 dead;         // photons that decayed in this step
    u64 ntot;         // photon count after appends (clamped), before compaction
    u64 S;            // photon count after compaction
    u64 holes;        // compaction: holes found in [0, S)
    u64 movers;       // compaction: survivors found in [S, ntot)
    u64 substeps[3];  // cumulative particle-sub-steps per species
    u64 particles[3]; // cumulative particle-steps per species
    u64 emissions, pairs, clips, capped, nonfinite, steps;
    u64 max_p_bits;   // largest acceptance probability (bits of a non-negative double)
    u64 status_bits;  // bit 0: capacity exceeded, bit 1: non-finite input
    u64 required[3];  // largest count requested per species (capacity errors)
};

struct SpeciesDev {
    u64 *n;
    u64 cap;
    double *x, *y, *z;
    void *ux, *uy, *uz, *w;
    uint64_t *id, *parent;
    uint32_t *events;
};

struct FieldDev {
    const void *ex, *ey, *ez, *bx, *by, *bz;
    u64 stride;
};

struct StepArgs {
    SpeciesDev sp[3];  // electrons, positrons, photons
    FieldDev fl[3];
    DevState *st;
    double dt, p_max, pair_coef;
    uint64_t seed;
    uint32_t step, max_sub;
    int emission, pairs;  // which algorithms run in this step
    uint8_t *alive;     // photon flags, one per photon slot
    u64 *hole_idx;      // compaction lists
    u64 *mover_idx;
};

// Kernels of one step, in launch order, and the standalone synchrotron kernel.
enum KernelId { K_BEGIN = 0, K_PHOTON, K_LEPTON, K_END, K_FILL, K_MOVE, K_SYNCHROTRON, K_COUNT };

// Enqueue one kernel of a step (precision: 0 = F64, 1 = MIXED).
hipError_t launch_kernel(int id, const StepArgs &a, int precision, int blocks, hipStream_t s);

// Enqueue the elementwise synchrotron kernel (dtype: 0 = float, 1 = double).
hipError_t launch_synchrotron(const void *x, void *F, void *G, u64 n, int dtype, DevState *st,
                              int blocks, hipStream_t s);

}  // namespace qed
