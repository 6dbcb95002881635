/*
 * qed.h -- C ABI of the MI355X (gfx950) QED event generator.
 *
 * The library implements the particle-push stage of a QED-PIC step as described by
 * Volokitin et al., "Optimized routines for event generators in QED-PIC codes"
 * (arXiv:2008.10468): for every electron and positron Algorithm 1 (adaptive
 * sub-stepping, Boris push, photon emission with probability density eq. (1)), and
 * for every photon Algorithm 2 (straight-line motion, pair creation with density
 * eq. (2)); the number of sub-steps per particle follows the upper bounds f(b) of
 * Sec. 3.1.1 and the target per-sub-step probability P_max; the synchrotron
 * functions F(x) = x int_x^inf K_{5/3} and G(x) = x K_{2/3} of Sec. 3.2.1 are
 * evaluated from piecewise polynomial fits.
 *
 * Conventions (all entry points):
 *   - Units: time in hbar/(m c^2), lengths in hbar/(m c), E and B in units of the
 *     Schwinger field, lepton momenta u = p/(m c), photon momenta k = hbar k/(m c).
 *   - Pointers inside qed_species / qed_field and the x/F/G arrays of
 *     qed_synchrotron are DEVICE pointers owned by the caller; the library never
 *     frees or reallocates them.  The library owns its own scratch from qed_init
 *     to qed_finalize.
 *   - Work is enqueued on the stream given in qed_config and returns without
 *     waiting; qed_sync waits and reports errors detected on the device.
 *   - Every function returns a qed_status; nothing throws across the ABI.
 *     Arguments are validated before any device work; on QED_ERR_INVALID_ARG
 *     nothing was enqueued.
 *   - A context is bound to one device and one stream and is not thread-safe.
 */
#ifndef QED_H
#define QED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QED_API __attribute__((visibility("default")))

typedef enum qed_status {
    QED_OK = 0,
    QED_ERR_INVALID_ARG = -1, /* bad argument; nothing was enqueued */
    QED_ERR_CAPACITY = -2,    /* appends exceeded a species' capacity (see qed_report) */
    QED_ERR_NONFINITE = -3,   /* non-finite input; affected particles/values skipped */
    QED_ERR_HIP = -4,         /* a HIP runtime call failed */
    QED_ERR_STATE = -5,       /* call not valid in the context's current state */
    QED_ERR_SCRATCH = -6      /* qed_step_static: a capacity above QED_STATIC_MAX_SLOTS */
} qed_status;

typedef enum qed_dtype { QED_F32 = 0, QED_F64 = 1 } qed_dtype;

/* QED_PREC_F64: every quantity in double precision (53-bit uniforms, one Philox
 *   block per sub-step).
 * QED_PREC_MIXED: momenta, weights, fields, push and synchrotron functions in
 *   float; positions, the sub-step count and length, and the start-of-step chi in
 *   double (24-bit uniforms, one Philox block per two sub-steps). */
typedef enum qed_precision { QED_PREC_F64 = 0, QED_PREC_MIXED = 1 } qed_precision;

/* How a lepton decides when it emits and with which energy.
 * QED_SAMPLER_REJECTION: Algorithm 1 as printed, one candidate (x, y) per sub-step
 *   accepted against eq. (1).
 * QED_SAMPLER_SURROGATE: the same sub-steps and push, but the emission time comes
 *   from the optical depth: each sub-step subtracts W(chi, gamma) sub_t from the
 *   particle's remaining optical depth tau (accumulated in double), with the total
 *   rate W = int_0^1 eq. (1) dx per unit time from a fit; when tau reaches zero
 *   the particle emits and draws tau = -ln(u').  The energy fraction comes from
 *   the learned inverse CDF of eq. (1) set by qed_sampler_set, or, for chi outside
 *   its range or in a bin flagged as not accurate enough, from rejection sampling
 *   of eq. (1) at that chi.  Statistically equivalent to Algorithm 1, not
 *   particle-by-particle identical.  QED_PREC_MIXED only. */
typedef enum qed_sampler { QED_SAMPLER_REJECTION = 0, QED_SAMPLER_SURROGATE = 1 } qed_sampler;

/* Scheduling of the per-particle work (results are identical for both). */
typedef enum qed_scheduler {
    QED_SCHED_NAIVE = 0,  /* one lane per particle in buffer order */
    QED_SCHED_BINNED = 1, /* sub-step-count binned persistent work queue */
    QED_SCHED_TILED = 2   /* one pass: each wave sorts tiles of 256 consecutive particles
                             by sub-step count in LDS and runs them in that order */
} qed_scheduler;

/* One particle species, structure of arrays.  Slot i of every array belongs to
 * the same particle.  Momenta and weights are float for QED_PREC_MIXED and
 * double for QED_PREC_F64. */
typedef struct qed_species {
    uint64_t *n;        /* device: live count; read at step start, advanced by appends */
    uint64_t capacity;  /* slots available in every array */
    double *x, *y, *z;  /* positions */
    void *ux, *uy, *uz; /* u = p/(m c) for e-/e+, k = hbar k/(m c) for photons */
    void *w;            /* macro-particle weight */
    uint64_t *id;       /* unique particle id; keys the particle's random stream */
    uint64_t *parent;   /* optional (NULL): id of the parent, written for new particles */
    uint32_t *events;   /* optional (NULL): events of each pre-existing particle in the
                           last step (emissions of a lepton; 1 if a photon decayed) */
    double *tau;        /* optical depth left until the next event: electrons and
                           positrons with sampler QED_SAMPLER_SURROGATE, photons with
                           pair_sampler QED_SAMPLER_SURROGATE (required there, ignored
                           otherwise); a value <= 0 or NaN makes the particle draw a
                           fresh one.  Particles the library creates get -1, and the
                           value moves with a photon when the buffer is compacted. */
    double *birth;      /* with cascade_generations > 0 (required there, ignored
                           otherwise): written for every particle appended in a step,
                           the time within the step (0 .. dt) at which it was created,
                           and kept with the particle when the photon buffer is
                           compacted; read for the particles of each cascade pass.
                           Slots of particles present at the step start are neither
                           read nor written. */
} qed_species;

typedef struct qed_particles {
    qed_species electrons, positrons, photons;
} qed_particles;

/* Field seen by a species, frozen for the step (interpolated by the caller).
 * stride 0: one value for every particle; stride 1: one value per particle slot.
 * Same float/double type as the momenta. */
typedef struct qed_field {
    const void *ex, *ey, *ez, *bx, *by, *bz;
    uint64_t stride;
} qed_field;

typedef struct qed_config {
    int device;             /* HIP device ordinal */
    void *stream;           /* hipStream_t (NULL: the null stream) */
    int precision;          /* qed_precision */
    double p_max;           /* target event probability per sub-step, in (0, 1]; 0.01 */
    int emission;           /* run Algorithm 1 on electrons and positrons */
    int pairs;              /* run Algorithm 2 on photons */
    int scheduler;          /* qed_scheduler */
    double pair_bound_coef; /* coefficient of the pair bound f = coef c b; 0.1 */
    uint32_t max_substeps;  /* cap on sub-steps per particle and step; 1 << 24 */
    int sampler;            /* qed_sampler; QED_SAMPLER_REJECTION */
    uint32_t cascade_generations; /* in-step cascades (Sec. 2.2: the sub-stepping lets
                           a cascade of events develop inside one time step): after the
                           main pass, this many passes in which the particles created by
                           the previous pass run Algorithms 1 and 2 over the rest of the
                           step, from their birth time to dt.  0 (default): new particles
                           first act in the next step.  > 0 needs QED_SAMPLER_REJECTION,
                           the birth array of every species and stride-0 fields (one
                           field for every particle: the library has no field for a new
                           slot); the cascade passes use the one-lane-per-particle
                           kernels whatever the scheduler.  At most 64. */
    double surrogate_p_max; /* QED_SAMPLER_SURROGATE: target of the lepton sub-step bound
                           (as p_max, which pair creation keeps), in (0, 1]; 0.1.  The
                           optical depth gives the emission law at any sub-step length;
                           the sub-steps resolve the change of chi along the path.  The
                           emissions of a sub-step happen at its end: each draws the next
                           optical depth, the rest of the sub-step's integrated rate counts
                           against it, and while it is still crossed the particle emits
                           again, so no emission is lost or deferred. */
    int pair_sampler;       /* qed_sampler for pair creation; QED_SAMPLER_REJECTION:
                           Algorithm 2 with sub-steps.  QED_SAMPLER_SURROGATE (mixed
                           precision, no cascades; photons need tau): in the frozen field
                           of a step a photon's chi and energy are constant, so with the
                           total rate W = alpha (chi / eps) T(chi) (eq. (2) integrated over
                           the energy split, a fit) it decays at t = tau / W if that falls
                           inside the step, else tau -= W dt; no sub-steps.  The split is
                           drawn from eq. (2) at that chi by rejection.  Photons then run
                           one pass with no sub-step loop. */
} qed_config;

/* Errors and counts observed on the device since the previous qed_sync. */
typedef struct qed_report {
    int32_t status;                /* QED_OK, QED_ERR_CAPACITY or QED_ERR_NONFINITE */
    int32_t pad;
    uint64_t required_capacity[3]; /* e-, e+, photons: slots the last step needed */
    uint64_t nonfinite;            /* particles skipped for non-finite input */
    uint64_t n[3];                 /* live counts now */
} qed_report;

/* Cumulative counters since qed_init or qed_reset_stats. */
typedef struct qed_stats {
    uint64_t steps;
    uint64_t substeps[3]; /* particle-sub-steps of e-, e+, photons */
    uint64_t particles[3];/* particle-steps (particles processed, summed over steps) */
    uint64_t heavy_particles, heavy_substeps; /* part of the above run by the heavy-queue
                                                 kernel of the binned scheduler */
    uint64_t sampled_photons, sampled_substeps; /* photons (and their sub-steps) that ran
                                                   the pair sampling loop; the others
                                                   could not decay and only moved */
    uint64_t emissions;   /* photons emitted */
    uint64_t pairs;       /* photons that decayed into pairs */
    uint64_t clips;       /* sub-steps whose acceptance probability exceeded 1 */
    uint64_t capped;      /* particle-steps whose sub-step count hit max_substeps */
    double max_p;         /* largest acceptance probability evaluated (a sub-step whose
                             test value lies above a cheap bound of it is rejected
                             without evaluating it) */
    uint64_t learned_events;  /* surrogate: energies drawn from the learned inverse CDF */
    uint64_t fallback_events; /* surrogate: energies drawn by rejection */
    uint64_t fallback_draws;  /* surrogate: candidates those rejections used */
    uint64_t envelope_clips;  /* surrogate: candidates above the rejection envelope */
    uint64_t pair_learned;    /* photon optical-depth path: energy splits from the network, */
    uint64_t pair_fallback;   /* by rejection, */
    uint64_t pair_fallback_draws;  /* the candidates those rejections used */
    uint64_t pair_envelope_clips;  /* and the candidates above the envelope */
    uint64_t chi_guard;       /* mixed precision: lepton sub-steps whose chi was recomputed in
                                 double because its float form would cancel (crossed fields,
                                 momentum along E x B; chi as defined beside eq. (1)) */
} qed_stats;

typedef struct qed_ctx qed_ctx;

/* Fill *cfg with the defaults listed in qed_config. */
QED_API qed_status qed_config_default(qed_config *cfg);

/* Create a context: selects cfg->device, allocates the library's scratch and
 * uploads the coefficient tables.  INVALID_ARG for a bad configuration. */
QED_API qed_status qed_init(qed_ctx **ctx, const qed_config *cfg);

/* One global step of length dt (> 0) for all species (Algorithms 1 and 2,
 * Sec. 2.2 and 3.1).  fields[0..2] are the fields seen by electrons, positrons
 * and photons.  Particles created in this step (photons from emission, pairs)
 * are appended after the live particles and first act in the next step, or,
 * with cascade_generations > 0, in the cascade passes of this step.
 * Photons that decay are removed; the order of the photon buffer may change.
 * The random stream of a particle is keyed by (seed, id, step, sub-step), so
 * results do not depend on buffer order or scheduling.  Asynchronous: errors
 * on the device (capacity, non-finite input) are reported by qed_sync.  On
 * QED_ERR_CAPACITY the buffers' contents are unspecified; retrying the step
 * from the caller's copy with larger buffers reproduces the same result. */
QED_API qed_status qed_step(qed_ctx *ctx, qed_particles *p, const qed_field fields[3], double dt,
                            uint64_t seed, uint32_t step);

/* qed_step with a device-side step counter (the random streams are keyed by the
 * step number, Sec. 2.2's per-particle draws): step is a DEVICE pointer to one
 * uint32; the step reads its number there when it runs and adds one at its end.
 * A graph that records one such call (qed_graph_*) and is replayed K times thus
 * runs steps s, s+1, ..., s+K-1, as K eager qed_step calls would.  The caller
 * owns the counter; NULL: QED_ERR_INVALID_ARG.  Otherwise as qed_step. */
QED_API qed_status qed_step_counted(qed_ctx *ctx, qed_particles *p, const qed_field fields[3], double dt,
                                    uint64_t seed, uint32_t *step);

/* Largest capacity per species that qed_step_static serves (its per-slot scratch,
 * 53 MiB per GPU, held from the library's first qed_init on that GPU until the
 * process ends). */
#define QED_STATIC_MAX_SLOTS (1u << 20)

/* qed_step for callers that cannot allocate device memory or wait on the host
 * inside the call: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Identical results to qed_step (the same kernels);
 * differences:
 *   - the per-slot scratch of the step (photon flags, the dead list and the
 *     compaction lists; the binned scheduler's sub-step counts and queues; the
 *     per-slot cell records of qed_substep_cells) lives in one static device
 *     array per GPU instead of context buffers, so the call never allocates,
 *     frees or synchronises;
 *   - every species whose scratch the step uses (photons when pairs run, e- and
 *     e+ with the binned scheduler, all species with sub-steps per cell) must have
 *     capacity <= QED_STATIC_MAX_SLOTS, else QED_ERR_SCRATCH and nothing is
 *     enqueued;
 *   - the array is shared by every context and stream on one GPU and keeps the
 *     last call's contents: calls that overlap in time on one GPU race (order
 *     them on one stream, or with events).
 * The context (qed_init) and any network or cell geometry (qed_sampler_set,
 * qed_substep_cells) must be set up beforehand; those calls allocate.  Other
 * errors as qed_step. */
QED_API qed_status qed_step_static(qed_ctx *ctx, qed_particles *p, const qed_field fields[3], double dt,
                                   uint64_t seed, uint32_t step);

/* Wait for the context's stream; fill *rep (may be NULL) and return its status.
 * Clears the sticky device status. */
QED_API qed_status qed_sync(qed_ctx *ctx, qed_report *rep);

/* Elementwise synchrotron functions F(x) = x int_x^inf K_{5/3}(t) dt and
 * G(x) = x K_{2/3}(x) (Sec. 3.2.1) for n values of type dtype.  F or G may be
 * NULL.  x = 0 gives 0; large x underflows to 0; x < 0 or NaN gives NaN and
 * counts as non-finite input (reported by qed_sync).  Relative error against
 * the exact functions: about 3e-7 (float) and 1e-14 (double) while the result
 * is a normal number. */
QED_API qed_status qed_synchrotron(qed_ctx *ctx, const void *x, void *F, void *G, uint64_t n,
                                   int dtype);

QED_API qed_status qed_get_stats(qed_ctx *ctx, qed_stats *out);
QED_API qed_status qed_reset_stats(qed_ctx *ctx);

/* Launch shape of the kernels (the autotuner's search space).  Results never
 * depend on it: random numbers are keyed by particle, not by lane. */
typedef struct qed_tuning {
    uint32_t lepton_blocks_per_cu; /* grid of the naive lepton kernel and the light pass, in
                                      256-thread blocks per CU (1..1024; no grid exceeds one
                                      thread per particle slot) */
    uint32_t heavy_blocks_per_cu;  /* persistent heavy-queue kernel, blocks per CU (1..64) */
    uint32_t photon_blocks_per_cu; /* photon kernel, blocks per CU (1..1024) */
    uint32_t light_max;            /* binned scheduler: particles with at most this many
                                      sub-steps run in tiles sorted by sub-step count; the
                                      rest go through the global heavy queue (0: every
                                      particle the pre-pass did not finish goes through the
                                      queue, and the tile pass is not launched) */
    uint32_t chunk;                /* binned scheduler: queue entries a wave claims at once
                                      (a multiple of 64, >= 64) */
    uint32_t resolve_batch;        /* surrogate sampler: emissions a wave lets wait before it
                                      resolves them together (1..64; results do not depend
                                      on it) */
    uint32_t prepass_blocks_per_cu; /* binned scheduler: grid of the pre-pass (1..1024) */
    uint32_t prepass_finish;       /* binned scheduler, 0 or 1: the pre-pass itself finishes
                                      particles whose step is a single sub-step without an
                                      event, instead of the light pass reading them again
                                      (results do not depend on it) */
    uint32_t scatter_blocks_per_cu; /* binned scheduler: grid of the pass that places the heavy
                                      particles into their bins (1..1024; each block reserves
                                      its share of every bin it holds with one atomic add) */
    uint32_t bins_per_octave;      /* binned scheduler: sub-step-count bins per octave of N
                                      (4..32; the heavy queue is ordered by bin, so finer bins
                                      give the lanes of a wave closer counts) */
    uint32_t light_tile;           /* binned scheduler: slots per wave tile of the light pass
                                      (64..512, a multiple of 64) */
    uint32_t tiled_slots;          /* tiled scheduler: slots per wave tile (64..256, a multiple
                                      of 64) */
    uint32_t deposit_sort_min;     /* qed_deposit sorts the particles by grid tile (4^3 cells)
                                      and sums dense tiles in LDS when the species' capacity
                                      is at least this (0: always; 0xffffffff: never, every
                                      call adds per wave of 64 particles); results agree up to
                                      the order of the additions */
} qed_tuning;

/* Read / replace the context's launch shape; INVALID_ARG if a field is out of range. */
QED_API qed_status qed_get_tuning(qed_ctx *ctx, qed_tuning *out);
QED_API qed_status qed_set_tuning(qed_ctx *ctx, const qed_tuning *t);

/* Per-kernel timing of the library's own launches, for measurement: while
 * enabled, every kernel the context enqueues is bracketed by two HIP events on
 * the context's stream.  qed_profile_read waits for the stream, writes one entry
 * per kernel that ran since the last read (at most max entries; *count gets the
 * number written) and clears the record.  name points to a static string. */
typedef struct qed_kernel_time {
    const char *name;
    uint64_t launches;
    double total_ms;
} qed_kernel_time;

QED_API qed_status qed_profile_enable(qed_ctx *ctx, int on);
QED_API qed_status qed_profile_read(qed_ctx *ctx, qed_kernel_time *out, int max, int *count);

/* Graph capture of whole steps.  Between qed_graph_begin and qed_graph_end the
 * work enqueued by qed_step on the context's stream is recorded into a HIP graph
 * instead of being run; qed_graph_launch replays it (all recorded steps, with the
 * arguments they were recorded with: buffers, counts pointers, dt, seed, step).
 * The context's stream must be a created stream (not the null stream), and the
 * scratch must already fit the buffers (run one qed_step eagerly first):
 * otherwise QED_ERR_STATE.  Counts stay on the device, so recorded steps handle
 * any number of particles up to the recorded capacities. */
typedef struct qed_graph qed_graph;
QED_API qed_status qed_graph_begin(qed_ctx *ctx);
QED_API qed_status qed_graph_end(qed_ctx *ctx, qed_graph **out);
QED_API qed_status qed_graph_launch(qed_ctx *ctx, qed_graph *g);
QED_API void qed_graph_destroy(qed_graph *g);

/* Learned inverse CDF of the emitted energy (the surrogate sampler's model).
 * Network: inputs s = 2 (log10 chi - lo) / (hi - lo) - 1 and v = (-ln(1 - u))^(1/3) - 1; three
 * hidden layers of 64 units with activation a(t) = t / sqrt(1 + t^2); output y;
 * the candidate x = delta^(1/3) of eq. (1) is y (b / (1 + b))^(1/3), b = 3 chi / 2,
 * clamped to (0, 1).  Layer 1 (2 -> 64) and the output layer (64 -> 1) run in
 * float; the two 64 x 64 layers take bfloat16 weights and activations with float
 * accumulation (matrix cores).  params holds QED_MLP_NPARAMS floats in the order
 * W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4 (W[out][in]).
 * fallback[j] != 0 sends chi bin j (nbins bins uniform in log10 chi over [lo, hi))
 * to rejection sampling.  All pointers are HOST pointers; the model is copied. */
#define QED_MLP_HIDDEN 64
#define QED_MLP_NPARAMS 8577
#define QED_MLP_MAX_BINS 256
typedef struct qed_sampler_model {
    const float *params;
    const uint8_t *fallback;
    int32_t nbins;          /* 1 .. QED_MLP_MAX_BINS */
    int32_t pad;
    double log10_chi_lo, log10_chi_hi;
} qed_sampler_model;

/* Install (m != NULL) or remove (m == NULL: rejection for every chi) the model.
 * Stream-ordered with the context's later steps. */
QED_API qed_status qed_sampler_set(qed_ctx *ctx, const qed_sampler_model *m);

/* Energy-fraction candidates x = delta^(1/3) for n (chi, u) pairs (float DEVICE
 * arrays) as the surrogate sampler draws them with the installed model: the
 * network where it is used, else NaN (the bins that fall back to rejection). */
QED_API qed_status qed_sampler_infer(qed_ctx *ctx, const float *chi, const float *u, float *x,
                                     uint64_t n);

/* Total emission rate of the surrogate sampler: for n float values chi (DEVICE),
 * writes chi q(chi) (DEVICE) such that the probability of an emission in a
 * sub-step of length s is alpha s chi q(chi) / gamma, i.e. eq. (1) integrated
 * over the candidate x in [0, 1] (from the fit the generator uses). */
QED_API qed_status qed_emission_rate(qed_ctx *ctx, const float *chi, float *chi_q, uint64_t n);

/* Total pair-creation rate of the photon optical-depth path: for n float values
 * chi (DEVICE), writes T(chi) (DEVICE) such that a photon of energy eps decays in a
 * time s with probability alpha s (chi / eps) T(chi) for small s, i.e. eq. (2)
 * integrated over the energy split (from the fit the generator uses; 0 below
 * chi ~ 0.03, where the value underflows). */
QED_API qed_status qed_pair_rate(qed_ctx *ctx, const float *chi, float *T, uint64_t n);

/* Grid coupling: the PIC stages around the particle push (Sec. 2.1: stage 2, field
 * interpolation from the grid to the particles; stage 4, current deposition), on a
 * periodic Cartesian Yee grid of nx * ny * nz cells of size dx, dy, dz from the
 * origin (x0, y0, z0).  Arrays hold nx * ny * nz values indexed (k ny + j) nx + i;
 * each component sits at its Yee position, in cells from node (i, j, k): Ex and Jx
 * (1/2, 0, 0), Ey and Jy (0, 1/2, 0), Ez and Jz (0, 0, 1/2), Bx (0, 1/2, 1/2),
 * By (1/2, 0, 1/2), Bz (1/2, 1/2, 0).  Both stages use linear (cloud-in-cell)
 * weights on the component's lattice, periodic in every direction, computed in
 * double.  Field arrays are DEVICE pointers in the context's float type; nx, ny,
 * nz >= 1 with nx ny nz < 2^31, dx, dy, dz > 0, else QED_ERR_INVALID_ARG.
 * Stream-ordered on the context's stream, like qed_step. */
typedef struct qed_grid {
    const void *ex, *ey, *ez, *bx, *by, *bz;
    uint32_t nx, ny, nz, pad;
    double x0, y0, z0, dx, dy, dz;
} qed_grid;

/* Stage 2: E and B at every particle of the species (slots below its live count,
 * read on the device), written to out[0..5] = Ex, Ey, Ez, Bx, By, Bz (DEVICE arrays
 * of at least capacity values, the context's float type): the per-slot fields
 * (stride 1) that qed_step reads.  A particle whose position is not finite gets NaN
 * fields (qed_step then skips it as non-finite input).  The species needs n, x, y, z. */
QED_API qed_status qed_gather(qed_ctx *ctx, const qed_grid *grid, const qed_species *sp, void *const out[3 + 3]);

/* Stage 4: adds every particle's current density charge * w * u / gamma / (dx dy dz),
 * spread with the same weights, to jx, jy, jz: DEVICE double arrays on the Ex, Ey, Ez
 * lattices, in ordinary device memory such as hipMalloc returns (the sums use the
 * hardware's double atomic add, which fine-grained or host memory does not support);
 * the caller clears them, and the order of the additions, hence the last bits, may
 * vary.  charge: -1 for electrons, +1 for positrons (in units of e; the velocity is in
 * units of c).  The grid's field pointers are not used.  Particles with a non-finite
 * position, momentum or weight deposit nothing.  The species needs n, x, y, z, ux, uy,
 * uz, w.  From a capacity of qed_tuning.deposit_sort_min slots (and for grids of at most
 * 2^18 tiles of 4^3 cells) the call sorts the particles by tile, sums each tile's
 * currents in LDS and adds every grid point once, without atomic adds on the grid, in
 * scratch the context allocates on first use and keeps (about 70 bytes per slot and
 * 5 KB per tile); where that scratch cannot be had (while a graph is being recorded,
 * or out of memory) it adds per wave of particles with atomic adds instead. */
QED_API qed_status qed_deposit(qed_ctx *ctx, const qed_grid *grid, const qed_species *sp, double charge,
                               double *jx, double *jy, double *jz);

/* Event-gap diagnostic (Sec. 3.1.1, Fig. 1: how many sub-steps pass between a
 * particle's events).  hist is a DEVICE array of 2 * nbins uint64 owned by the
 * caller: [0, nbins) counts emissions (Algorithm 1), [nbins, 2 nbins) pair creations
 * (Algorithm 2) by the number of sub-steps since the particle's previous event in
 * the same step, or since the step start for its first one (1 = the next sub-step);
 * larger gaps go to the last bin.  Every following qed_step adds to it (the caller
 * clears it); NULL disables it (the default).  The optical-depth paths do not count.
 * nbins >= 2, else QED_ERR_INVALID_ARG. */
QED_API qed_status qed_event_gaps(qed_ctx *ctx, uint64_t *hist, uint32_t nbins);

/* Sub-steps chosen per cell (Algorithms 1 and 2, step 1: the sub-step is computed for
 * the current cell).  With a cell geometry set, every following qed_step first finds
 * each particle's own count N of Sec. 3.1.1 (as without cells), then runs every
 * particle with the largest N of its group in its cell: electrons and positrons form
 * one group (Algorithm 1), photons another (Algorithm 2).  Cell (i, j, k) is
 * [x0 + i dx, x0 + (i + 1) dx) x [y0 + j dy, ...) x [z0 + k dz, ...), periodic in all three
 * indices (the node cells of the qed_gather grid); a particle's cell is taken from
 * its position at the step start (exactly while |(x - x0) / dx| < 2^53 / nx).  A
 * particle with a non-finite position, momentum or field keeps its own count and
 * joins no cell.  The field pointers of cells are not used.  NULL returns to
 * per-particle counts (the default).  Needs the rejection samplers and no cascades
 * (QED_ERR_STATE otherwise, and while a graph is being recorded); INVALID_ARG for
 * nx, ny or nz < 1, nx ny nz > 2^28, cell sizes that are not positive and finite, or
 * a non-finite origin.  The library allocates 2 nx ny nz uint32 counts (HOST-side
 * geometry, copied); a graph keeps the geometry in force when it was recorded, and
 * buffers it may use stay allocated until qed_finalize. */
QED_API qed_status qed_substep_cells(qed_ctx *ctx, const qed_grid *cells);

/* The normalised CDF of eq. (1) over the candidate x, as the trainer tabulates it
 * (double, from the double fits of F and G, trapezoid rule): nchi (>= 2) values
 * of chi log-uniform over [10^lo, 10^hi], each at the nx + 1 points
 * x = 1 - (1 - k/nx)^2, k = 0..nx (nx a multiple of 256).  cdf_out (HOST, nchi
 * (nx + 1) doubles) gets the CDF rows, total_out (HOST, nchi doubles, may be NULL)
 * the integral of eq. (1) over x divided by c b.  Synchronous. */
QED_API qed_status qed_emission_cdf(qed_ctx *ctx, double log10_chi_lo, double log10_chi_hi, uint32_t nchi,
                                    uint32_t nx, double *cdf_out, double *total_out);

/* Training of the sampler's network on this GPU.  Samples: log10 chi uniform over
 * [lo, hi], u uniform, target x = CDF_chi^{-1}(u) from the table above; loss:
 * the squared error of the network output y weighted by the squared density
 * dCDF/dy at the target (so it approximates the squared CDF error); Adam with a
 * cosine-decayed step size; the batch is blocks x 4 waves x batch_tiles x 16
 * samples.  After training, every chi bin is checked on a grid of 1024 u values
 * at per_bin values of chi: the largest |CDF_chi(x(chi, u)) - u| of the packed
 * network, and bins above tolerance are flagged to fall back to rejection. */
typedef struct qed_train_config {
    double log10_chi_lo, log10_chi_hi; /* chi range of the network; -3, 2 */
    uint32_t table_chi, table_x;       /* CDF table; 1025 x 8192 */
    uint32_t steps;                    /* optimizer steps; 60000 */
    uint32_t blocks, batch_tiles;      /* batch = blocks * 64 * batch_tiles; 256, 4 */
    float lr, lr_final;                /* 1e-2 -> 3e-5 */
    uint64_t seed;                     /* data and initial weights; 1 */
    int32_t nbins, per_bin;            /* validation; 50, 5 */
    double tolerance;                  /* CDF error above which a bin falls back; 1e-3 */
    int32_t target;                    /* 0: the emitted energy (eq. (1)); 1: the energy
                                          split of pair creation (eq. (2)); 0 */
    int32_t pad;
} qed_train_config;

QED_API qed_status qed_train_config_default(qed_train_config *cfg);

/* The photon path's learned energy split (pair_sampler QED_SAMPLER_SURROGATE): a
 * network of the same shape trained with target 1 on the half-distribution of the
 * electron's fraction d about 1/2 (eq. (2) is symmetric): inputs s as above and
 * v = sqrt(-ln(1 - u')) - 1 of u' in [0, 1); output y with |d - 1/2| = y w(chi),
 * w(chi) = sqrt(3 chi / 64) / sqrt(1 + 3 chi / 16).  A decaying photon draws u,
 * takes u' = |2u - 1| and the side of 1/2 from u < 1/2.  Bins flagged to fall back,
 * and chi outside the range, use rejection against the fitted envelope.  NULL
 * removes it.  The model struct is that of qed_sampler_set; HOST pointers, copied. */
QED_API qed_status qed_pair_sampler_set(qed_ctx *ctx, const qed_sampler_model *m);

/* d for n (chi, u) (float DEVICE arrays) as the photon path draws it with the
 * installed split network; NaN where it falls back.  QED_ERR_STATE without a model. */
QED_API qed_status qed_pair_sampler_infer(qed_ctx *ctx, const float *chi, const float *u, float *d,
                                          uint64_t n);

/* Synchronous.  init_params (HOST, QED_MLP_NPARAMS floats) may be NULL for a
 * seeded initialisation.  Outputs (HOST): params_out (QED_MLP_NPARAMS), and,
 * where not NULL, loss_out (steps values), bin_err_out and fallback_out (nbins
 * values each). */
QED_API qed_status qed_train_sampler(qed_ctx *ctx, const qed_train_config *cfg, const float *init_params,
                                     float *params_out, float *loss_out, float *bin_err_out,
                                     uint8_t *fallback_out);

/* Loss and gradient of the training loss for given parameters and samples, from
 * the same kernels as training (for checks).  samples: HOST, n rows of
 * (s, v, y_target, weight), n a positive multiple of 64.  loss = (1/n) sum w (y -
 * y_target)^2.  grad_out: HOST, QED_MLP_NPARAMS.  Synchronous. */
QED_API qed_status qed_mlp_gradient(qed_ctx *ctx, const float *params, const float *samples, uint64_t n,
                                    float *loss_out, float *grad_out);

/* Release the context's scratch.  NULL is allowed. */
QED_API void qed_finalize(qed_ctx *ctx);

QED_API const char *qed_status_string(qed_status s);

#ifdef __cplusplus
}
#endif

#endif /* QED_H */
