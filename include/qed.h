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
    QED_ERR_STATE = -5        /* call not valid in the context's current state */
} qed_status;

typedef enum qed_dtype { QED_F32 = 0, QED_F64 = 1 } qed_dtype;

/* QED_PREC_F64: every quantity in double precision (53-bit uniforms, one Philox
 *   block per sub-step).
 * QED_PREC_MIXED: momenta, weights, fields, push and synchrotron functions in
 *   float; positions, the sub-step count and length, and the start-of-step chi in
 *   double (24-bit uniforms, one Philox block per two sub-steps). */
typedef enum qed_precision { QED_PREC_F64 = 0, QED_PREC_MIXED = 1 } qed_precision;

/* Scheduling of the per-particle work (results are identical for both). */
typedef enum qed_scheduler {
    QED_SCHED_NAIVE = 0, /* one lane per particle in buffer order */
    QED_SCHED_BINNED = 1 /* sub-step-count binned persistent work queue */
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
    double max_p;         /* largest acceptance probability evaluated */
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
 * are appended after the live particles and first act in the next step.
 * Photons that decay are removed; the order of the photon buffer may change.
 * The random stream of a particle is keyed by (seed, id, step, sub-step), so
 * results do not depend on buffer order or scheduling.  Asynchronous: errors
 * on the device (capacity, non-finite input) are reported by qed_sync.  On
 * QED_ERR_CAPACITY the buffers' contents are unspecified; retrying the step
 * from the caller's copy with larger buffers reproduces the same result. */
QED_API qed_status qed_step(qed_ctx *ctx, qed_particles *p, const qed_field fields[3], double dt,
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
    uint32_t lepton_blocks_per_cu; /* grid of the naive lepton kernel, the light pass and
                                      the pre-pass, in 256-thread blocks per CU (>= 1) */
    uint32_t heavy_blocks_per_cu;  /* persistent heavy-queue kernel, blocks per CU (>= 1) */
    uint32_t photon_blocks_per_cu; /* photon kernel, blocks per CU (>= 1) */
    uint32_t light_max;            /* binned scheduler: particles with at most this many
                                      sub-steps run in tiles sorted by sub-step count; the
                                      rest go through the global heavy queue (>= 1) */
    uint32_t chunk;                /* binned scheduler: queue entries a wave claims at once
                                      (a multiple of 64, >= 64) */
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

/* Release the context's scratch.  NULL is allowed. */
QED_API void qed_finalize(qed_ctx *ctx);

QED_API const char *qed_status_string(qed_status s);

#ifdef __cplusplus
}
#endif

#endif /* QED_H */
