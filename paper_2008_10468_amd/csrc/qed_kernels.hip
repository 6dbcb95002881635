// Kernels of the QED event generator for gfx950 (wave64).
//
// One global step (Sec. 2.2) is the sequence
//   k_begin    snapshot the live counts (particles appended later in the step wait
//              for the next step or a cascade pass) and clear the per-step counters;
//   k_cell_clear / k_cell_max   only with sub-steps chosen per cell: the largest
//              own sub-step count of each group in each cell, and each slot's cell;
//   k_photon   Algorithm 2 for every photon: one streaming pass moves every photon
//              and writes its end-of-step position; the photons that provably cannot
//              decay in the step are then done, the others are queued per wave in LDS
//              and sampled 64 at a time (pair creation with density eq. (2)); pairs
//              are appended to the e-/e+ buffers, the photon is flagged dead and its
//              slot is put on the dead list.  On the photon optical-depth path
//              k_photon_surr replaces it (exact decay time, no sub-steps);
//   Algorithm 1 for every electron and positron (Boris sub-steps, emission with
//   density eq. (1), recoil, photons appended), scheduled one of three ways:
//     naive:   k_lepton, one lane per particle in buffer order;
//     binned:  k_prepass computes each particle's sub-step count N and a histogram
//              over 1/16-octave bins of N; k_scan and k_scatter build a work
//              queue of the heavy particles (N > light_max) sorted by bin, heaviest
//              first; k_light runs the light particles in tiles sorted by N; k_heavy
//              is a persistent kernel whose waves claim chunks of the queue, so the
//              64 lanes of a wave carry nearly the same N;
//     tiled:   k_tiled sorts 256-slot tiles by N in LDS and runs them heaviest first;
//   each has an instance for the lepton optical-depth path (surrogate sampler);
//   cascade passes (cascade_generations > 0): k_gen, then k_photon and k_lepton over
//              the particles created by the previous pass, from their birth times;
//   k_end      clamp counts to capacity (reporting overflow), size the compaction;
//   k_fill / k_move  fill the holes left by decayed photons in [0, S) with the
//              survivors found in [S, n): both scans are O(decays).
// Children are staged per wave in LDS and appended with one atomic per flush; pairs
// take one atomic per wave and sub-step with a decay.  Random numbers are keyed by
// (seed, id, step, sub-step), so every schedule gives the same per-particle result.
// The sub-step count of a particle comes from the bounds f(b) of Sec. 3.1.1,
// evaluated in double at the step start.
#include <type_traits>

#include "qed_device.hpp"
#include "qed_internal.hpp"
#include "qed_mlp.hpp"
#include "qed_pair.hpp"
#include "qed_rate.hpp"
#include "qed_synchro.hpp"

namespace qed {

namespace {

constexpr int kBlock = 256;

// Logarithm of the smallest uniform y of each path, (2k+1) 2^-b with k = 0.
template <class R>
struct YMin;
template <>
struct YMin<float> {
    static constexpr float log = -16.6355323f;  // ln 2^-24
};
template <>
struct YMin<double> {
    static constexpr float log = -36.7368005f;  // ln 2^-53
};

// True if no candidate of this photon can be accepted in this step.  With
// d = x(1-x) <= 1/4 the argument of eq. (2) obeys z = 2/(3 chi d) >= z0 = 8/(3 chi);
// P_p = A (G(z) - d F(z)) <= A G(z) with A = alpha st sqrt(3)/(2 pi) chi/eps; G
// decreases for z > 0.42, and for z >= 1 G(z) <= sqrt(pi z/2) e^-z (1 + 7/(72 z))
// (the K_{2/3} asymptotic series truncated after its positive first correction is
// an upper bound).  If twice that bound is below the smallest uniform y, no y can
// fall under P_p: the photon only moves, exactly as sampling would leave it.
// The test runs in float in the log domain, ln(twice the bound) =
// ln(2 A sqrt(pi z0 / 2) (1 + 7 / (72 z0))) - z0, against ln y_min less a margin of
// 1e-3, far above the float rounding of these few operations; an overflow or a
// NaN answers "not quiet", and so does z0 within 1e-3 of the bound's validity
// limit.  A photon wrongly called not quiet is only sampled, which is always exact.
template <class R>
__device__ __forceinline__ bool photon_quiet(double chi, double eps, double st) {
    if (!(chi > 0.0) || !(eps > 0.0)) return true;
    const float cf = (float)chi;
    const float z0 = (8.0f / 3.0f) * __builtin_amdgcn_rcpf(cf);
    if (!(z0 >= 1.001f)) return false;
    const float A = (float)(kAlpha * kSqrt3 / (2.0 * kPi)) * (float)st * cf * __builtin_amdgcn_rcpf((float)eps);
    const float lub = __logf(2.0f * A * __builtin_amdgcn_sqrtf((float)(0.5 * kPi) * z0) *
                             (1.0f + (7.0f / 72.0f) * __builtin_amdgcn_rcpf(z0))) - z0;
    return lub < YMin<R>::log - 1e-3f;
}

__device__ __forceinline__ u64 lanemask_lt() {
    const int l = __lane_id();
    return (1ull << l) - 1ull;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <class R>
__device__ __forceinline__ bool finite3(R a, R b, R c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// Per-lane tallies, reduced once per wave at kernel end.
template <class R>
struct Tally {
    u64 substeps = 0;
    uint32_t events = 0, clips = 0, capped = 0, nonfinite = 0, particles = 0;
    uint32_t learned = 0, fallback = 0, fb_draws = 0, env_clips = 0;  // surrogate sampler
    uint32_t guard = 0;  // float chi recomputed in double (crossed-field cancellation)
    R max_p = 0;
};

// Sum over the wave, skipped (no cross-lane traffic) when the counter is zero in
// every lane, which is the common case for the rare-event counters.
template <class T>
__device__ __forceinline__ T wave_sum_nz(T v) {
    if (__ballot(v != T(0)) == 0) return T(0);
    return wave_sum(v);
}

// Block-wide reduction of NT tallies, then one atomic per non-zero counter and
// block.  Every thread of the block must call it.  work[q] of tally q: 0 = plain,
// 1 = heavy-queue kernel, 2 = photon sampling pass (their particles and sub-steps
// are also counted separately).
template <class R, int NT>
__device__ __forceinline__ void flush_tallies(const Tally<R> *tt, const int *work, DevState *st, int species) {
    constexpr int kN = 11;
    __shared__ u64 red[NT][kBlock / 64][kN + 1];
    const int wv = threadIdx.x / 64;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const Tally<R> &t = tt[q];
        const u64 v[kN] = {wave_sum_nz(t.substeps), (u64)wave_sum_nz(t.events), (u64)wave_sum_nz(t.clips),
                           (u64)wave_sum_nz(t.capped), (u64)wave_sum_nz(t.nonfinite),
                           (u64)wave_sum_nz(t.particles), (u64)wave_sum_nz(t.learned),
                           (u64)wave_sum_nz(t.fallback), (u64)wave_sum_nz(t.fb_draws),
                           (u64)wave_sum_nz(t.env_clips), (u64)wave_sum_nz(t.guard)};
        const double mp = __ballot(t.max_p > R(0)) ? wave_max((double)t.max_p) : 0.0;
        if (__lane_id() == 0) {
            for (int k = 0; k < kN; ++k) red[q][wv][k] = v[k];
            red[q][wv][kN] = (u64)__double_as_longlong(mp);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool ph = species == 2;
        for (int q = 0; q < NT; ++q) {
            u64 tot[kN] = {}, mb = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                for (int k = 0; k < kN; ++k) tot[k] += red[q][w][k];
                mb = red[q][w][kN] > mb ? red[q][w][kN] : mb;
            }
            if (tot[6]) atomicAdd(ph ? &st->pair_learned : &st->learned_events, tot[6]);
            if (tot[7]) atomicAdd(ph ? &st->pair_fallback : &st->fallback_events, tot[7]);
            if (tot[8]) atomicAdd(ph ? &st->pair_fallback_draws : &st->fallback_draws, tot[8]);
            if (tot[9]) atomicAdd(ph ? &st->pair_envelope_clips : &st->envelope_clips, tot[9]);
            if (tot[10]) atomicAdd(&st->chi_guard, tot[10]);
            if (tot[0]) atomicAdd(&st->substeps[species], tot[0]);
            if (tot[1]) atomicAdd(ph ? &st->pairs : &st->emissions, tot[1]);
            if (tot[2]) atomicAdd(&st->clips, tot[2]);
            if (tot[3]) atomicAdd(&st->capped, tot[3]);
            if (tot[4]) {
                atomicAdd(&st->nonfinite, tot[4]);
                atomicOr(&st->status_bits, 2ull);
            }
            if (work[q] == 1) {
                if (tot[5]) atomicAdd(&st->heavy_particles, tot[5]);
                if (tot[0]) atomicAdd(&st->heavy_substeps, tot[0]);
            } else if (work[q] == 2) {
                if (tot[5]) atomicAdd(&st->sampled_photons, tot[5]);
                if (tot[0]) atomicAdd(&st->sampled_substeps, tot[0]);
            }
            if (mb) atomicMax(&st->max_p_bits, mb);
        }
    }
}

template <class R>
__device__ __forceinline__ void flush_tally(const Tally<R> &t, DevState *st, int species, int work = 0) {
    const int w[1] = {work};
    flush_tallies<R, 1>(&t, w, st, species);
}

// Children of one wave staged in LDS and written out with one atomic per flush.
// A child's id (a Philox block of its parent's id and counter) is formed when the
// buffer is written out, by all the flushing lanes together, rather than by the
// few lanes that emit in one sub-step.
// Every flush is an atomic on the one counter of the species that all waves of the
// chip share.  TB: with birth times.  The optical-depth path (TB false: it runs no
// cascades) emits its photons about twice as fast as Algorithm 1's loop in a hot
// spot, and waits on those atomics, so its buffer holds 128 children (each atomic
// then covers twice the writes; 52 bytes of LDS per entry); the plain path's 64
// entries keep its LDS small at no measurable cost.
template <class R, bool TB = true>
struct ChildBuf {
    static constexpr uint32_t kCap = TB ? 64 : 128;
    double x[kCap], y[kCap], z[kCap];
    R px[kCap], py[kCap], pz[kCap], w[kCap];
    uint64_t parent[kCap];
    uint32_t ctr[kCap];        // the id's counter word (the event's index)
    double tb[TB ? kCap : 1];  // birth time within the step
    uint32_t count;
};

// Write the staged children to the species' tail.  Called by the active lanes of
// a wave (any subset); they share the writes.
template <class R, bool TB>
__device__ __forceinline__ void flush_children(ChildBuf<R, TB> &cb, const SpeciesDev &dst, uint64_t seed,
                                               uint32_t step) {
    __syncwarp();
    const uint32_t n = cb.count;
    if (n == 0) return;
    const u64 exec = __ballot(1);
    const int leader = __ffsll((long long)exec) - 1;
    const uint32_t nact = (uint32_t)__popcll(exec);
    const uint32_t me = (uint32_t)__popcll(exec & lanemask_lt());
    u64 base = 0;
    if (__lane_id() == leader) base = atomicAdd(dst.n, (u64)n);
    base = __shfl(base, leader);
    for (uint32_t e = me; e < n; e += nact) {
        const u64 slot = base + e;
        if (slot < dst.cap) {
            dst.x[slot] = cb.x[e];
            dst.y[slot] = cb.y[e];
            dst.z[slot] = cb.z[e];
            ((R *)dst.ux)[slot] = cb.px[e];
            ((R *)dst.uy)[slot] = cb.py[e];
            ((R *)dst.uz)[slot] = cb.pz[e];
            ((R *)dst.w)[slot] = cb.w[e];
            dst.id[slot] = child_id(seed, cb.parent[e], step, cb.ctr[e], 0);
            if (dst.parent) dst.parent[slot] = cb.parent[e];
            if constexpr (TB)
                if (dst.birth) dst.birth[slot] = cb.tb[e];
            if (dst.tau) dst.tau[slot] = -1.0;
        }
    }
    __syncwarp();
    cb.count = 0;
    __syncwarp();
}

// Random pair (x, y) of sub-step k.  Float path: one Philox block serves two
// sub-steps (words 0,1 for even k, 2,3 for odd k), 24-bit uniforms.  Double path:
// one block per sub-step, 53-bit uniforms from words (0,1) and (2,3).
template <class R>
struct Draw;

template <>
struct Draw<float> {
    u32x4 w;
    __device__ __forceinline__ void get(uint32_t k, uint32_t idlo, uint32_t idhi, uint32_t step,
                                        uint32_t klo, uint32_t khi, float &x, float &y) {
        if ((k & 1u) == 0u) w = philox10(idlo, idhi, step, k >> 1, klo, khi);
        const bool odd = (k & 1u) != 0u;
        x = u24(odd ? w.z : w.x);
        y = u24(odd ? w.w : w.y);
    }
};

template <>
struct Draw<double> {
    __device__ __forceinline__ void get(uint32_t k, uint32_t idlo, uint32_t idhi, uint32_t step,
                                        uint32_t klo, uint32_t khi, double &x, double &y) {
        const u32x4 w = philox10(idlo, idhi, step, k, klo, khi);
        x = u53(w.x, w.y);
        y = u53(w.z, w.w);
    }
};

// chi inside the sub-step loop.
template <int FK>
__device__ __forceinline__ float chi_sub(float ux, float uy, float uz, float g, float ex, float ey,
                                         float ez, float bx, float by, float bz, float e2, uint32_t &guard) {
    return chi_lepton_f32<FK>(ux, uy, uz, g, ex, ey, ez, bx, by, bz, e2, guard);
}
template <int FK>
__device__ __forceinline__ double chi_sub(double ux, double uy, double uz, double g, double ex,
                                          double ey, double ez, double bx, double by, double bz,
                                          double, uint32_t &) {
    return chi_def(g, ux, uy, uz, ex, ey, ez, bx, by, bz);
}

template <class R>
struct Lepton {
    R ux, uy, uz, ex, ey, ez, bx, by, bz;
};

template <class R>
__device__ __forceinline__ Lepton<R> load_lepton(const StepArgs &a, int s, u64 i) {
    const SpeciesDev &sp = a.sp[s];
    const FieldDev &fl = a.fl[s];
    const u64 f = i * fl.stride;
    Lepton<R> p;
    p.ux = ((const R *)sp.ux)[i];
    p.uy = ((const R *)sp.uy)[i];
    p.uz = ((const R *)sp.uz)[i];
    p.ex = ((const R *)fl.ex)[f];
    p.ey = ((const R *)fl.ey)[f];
    p.ez = ((const R *)fl.ez)[f];
    p.bx = ((const R *)fl.bx)[f];
    p.by = ((const R *)fl.by)[f];
    p.bz = ((const R *)fl.bz)[f];
    return p;
}

// Periodic index of the cell along one axis that holds coordinate v (cells of size
// d from o); false when (v - o) / d is not finite.  Exact while |(v - o) / d| stays
// below 2^53 / n; beyond that the index is only kept inside [0, n).
__device__ __forceinline__ bool wrap_cell(double v, double o, double d, uint32_t n, uint32_t &i) {
    const double q = (v - o) / d;
    if (!isfinite(q)) return false;
    const double f = floor(q);
    double r = f - (double)n * floor(f / (double)n);
    r = r < 0.0 ? 0.0 : (r > (double)(n - 1) ? (double)(n - 1) : r);
    i = (uint32_t)r;
    return true;
}

__device__ __forceinline__ bool cell_of(const CellDev &c, double x, double y, double z, uint32_t &cell) {
    uint32_t i, j, k;
    if (!wrap_cell(x, c.x0, c.dx, c.nx, i) || !wrap_cell(y, c.y0, c.dy, c.ny, j) ||
        !wrap_cell(z, c.z0, c.dz, c.nz, k))
        return false;
    cell = (k * c.ny + j) * c.nx + i;
    return true;
}

// Step 1 of Algorithms 1 and 2 with the sub-step chosen for the cell: the largest
// own count of the particle's group (g: 0 leptons, 1 photons) in the cell holding
// its step-start position (slot: 1 + that cell's index, as k_cell_max recorded it).
// The particle's own count when its input was not finite (own 0) or its position is
// not finite (slot 0).  The passes read the recorded cell rather than recomputing it
// from the position, which keeps the sub-step loops' register budget.
__device__ __forceinline__ uint32_t cell_nsub(const StepArgs &a, int g, uint32_t slot, uint32_t own) {
    if (own == 0 || slot == 0) return own;
    const uint32_t v = a.cells.n[g][slot - 1];
    return v > own ? v : own;
}

// Algorithm 2, step start: a photon's own sub-step count over dti.
__device__ __forceinline__ uint32_t photon_nsub(const StepArgs &a, double chi, double eps, double dti,
                                                bool *capped) {
    *capped = false;
    if (!(eps > 0.0)) return 1;
    return nsub(bound_pair(chi, eps, dti, a.pair_coef), a.p_max, a.max_sub, capped);
}

// Algorithm 1, step start: the particle's own sub-step count from the bound over the
// interval dt (double).  0 for non-finite input (the particle is left alone).
template <class R>
__device__ __forceinline__ uint32_t lepton_nsub_own(const StepArgs &a, const Lepton<R> &p, Tally<R> &tl,
                                                    double dt) {
    if (!(finite3(p.ux, p.uy, p.uz) && finite3(p.ex, p.ey, p.ez) && finite3(p.bx, p.by, p.bz))) {
        tl.nonfinite++;
        return 0;
    }
    const double gd = sqrt(1.0 + (double)p.ux * p.ux + (double)p.uy * p.uy + (double)p.uz * p.uz);
    const double chi0 = chi_def(gd, p.ux, p.uy, p.uz, p.ex, p.ey, p.ez, p.bx, p.by, p.bz);
    bool capped;
    const uint32_t N = nsub(bound_emission(chi0, gd, dt), a.p_max_lep, a.max_sub, &capped);
    tl.capped += capped;
    return N;
}

// The count lepton i of species s runs with: its own, or its cell's.
template <class R>
__device__ __forceinline__ uint32_t lepton_nsub(const StepArgs &a, int s, u64 i, const Lepton<R> &p, Tally<R> &tl,
                                                double dt) {
    const uint32_t N = lepton_nsub_own(a, p, tl, dt);
    return a.cells.n[0] ? cell_nsub(a, 0, a.cells.slot[s][i], N) : N;
}

// Photon emission of the accepting lanes (acc; m = their ballot): the photon of
// energy fraction delta = x3 along u is staged in the wave's LDS buffer with the
// parent's position and weight, and the parent recoils to gamma' = (1 - delta)
// gamma in the same direction.  Called by every lane of the wave that is still in
// the sub-step loop.  k: the sub-step (birth time t0 + (k + 1) st); ctr: the
// counter of the photon's id (the sub-step in Algorithm 1, the emission's index in
// the step for the surrogate, which can emit more than once in a sub-step).
// A lepton's position and weight at the start of the step, held for its emissions
// and its end-of-step position (the step does not change them in memory).
template <class R>
struct Origin {
    double x, y, z;
    R w;
};

template <class R>
__device__ __forceinline__ Origin<R> origin_of(const SpeciesDev &sp, u64 i) {
    return Origin<R>{sp.x[i], sp.y[i], sp.z[i], ((const R *)sp.w)[i]};
}

template <class R, bool TB>
__device__ __forceinline__ void stage_emission(const StepArgs &a, const Origin<R> &org, uint64_t pid,
                                               uint32_t ctr, uint32_t k, bool acc, u64 m, R x3, R omx3, R g,
                                               R u2, R dx,
                                               R dy, R dz, R &ux, R &uy, R &uz, ChildBuf<R, TB> &cb,
                                               uint32_t &nev, double t0, double st, uint32_t step) {
    const uint32_t c = (uint32_t)__popcll(m);
    __syncwarp();
    if (cb.count + c > ChildBuf<R, TB>::kCap) flush_children(cb, a.sp[2], a.seed, step);
    const uint32_t n0 = cb.count;
    if (acc) {
        const uint32_t e = n0 + (uint32_t)__popcll(m & lanemask_lt());
        const R umag = sqrt_(u2);
        const R inv = umag > R(0) ? rcp(umag) : R(0);
        const R eph = x3 * g * inv;
        cb.x[e] = org.x + (double)dx;
        cb.y[e] = org.y + (double)dy;
        cb.z[e] = org.z + (double)dz;
        cb.px[e] = ux * eph;
        cb.py[e] = uy * eph;
        cb.pz[e] = uz * eph;
        cb.w[e] = org.w;
        cb.ctr[e] = ctr;
        cb.parent[e] = pid;
        if constexpr (TB) cb.tb[e] = t0 + (double)(k + 1) * st;
        // gamma' = (1 - delta) gamma, same direction
        const R g1 = omx3 * g;
        const R u1 = sqrt_(fmax(g1 * g1 - R(1), R(0)));
        const R sc = u1 * inv;
        ux *= sc;
        uy *= sc;
        uz *= sc;
        nev++;
    }
    __syncwarp();
    cb.count = n0 + c;
    __syncwarp();
}

// One sub-step of Algorithm 1 after the push constants are set: Boris push and
// move, chi after the push, the candidate (x, y) of sub-step k and the acceptance
// probability of eq. (1), y < 3 x^2 P(x^3) = (c b / x) ((1 - x^3) F(z) + x^6 G(z)),
// z = x^3 / (b (1 - x^3)).  Shared by the sub-step loop and the pre-pass (which
// finishes particles of one quiet sub-step), so both round identically.
template <class R, int FK>
struct SubStep {
    R u2, g, x3, omx3, pm, y;
};

template <class R, int FK>
__device__ __forceinline__ SubStep<R, FK> substep(const Lepton<R> &p, R hex, R hey, R hez, R hq, R e2, R str, R kcb,
                                                  uint32_t k, uint32_t idlo, uint32_t idhi, uint32_t step,
                                                  uint32_t klo, uint32_t khi, Draw<R> &draw, const SynTable<R> &tab,
                                                  R &ux, R &uy, R &uz, R &dx, R &dy, R &dz, const Rot<R> &rs,
                                                  uint32_t &guard) {
    SubStep<R, FK> o;
    // push: Boris rotation and move (pure magnetic field: with the held rotation;
    // o.u2 is then not set, an emission takes |u|^2 itself)
    R ig, vs;
    if constexpr (FK == 2) {
        rotate(ux, uy, uz, rs);
        ig = rs.ig;
        o.g = rs.g;
        o.u2 = R(0);
        vs = rs.vs;
    } else {
        boris<R, FK>(ux, uy, uz, hex, hey, hez, hq, p.bx, p.by, p.bz);
        ig = inv_gamma(ux, uy, uz, o.u2);
        o.g = (R(1) + o.u2) * ig;
        vs = str * ig;
    }
    dx += ux * vs;
    dy += uy * vs;
    dz += uz * vs;
    // quantum parameter after the push (pure magnetic field: held, the rotation keeps it)
    R chi;
    if constexpr (FK == 2)
        chi = rs.chi;
    else
        chi = chi_sub<FK>(ux, uy, uz, o.g, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, e2, guard);
    // candidate x and test value y
    R x;
    draw.get(k, idlo, idhi, step, klo, khi, x, o.y);
    const R x2 = x * x;
    o.x3 = x2 * x;
    o.omx3 = (R(1) - x) * (R(1) + x + x2);
    const R b = R(1.5) * chi;
    const R z = o.x3 * rcp(b * o.omx3);
    R F, G;
    syn_eval(z, tab, F, G);
    o.pm = kcb * chi * ig * rcp(x) * (o.omx3 * F + o.x3 * o.x3 * G);
    return o;
}

// Push constants of a lepton (s = 0: q = -1, s = 1: q = +1) over sub-steps of st.
template <class R>
struct PushConst {
    R hq, hex, hey, hez, e2, str, kcb;
};

template <class R>
__device__ __forceinline__ PushConst<R> push_const(const Lepton<R> &p, int s, double st) {
    PushConst<R> c;
    c.hq = (R)((s == 0 ? -0.5 : 0.5) * st);
    c.hex = c.hq * p.ex;
    c.hey = c.hq * p.ey;
    c.hez = c.hq * p.ez;
    c.e2 = p.ex * p.ex + p.ey * p.ey + p.ez * p.ez;
    c.str = (R)st;
    // c b = kcb chi / gamma, with c = sqrt(3) alpha st / (pi gamma) and b = 3 chi / 2
    c.kcb = (R)(1.5 * kSqrt3 * kAlpha / kPi * st);
    return c;
}

// The held state of a pure-magnetic-field lepton (Rot) with its chi, from u.
template <class R>
__device__ __forceinline__ Rot<R> rot_chi(const Lepton<R> &p, const PushConst<R> &c, R ux, R uy, R uz) {
    Rot<R> r = rot_of(ux, uy, uz, c.hq, p.bx, p.by, p.bz, c.str);
    uint32_t none = 0;  // no cross term in a pure magnetic field: the double recomputation never runs
    r.chi = chi_sub<2>(ux, uy, uz, r.g, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, c.e2, none);
    return r;
}

// Algorithm 1's sub-step loop for one electron (s = 0, q = -1) or positron (s = 1,
// q = +1) with N >= 1 sub-steps.  s is uniform across the wave.  FK: field kind
// (0 general, 1 pure E, 2 pure B), see boris().
template <class R, int FK>
__device__ __forceinline__ void lepton_loop(const StepArgs &a, int s, u64 i, uint32_t N, Lepton<R> p,
                                            const SynTable<R> &tab, ChildBuf<R> &cb, Tally<R> &tl, double t0) {
    const SpeciesDev &sp = a.sp[s];
    const uint64_t pid = sp.id[i];
    const Origin<R> org = origin_of<R>(sp, i);
    const double st = (a.dt - t0) / (double)N;
    const PushConst<R> c = push_const(p, s, st);
    const uint32_t idlo = (uint32_t)pid, idhi = (uint32_t)(pid >> 32);
    const uint32_t klo = (uint32_t)a.seed, khi = (uint32_t)(a.seed >> 32);
    const uint32_t step = step_of(a);
    R ux = p.ux, uy = p.uy, uz = p.uz;
    R dx = 0, dy = 0, dz = 0;
    uint32_t nev = 0;
    uint32_t last = 0;  // sub-steps done at this particle's previous event
    Rot<R> rs{};
    if constexpr (FK == 2) rs = rot_chi(p, c, ux, uy, uz);
    Draw<R> draw;
    for (uint32_t k = 0; k < N; ++k) {
        const SubStep<R, FK> o = substep<R, FK>(p, c.hex, c.hey, c.hez, c.hq, c.e2, c.str, c.kcb, k, idlo, idhi, step,
                                                klo, khi, draw, tab, ux, uy, uz, dx, dy, dz, rs, tl.guard);
        tl.max_p = fmax(tl.max_p, o.pm);
        tl.clips += o.pm > R(1);
        const bool acc = o.y < o.pm;
        // emission: stage the photon in the wave's LDS buffer, recoil on the parent
        const u64 m = __ballot(acc);
        if (m) {
            const R u2 = FK == 2 ? ux * ux + uy * uy + uz * uz : o.u2;
            stage_emission<R>(a, org, pid, k, k, acc, m, o.x3, o.omx3, o.g, u2, dx, dy, dz, ux, uy, uz, cb, nev,
                              t0, st, step);
            if constexpr (FK == 2)
                if (acc) rs = rot_chi(p, c, ux, uy, uz);   // after the recoil
            if (acc && a.gap_hist) {
                count_gap(a, 0, k + 1 - last);
                last = k + 1;
            }
        }
    }
    ((R *)sp.ux)[i] = ux;
    ((R *)sp.uy)[i] = uy;
    ((R *)sp.uz)[i] = uz;
    sp.x[i] = org.x + (double)dx;
    sp.y[i] = org.y + (double)dy;
    sp.z[i] = org.z + (double)dz;
    if (sp.events) sp.events[i] = nev;
    tl.substeps += N;
    tl.events += nev;
}

template <class R>
__device__ __forceinline__ void lepton_run(const StepArgs &a, int s, u64 i, uint32_t N, Lepton<R> p,
                                           const SynTable<R> &tab, ChildBuf<R> &cb, Tally<R> &tl, double t0) {
    const bool noB = p.bx == R(0) && p.by == R(0) && p.bz == R(0);
    const bool noE = p.ex == R(0) && p.ey == R(0) && p.ez == R(0);
    if (noB)
        lepton_loop<R, 1>(a, s, i, N, p, tab, cb, tl, t0);
    else if (noE)
        lepton_loop<R, 2>(a, s, i, N, p, tab, cb, tl, t0);
    else
        lepton_loop<R, 0>(a, s, i, N, p, tab, cb, tl, t0);
}

// ---------------------------------------------------------------------------
// Surrogate sampler (mixed precision): the sub-steps and push of Algorithm 1,
// with the emission time from the optical depth and the energy from the learned
// inverse CDF (or rejection sampling of eq. (1) at the current chi).
// ---------------------------------------------------------------------------
// Key tag of the surrogate's random stream: the draws of particle id in step
// `step` are Philox blocks (id_lo, id_hi, step, j) under the seed key xor'ed
// with this tag, j counting the particle's draws within the step.
constexpr uint32_t kSurrTagLo = 0x2545F491u, kSurrTagHi = 0x9E3779B9u;
constexpr uint32_t kMaxRejections = 1u << 12;

struct SurrLds {
    RateTable rate;
    MlpLds mlp;
    MlpWave ws[kBlock / 64];
    int have_model;
};

__device__ __forceinline__ void surr_stage(const StepArgs &a, SurrLds &S) {
    if (a.model) mlp_stage(a.model, S.mlp);
    if (threadIdx.x == 0) S.have_model = a.model != nullptr;
    rate_stage(S.rate);  // ends with a barrier
}

// x = delta^(1/3) from eq. (1) at fixed chi by rejection against the envelope.
__device__ __forceinline__ float surr_reject(float chi, const SurrLds &S, const SynTable<float> &tab,
                                             uint32_t idlo, uint32_t idhi, uint32_t step, uint32_t klo,
                                             uint32_t khi, uint32_t &j, Tally<float> &tl) {
    const float b = 1.5f * chi;
    const float env = rate_envelope(chi, S.rate);
    u32x4 w = {0u, 0u, 0u, 0u};
    float x = 0.5f;
    for (uint32_t it = 0; it < kMaxRejections; ++it) {
        if ((it & 1u) == 0u) w = philox10(idlo, idhi, step, j++, klo, khi);
        const bool odd = (it & 1u) != 0u;
        x = u24(odd ? w.z : w.x);
        const float y = u24(odd ? w.w : w.y);
        const float x2 = x * x, x3 = x2 * x;
        const float omx3 = (1.0f - x) * (1.0f + x + x2);
        float F, G;
        syn_eval(x3 * rcp(b * omx3), tab, F, G);
        const float d = (omx3 * F + x3 * x3 * G) * rcp(x);
        tl.fb_draws++;
        tl.env_clips += d > env;
        if (y * env < d) break;
    }
    return x;
}

// One sub-step of the optical-depth path: Boris push and move, chi after the
// push, and the optical depth used up, alpha sub_t chi q(chi) / gamma (float
// product, double accumulation).  Shared by the sub-step loop and the pre-pass.
template <int FK>
__device__ __forceinline__ void substep_surr(const Lepton<float> &p, const PushConst<float> &c, float wk,
                                             const RateTable &rate, float &ux, float &uy, float &uz, float &dx,
                                             float &dy, float &dz, const Rot<float> &rs, double &tau,
                                             uint32_t &guard) {
    using R = float;
    R ig, g, vs;
    if constexpr (FK == 2) {
        rotate(ux, uy, uz, rs);
        ig = rs.ig;
        g = rs.g;
        vs = rs.vs;
    } else {
        boris<R, FK>(ux, uy, uz, c.hex, c.hey, c.hez, c.hq, p.bx, p.by, p.bz);
        R u2;
        ig = inv_gamma(ux, uy, uz, u2);
        g = (R(1) + u2) * ig;
        vs = c.str * ig;
    }
    dx += ux * vs;
    dy += uy * vs;
    dz += uz * vs;
    R rw;
    if constexpr (FK == 2) {
        rw = rs.rw;   // chi and gamma are held, so is the rate
    } else {
        const R chi = chi_sub<FK>(ux, uy, uz, g, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, c.e2, guard);
        rw = rate_chi_q(chi, rate) * ig;
    }
    tau -= (double)(wk * rw);
}

// Emissions are resolved in batches: a lane whose optical depth runs out only
// marks the crossing and waits (it does not advance) while the other lanes go on;
// once a.resolve_batch lanes wait, or no lane can advance, the waiting lanes
// together draw their random numbers, take their energies (network rows on the
// matrix cores, or rejection), stage the photons, apply the recoils and go on.
// Everything a crossing costs beyond the sub-step itself (the Philox blocks, the
// double logarithm of the next optical depth, the energy, the photon) thus runs
// with the waiting lanes together instead of stalling the wave at every crossing.
// A lane's own sequence of operations and draws does not depend on when its
// emission is resolved, so the result is the same for any batch size and any
// scheduler.  N: this lane's sub-steps (0 for a lane without a particle).  All
// 64 lanes of the wave call it.  DUAL: network passes of up to 32 rows (two
// groups sharing their weight reads; the heavy queue, whose register budget has
// room for them), else 16.
template <int FK, bool DUAL>
__device__ __forceinline__ void lepton_loop_surr(const StepArgs &a, int s, u64 i, uint32_t N,
                                                 const Lepton<float> &p, const SynTable<float> &tab, SurrLds &S,
                                                 ChildBuf<float, false> &cb, Tally<float> &tl) {
    using R = float;
    const SpeciesDev &sp = a.sp[s];
    const bool has = N > 0;
    const uint64_t pid = has ? sp.id[i] : 0ull;
    const Origin<R> org = has ? origin_of<R>(sp, i) : Origin<R>{0.0, 0.0, 0.0, R(0)};
    const double st = has ? a.dt / (double)N : 0.0;
    const PushConst<R> c = push_const(p, s, st);
    const R e2 = c.e2;
    // W sub_t = alpha sub_t chi q(chi) / gamma
    const R wk = (R)(kAlpha * st);
    const uint32_t idlo = (uint32_t)pid, idhi = (uint32_t)(pid >> 32);
    const uint32_t klo = (uint32_t)a.seed ^ kSurrTagLo, khi = (uint32_t)(a.seed >> 32) ^ kSurrTagHi;
    const uint32_t step = step_of(a);
    const int batch = (int)a.resolve_batch;
    MlpWave &ws = S.ws[threadIdx.x / 64];
    uint32_t j = 0;
    double tau = has ? sp.tau[i] : 1.0;
    if (has && !(tau > 0.0)) {
        const u32x4 w = philox10(idlo, idhi, step, j++, klo, khi);
        tau = neg_ln(u53(w.x, w.y));
    }
    R ux = p.ux, uy = p.uy, uz = p.uz;
    R dx = 0, dy = 0, dz = 0;
    Rot<R> rs{};
    if constexpr (FK == 2) {
        rs = rot_chi(p, c, ux, uy, uz);
        rs.rw = rate_chi_q(rs.chi, S.rate) * rs.ig;
    }
    uint32_t nev = 0;
    uint32_t k = 0;     // next sub-step of this lane
    bool pend = false;  // an emission waits for its energy
    uint32_t pk = 0;    // its sub-step
    // A waiting lane keeps its momentum at the crossing, so chi, gamma and the rate
    // there are recomputed when the emission is resolved instead of held; tau then
    // holds the overshoot (<= 0) of the sub-step that crossed.
    for (;;) {
        if (k < N && !pend) {
            if constexpr (FK == 2) {
                // The held rate does not change until the next emission, so the optical
                // depth falls by the same d every sub-step: go straight to the sub-step
                // where it crosses zero, or to the end of the step.  One sub-step runs as
                // the loop body (bit for bit what the pre-pass runs); more run in closed
                // form (rotate_many), with tau - m d in one rounding.  Every lane that can
                // move then reaches its crossing at once, and the resolves take them all.
                const double d = (double)(wk * rs.rw);
                uint32_t m = N - k;
                if (d > 0.0) {
                    const double q = ceil(tau / d);
                    if (q < (double)m) m = q < 1.0 ? 1u : (uint32_t)q;
                }
                if (m == 1u) {
                    substep_surr<2>(p, c, wk, S.rate, ux, uy, uz, dx, dy, dz, rs, tau, tl.guard);
                } else {
                    rotate_many(ux, uy, uz, dx, dy, dz, rs, m);
                    tau = fma(-(double)m, d, tau);
                }
                pend = tau <= 0.0;
                pk = k + m - 1u;
                k += m;
            } else {
                substep_surr<FK>(p, c, wk, S.rate, ux, uy, uz, dx, dy, dz, rs, tau, tl.guard);
                pend = tau <= 0.0;
                pk = k;
                ++k;
            }
        }
        const u64 mp = __ballot(pend);
        const u64 mr = __ballot(k < N && !pend);
        if (mp == 0 && mr == 0) break;
        if (mp == 0 || (__popcll(mp) < batch && mr != 0)) continue;
        // The waiting lanes: the uniform of the energy and the next optical depth,
        // then their state at the crossing.
        R pu = 0.5f, cu2 = 0, cg = 1, cchi = 0, crw = 1;
        double ptau = 1.0;
        if (pend) {
            const u32x4 w = philox10(idlo, idhi, step, j++, klo, khi);
            pu = u24(w.x);
            ptau = neg_ln(u53(w.z, w.w));
            cu2 = ux * ux + uy * uy + uz * uz;
            if constexpr (FK == 2) {   // the held state is the state at the crossing
                cg = rs.g;
                cchi = rs.chi;
                crw = rs.rw;
            } else {
                const R ig = rsqrt_(R(1) + cu2);
                cg = (R(1) + cu2) * ig;
                cchi = chi_sub<FK>(ux, uy, uz, cg, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, e2, tl.guard);
                crw = rate_chi_q(cchi, S.rate) * ig;
            }
        }
        bool use_net = false;
        R sin = 0.0f;
        if (pend && S.have_model) {
            bool in_range;
            int bin;
            sin = mlp_input_s(S.mlp, cchi, in_range, bin);
            use_net = in_range && !S.mlp.fallback[bin];
        }
        R yv = 0.0f;
        if (__ballot(use_net)) yv = mlp_infer_wave<DUAL>(S.mlp, ws, use_net, sin, mlp_input_v(pu));
        R x3 = 0, omx3 = 1;
        if (pend) {
            R x;
            if (use_net) {
                x = mlp_x_of_y(yv, cchi);
                tl.learned++;
            } else {
                x = surr_reject(cchi, S, tab, idlo, idhi, step, klo, khi, j, tl);
                tl.fallback++;
            }
            const R x2 = x * x;
            x3 = x2 * x;
            omx3 = (R(1) - x) * (R(1) + x + x2);
        }
        stage_emission<R>(a, org, pid, nev, pk, pend, mp, x3, omx3, cg, cu2, dx, dy, dz, ux, uy, uz, cb, nev,
                          0.0, st, step);
        // The part of the sub-step after the crossing (the overshoot, at the rate before
        // the emission) counts against the new optical depth at the rate after the
        // recoil.  If that crosses it again, the lane waits for another emission
        // before moving on.
        if (pend) {
            R rw;
            if constexpr (FK == 2) {   // the held state after the recoil
                rs = rot_chi(p, c, ux, uy, uz);
                rs.rw = rate_chi_q(rs.chi, S.rate) * rs.ig;
                rw = rs.rw;
            } else {
                R u2;
                const R ig = inv_gamma(ux, uy, uz, u2);
                const R g = (R(1) + u2) * ig;
                const R chi = chi_sub<FK>(ux, uy, uz, g, p.ex, p.ey, p.ez, p.bx, p.by, p.bz, e2, tl.guard);
                rw = rate_chi_q(chi, S.rate) * ig;
            }
            tau = ptau + tau * (double)(rw / crw);
            pend = tau <= 0.0;
        }
    }
    if (has) {
        ((R *)sp.ux)[i] = ux;
        ((R *)sp.uy)[i] = uy;
        ((R *)sp.uz)[i] = uz;
        sp.x[i] = org.x + (double)dx;
        sp.y[i] = org.y + (double)dy;
        sp.z[i] = org.z + (double)dz;
        sp.tau[i] = tau;
        if (sp.events) sp.events[i] = nev;
        tl.substeps += N;
        tl.events += nev;
    }
}

// One particle per lane, all lanes of the wave (has = false: no particle).
template <class R, bool SURR>
struct LeptonRunner;

template <class R>
struct LeptonRunner<R, false> {
    template <bool DUAL = false, class L>
    __device__ static void run(const StepArgs &a, int s, u64 i, uint32_t N, const Lepton<R> &p, L &lds,
                               ChildBuf<R> &cb, Tally<R> &t, double t0 = 0.0) {
        if (N) lepton_run<R>(a, s, i, N, p, lds.tab, cb, t, t0);
    }
};

template <>
struct LeptonRunner<float, true> {
    template <bool DUAL = false, class L>
    __device__ static void run(const StepArgs &a, int s, u64 i, uint32_t n, const Lepton<float> &p, L &lds,
                               ChildBuf<float, false> &cb, Tally<float> &t, double = 0.0) {
        if (__ballot(n != 0) == 0) return;
        // one field kind for the whole wave (the general form is valid for all)
        const bool noB = p.bx == 0.0f && p.by == 0.0f && p.bz == 0.0f;
        const bool noE = p.ex == 0.0f && p.ey == 0.0f && p.ez == 0.0f;
        const u64 live = __ballot(n != 0);
        if ((__ballot(n != 0 && noB) == live))
            lepton_loop_surr<1, DUAL>(a, s, i, n, p, lds.tab, lds.surr, cb, t);
        else if ((__ballot(n != 0 && noE) == live))
            lepton_loop_surr<2, DUAL>(a, s, i, n, p, lds.tab, lds.surr, cb, t);
        else
            lepton_loop_surr<0, DUAL>(a, s, i, n, p, lds.tab, lds.surr, cb, t);
    }
};

// ---------------------------------------------------------------------------
// Algorithm 2.
// ---------------------------------------------------------------------------
struct PhotonStart {
    double eps, chi;
    double t0;  // start time within the step (birth time in a cascade pass, else 0)
    uint32_t N;
};

// Algorithm 2's sub-step loop for one photon that can decay.
template <class R>
__device__ __forceinline__ void photon_sample(const StepArgs &a, u64 i, R kx, R ky, R kz, double x0, double y0,
                                              double z0, const PhotonStart &ps, const SynTable<R> &tab,
                                              const PairTable &pt, Tally<R> &tl) {
    const SpeciesDev &sp = a.sp[2];
    const SpeciesDev &el = a.sp[0];
    const SpeciesDev &po = a.sp[1];
    const uint32_t N = ps.N;
    const double st = (a.dt - ps.t0) / (double)N;
    const R inv = (R)(1.0 / ps.eps);
    const R dirx = kx * inv, diry = ky * inv, dirz = kz * inv;
    const R str = (R)st;
    // P_p(x) = alpha st sqrt(3)/(2 pi) (chi/eps) (G(z) - x(1-x) F(z)),  z = 2/(3 chi x (1-x))
    const R A = (R)(kAlpha * st * kSqrt3 / (2.0 * kPi) * ps.chi / ps.eps);
    const R chir = (R)ps.chi;
    const R epsr = (R)ps.eps;
    // Exact squeeze: P_p <= A env / (3/2 chi) for every x (the fitted envelope of
    // G - x(1-x) F, 5% above its maximum), so a test value y at or above that bound
    // rejects without evaluating F and G: the decision is the one eq. (2) gives.
    // chi below the envelope's table: no squeeze (such photons never get here).
    const R squeeze = ps.chi >= 0x1p-6 ? A * (R)(pair_envelope((float)ps.chi, pt) / (1.5f * (float)ps.chi))
                                       : R(2);
    const uint64_t pid = sp.id[i];
    const uint32_t idlo = (uint32_t)pid, idhi = (uint32_t)(pid >> 32);
    const uint32_t klo = (uint32_t)a.seed, khi = (uint32_t)(a.seed >> 32);
    const uint32_t step = step_of(a);
    R dx = 0, dy = 0, dz = 0;
    bool dead = false;
    uint32_t used = 0;
    Draw<R> draw;
    for (uint32_t k = 0; k < N && !dead; ++k) {
        used = k + 1;
        // move at the speed of light
        dx += dirx * str;
        dy += diry * str;
        dz += dirz * str;
        // candidate x, test value y, acceptance against eq. (2)
        R x, y;
        draw.get(k, idlo, idhi, step, klo, khi, x, y);
        bool acc = false;
        if (y < squeeze) {
            const R xx = x * (R(1) - x);
            const R z = R(2.0 / 3.0) * rcp(chir * xx);
            R F, G;
            syn_eval(z, tab, F, G);
            const R pp = A * (G - xx * F);
            tl.max_p = fmax(tl.max_p, pp);
            tl.clips += pp > R(1);
            acc = y < pp;
        }
        // pair creation: electron with x eps, positron with (1-x) eps, along k; delete
        const u64 m = __ballot(acc);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            u64 be = 0, bp = 0, bd = 0;
            if (__lane_id() == leader) {
                const u64 c = (u64)__popcll(m);
                be = atomicAdd(el.n, c);
                bp = atomicAdd(po.n, c);
                bd = atomicAdd(&a.st->dead, c);
            }
            be = __shfl(be, leader);
            bp = __shfl(bp, leader);
            bd = __shfl(bd, leader);
            if (acc) {
                const u64 r = (u64)__popcll(m & lanemask_lt());
                a.dead_idx[bd + r] = i;
                const double px = x0 + (double)dx, py = y0 + (double)dy, pz = z0 + (double)dz;
                const R w = ((const R *)sp.w)[i];
                const double tb = ps.t0 + (double)(k + 1) * st;
                const R ge = x * epsr, gp = (R(1) - x) * epsr;
                const R ue = sqrt_(fmax(ge * ge - R(1), R(0)));
                const R up = sqrt_(fmax(gp * gp - R(1), R(0)));
                if (be + r < el.cap) {
                    const u64 j = be + r;
                    el.x[j] = px;
                    el.y[j] = py;
                    el.z[j] = pz;
                    ((R *)el.ux)[j] = ue * dirx;
                    ((R *)el.uy)[j] = ue * diry;
                    ((R *)el.uz)[j] = ue * dirz;
                    ((R *)el.w)[j] = w;
                    el.id[j] = child_id(a.seed, pid, step, k, 0);
                    if (el.parent) el.parent[j] = pid;
                    if (el.tau) el.tau[j] = -1.0;
                    if (el.birth) el.birth[j] = tb;
                }
                if (bp + r < po.cap) {
                    const u64 j = bp + r;
                    po.x[j] = px;
                    po.y[j] = py;
                    po.z[j] = pz;
                    ((R *)po.ux)[j] = up * dirx;
                    ((R *)po.uy)[j] = up * diry;
                    ((R *)po.uz)[j] = up * dirz;
                    ((R *)po.w)[j] = w;
                    po.id[j] = child_id(a.seed, pid, step, k, 1);
                    if (po.parent) po.parent[j] = pid;
                    if (po.tau) po.tau[j] = -1.0;
                    if (po.birth) po.birth[j] = tb;
                }
                dead = true;
                count_gap(a, 1, k + 1);
            }
        }
    }
    // positions: the caller has written the end-of-step position (the survivor's);
    // the slot of a photon that decayed is removed by the compaction
    a.alive[i] = dead ? 0 : 1;
    if (sp.events) sp.events[i] = dead ? 1u : 0u;
    tl.substeps += used;
    tl.events += dead;
}

// Bin of a sub-step count (see kBins).
__device__ __forceinline__ int nbin(uint32_t N, uint32_t light_max, uint32_t per_octave) {
    if (N <= light_max) return 0;
    const int b = 1 + (int)floorf((float)per_octave * __log2f((float)N));
    return b < kBins - 1 ? b : kBins - 1;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// End-of-kernel flush of all wave buffers of the block with one atomic: every
// thread of the block must call it.
template <class R, bool TB>
__device__ __forceinline__ void flush_children_block(ChildBuf<R, TB> *cbs, const SpeciesDev &dst, uint64_t seed,
                                                     uint32_t step) {
    __shared__ u64 base_sh;
    __shared__ uint32_t pre[kBlock / 64 + 1];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t o = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            pre[w] = o;
            o += cbs[w].count;
        }
        pre[kBlock / 64] = o;
        base_sh = o ? atomicAdd(dst.n, (u64)o) : 0ull;
    }
    __syncthreads();
    const uint32_t total = pre[kBlock / 64];
    for (uint32_t e = threadIdx.x; e < total; e += kBlock) {
        int w = 0;
        while (w + 1 < kBlock / 64 && pre[w + 1] <= e) ++w;
        const ChildBuf<R, TB> &cb = cbs[w];
        const uint32_t k = e - pre[w];
        const u64 slot = base_sh + e;
        if (slot < dst.cap) {
            dst.x[slot] = cb.x[k];
            dst.y[slot] = cb.y[k];
            dst.z[slot] = cb.z[k];
            ((R *)dst.ux)[slot] = cb.px[k];
            ((R *)dst.uy)[slot] = cb.py[k];
            ((R *)dst.uz)[slot] = cb.pz[k];
            ((R *)dst.w)[slot] = cb.w[k];
            dst.id[slot] = child_id(seed, cb.parent[k], step, cb.ctr[k], 0);
            if (dst.parent) dst.parent[slot] = cb.parent[k];
            if constexpr (TB)
                if (dst.birth) dst.birth[slot] = cb.tb[k];
            if (dst.tau) dst.tau[slot] = -1.0;
        }
    }
}

// LDS of the lepton kernels: the coefficient table and one child buffer per wave,
// plus the rate table and the network for the surrogate sampler.
template <class R, bool SURR>
struct LeptonLds {
    SynTable<R> tab;
    ChildBuf<R> cb[kBlock / 64];
};

template <>
struct LeptonLds<float, true> {
    SynTable<float> tab;
    ChildBuf<float, false> cb[kBlock / 64];
    SurrLds surr;
};

template <class R, bool SURR>
__device__ __forceinline__ auto &lepton_lds_init(const StepArgs &a, LeptonLds<R, SURR> &L) {
    auto &cb = L.cb[threadIdx.x / 64];
    if (__lane_id() == 0) cb.count = 0;
    if constexpr (SURR) surr_stage(a, L.surr);
    syn_stage(L.tab);  // ends with a block barrier
    return cb;
}

// The particle of this lane (N = 0 and a zero record when there is none).
template <class R>
__device__ __forceinline__ uint32_t lepton_fetch(const StepArgs &a, int s, u64 i, bool has, Lepton<R> &p,
                                                 Tally<R> &t, double dt) {
    if (!has) {
        p = Lepton<R>{0, 0, 0, 0, 0, 0, 0, 0, 0};
        return 0;
    }
    p = load_lepton<R>(a, s, i);
    return lepton_nsub(a, s, i, p, t, dt);
}

// Naive scheduler: one lane per particle in buffer order; the loop runs with
// whole waves (lanes past the end carry no particle).  The pass covers the slots
// lo..hi of the device state; in a cascade pass (gen >= 1) each particle runs
// over the rest of the step from its birth time.
template <class R, bool SURR>
__global__ __launch_bounds__(kBlock) void k_lepton(StepArgs a) {
    __shared__ LeptonLds<R, SURR> L;
    auto &cb = lepton_lds_init<R, SURR>(a, L);
    const int s = blockIdx.y;
    const u64 lo = a.st->lo[s], hi = a.st->hi[s];
    Tally<R> t;
    for (u64 i0 = lo + (u64)blockIdx.x * kBlock + (threadIdx.x & ~63u); i0 < hi; i0 += (u64)gridDim.x * kBlock) {
        const u64 i = i0 + __lane_id();
        const bool has = i < hi;
        const double t0 = a.gen && has ? a.sp[s].birth[i] : 0.0;
        Lepton<R> p;
        const uint32_t N = lepton_fetch(a, s, i, has, p, t, a.dt - t0);
        if (has && N == 0 && a.sp[s].events) a.sp[s].events[i] = 0;
        LeptonRunner<R, SURR>::run(a, s, i, N, p, L, cb, t, t0);
    }
    flush_children_block(L.cb, a.sp[2], a.seed, step_of(a));
    flush_tally(t, a.st, s);
}

// A particle whose step has a single sub-step (N = 1, main pass) runs it here.  If
// it ends without an event the particle is finished: it is stored as the sub-step
// loop would store it (the same shared sub-step code, so bit for bit the same) and
// true is returned.  If it emits (or its optical depth runs out), nothing is
// written and false is returned: the light pass then runs the particle in full.
template <class R, int FK>
__device__ __forceinline__ bool finish_single_fk(const StepArgs &a, int s, u64 i, const Lepton<R> &p,
                                                 const SynTable<R> &tab, Tally<R> &tl) {
    const SpeciesDev &sp = a.sp[s];
    const uint64_t pid = sp.id[i];
    const double st = a.dt;
    const PushConst<R> c = push_const(p, s, st);
    R ux = p.ux, uy = p.uy, uz = p.uz;
    R dx = 0, dy = 0, dz = 0;
    Rot<R> rs{};
    if constexpr (FK == 2) rs = rot_chi(p, c, ux, uy, uz);
    uint32_t guard = 0;
    Draw<R> draw;
    const SubStep<R, FK> o = substep<R, FK>(p, c.hex, c.hey, c.hez, c.hq, c.e2, c.str, c.kcb, 0u, (uint32_t)pid,
                                            (uint32_t)(pid >> 32), step_of(a), (uint32_t)a.seed,
                                            (uint32_t)(a.seed >> 32), draw, tab, ux, uy, uz, dx, dy, dz, rs, guard);
    if (o.y < o.pm) return false;
    tl.max_p = fmax(tl.max_p, o.pm);
    tl.clips += o.pm > R(1);
    tl.guard += guard;
    ((R *)sp.ux)[i] = ux;
    ((R *)sp.uy)[i] = uy;
    ((R *)sp.uz)[i] = uz;
    sp.x[i] += (double)dx;
    sp.y[i] += (double)dy;
    sp.z[i] += (double)dz;
    if (sp.events) sp.events[i] = 0;
    tl.substeps += 1;
    return true;
}

template <int FK>
__device__ __forceinline__ bool finish_single_surr_fk(const StepArgs &a, int s, u64 i, const Lepton<float> &p,
                                                      const RateTable &rate, Tally<float> &tl) {
    const SpeciesDev &sp = a.sp[s];
    const uint64_t pid = sp.id[i];
    const double st = a.dt;
    const PushConst<float> c = push_const(p, s, st);
    const float wk = (float)(kAlpha * st);
    double tau = sp.tau[i];
    if (!(tau > 0.0)) {
        const u32x4 w = philox10((uint32_t)pid, (uint32_t)(pid >> 32), step_of(a), 0u, (uint32_t)a.seed ^ kSurrTagLo,
                                 (uint32_t)(a.seed >> 32) ^ kSurrTagHi);
        tau = neg_ln(u53(w.x, w.y));
    }
    float ux = p.ux, uy = p.uy, uz = p.uz;
    float dx = 0, dy = 0, dz = 0;
    Rot<float> rs{};
    if constexpr (FK == 2) {
        rs = rot_chi(p, c, ux, uy, uz);
        rs.rw = rate_chi_q(rs.chi, rate) * rs.ig;
    }
    uint32_t guard = 0;
    substep_surr<FK>(p, c, wk, rate, ux, uy, uz, dx, dy, dz, rs, tau, guard);
    if (tau <= 0.0) return false;
    tl.guard += guard;
    ((float *)sp.ux)[i] = ux;
    ((float *)sp.uy)[i] = uy;
    ((float *)sp.uz)[i] = uz;
    sp.x[i] += (double)dx;
    sp.y[i] += (double)dy;
    sp.z[i] += (double)dz;
    sp.tau[i] = tau;
    if (sp.events) sp.events[i] = 0;
    tl.substeps += 1;
    return true;
}

// LDS of the pre-pass: the histogram and the table the single-sub-step particles
// need (the synchrotron fits, or the total-rate fit on the optical-depth path).
template <class R, bool SURR>
struct PrepassLds {
    uint32_t h[kBins];
    SynTable<R> tab;
};

template <>
struct PrepassLds<float, true> {
    uint32_t h[kBins];
    RateTable rate;
};

template <class R, bool SURR>
__device__ __forceinline__ bool finish_single(const StepArgs &a, int s, u64 i, const Lepton<R> &p,
                                              const PrepassLds<R, SURR> &L, Tally<R> &tl) {
    // the field kind of the push and chi as the loops choose it (every kind gives the
    // general form's result for its fields)
    const bool noB = p.bx == R(0) && p.by == R(0) && p.bz == R(0);
    const bool noE = p.ex == R(0) && p.ey == R(0) && p.ez == R(0);
    if constexpr (SURR) {
        if (noB) return finish_single_surr_fk<1>(a, s, i, p, L.rate, tl);
        if (noE) return finish_single_surr_fk<2>(a, s, i, p, L.rate, tl);
        return finish_single_surr_fk<0>(a, s, i, p, L.rate, tl);
    } else {
        if (noB) return finish_single_fk<R, 1>(a, s, i, p, L.tab, tl);
        if (noE) return finish_single_fk<R, 2>(a, s, i, p, L.tab, tl);
        return finish_single_fk<R, 0>(a, s, i, p, L.tab, tl);
    }
}

// Pre-pass of the binned scheduler: every lepton's sub-step count N (the bound of
// Sec. 3.1.1 in double) and the histogram of the bins.  With a.prepass_finish,
// particles of a single quiet sub-step are finished here (N recorded as 0, like a
// skipped particle), so the light pass does not read them again.  A streaming pass:
// the float instances are held to 128 VGPRs so that 4 waves per SIMD hide its loads.
template <class R, bool SURR>
__global__ __launch_bounds__(kBlock, sizeof(R) == 4 ? 4 : 3) void k_prepass(StepArgs a) {
    __shared__ PrepassLds<R, SURR> L;
    uint32_t *h = L.h;
    const int s = blockIdx.y;
    for (int b = threadIdx.x; b < kBins; b += kBlock) h[b] = 0;
    if (a.prepass_finish) {
        if constexpr (SURR)
            rate_stage(L.rate);  // ends with a barrier
        else
            syn_stage(L.tab);    // ends with a barrier
    } else {
        __syncthreads();
    }
    const u64 n = a.st->n0[s];
    Tally<R> t;
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock) {
        const Lepton<R> p = load_lepton<R>(a, s, i);
        uint32_t N = lepton_nsub(a, s, i, p, t, a.dt);
        const bool done = N == 1 && a.prepass_finish && finish_single<R, SURR>(a, s, i, p, L, t);
        if (done) N = 0;
        a.nsub[s][i] = N;
        if (N)
            atomicAdd(&h[nbin(N, a.light_max, a.bins_per_octave)], 1u);
        else if (!done && a.sp[s].events)
            a.sp[s].events[i] = 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kBlock)
        if (h[b]) atomicAdd(&a.st->hist[s][b], h[b]);
    // finished particles' sub-steps, the skipped (non-finite) and the capped counts
    flush_tally(t, a.st, s);
}

// One block of kBins threads per species (y): heavy bins laid out heaviest first
// (offset of bin b: the counts of the bins above it).
__global__ __launch_bounds__(kBins) void k_scan(StepArgs a) {
    __shared__ uint32_t wsum[kBins / 64];
    const int s = blockIdx.y;
    const int b = kBins - 1 - (int)threadIdx.x;   // thread 0 takes the heaviest bin
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
    const uint32_t v = b >= 1 ? a.st->hist[s][b] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o);
        if ((int)lane >= o) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < kBins / 64; ++w) {
        before += w < wv ? wsum[w] : 0u;
        total += wsum[w];
    }
    if (b >= 1) {
        a.st->offset[s][b] = before + incl - v;
        a.st->cursor[s][b] = 0;
    }
    if (threadIdx.x == 0) {
        a.st->heavy[s] = total;
        a.st->queue[s] = 0;
    }
}

// Heavy slots into their bins.  Each block takes one contiguous range of slots:
// it counts the range's heavy particles per bin in LDS, reserves its segment of
// every bin with one global atomic per (block, bin), and then places them, with
// LDS ranks inside the segment (a second read of the range's counts).
__global__ __launch_bounds__(kBlock) void k_scatter(StepArgs a) {
    __shared__ uint32_t cnt[kBins], base[kBins];
    const int s = blockIdx.y;
    const u64 n = a.st->n0[s];
    const u64 per = ((n + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
    const u64 lo = (u64)blockIdx.x * per;
    const u64 hi = lo + per < n ? lo + per : n;
    for (int b = threadIdx.x; b < kBins; b += kBlock) cnt[b] = 0;
    __syncthreads();
    // kScatterBatch counts loaded before their bins are counted, so that the loads
    // of one thread overlap
    constexpr int kScatterBatch = 8;
    for (u64 i0 = lo + threadIdx.x; i0 < hi; i0 += (u64)kBlock * kScatterBatch) {
        uint32_t N[kScatterBatch];
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k) {
            const u64 i = i0 + (u64)k * kBlock;
            N[k] = i < hi ? a.nsub[s][i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k)
            if (N[k]) {
                const int bin = nbin(N[k], a.light_max, a.bins_per_octave);
                if (bin) atomicAdd(&cnt[bin], 1u);
            }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kBlock) {
        base[b] = cnt[b] ? atomicAdd(&a.st->cursor[s][b], cnt[b]) + a.st->offset[s][b] : 0u;
        cnt[b] = 0;
    }
    __syncthreads();
    for (u64 i0 = lo + threadIdx.x; i0 < hi; i0 += (u64)kBlock * kScatterBatch) {
        uint32_t N[kScatterBatch];
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k) {
            const u64 i = i0 + (u64)k * kBlock;
            N[k] = i < hi ? a.nsub[s][i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k)
            if (N[k]) {
                const int bin = nbin(N[k], a.light_max, a.bins_per_octave);
                if (bin) a.queue[s][base[bin] + atomicAdd(&cnt[bin], 1u)] = (uint32_t)(i0 + (u64)k * kBlock);
            }
    }
}

// Light pass: each wave takes tiles of a.light_tile consecutive slots (at most kTile);
// inside a tile the light particles (1 <= N <= light_max) are counting-sorted by N
// in the wave's LDS, heaviest first, and run 64 at a time in that order, so the
// lanes of a wave carry nearly the same N.  Waves never wait for each other, and
// the particle data stay in the tile's address window.
constexpr int kTile = 512;     // largest tile (8 slots per lane)
constexpr int kTileKeys = 64;  // N >= 63 share the heaviest key

template <class R, bool SURR>
__global__ __launch_bounds__(kBlock) void k_light(StepArgs a) {
    __shared__ LeptonLds<R, SURR> L;
    __shared__ uint32_t hist_sh[kBlock / 64][kTileKeys];
    __shared__ uint16_t order_sh[kBlock / 64][kTile];
    auto &cb = lepton_lds_init<R, SURR>(a, L);
    const int s = blockIdx.y;
    const u64 n = a.st->n0[s];
    const uint32_t lmax = a.light_max;
    const uint32_t lane = __lane_id();
    const int wv = threadIdx.x / 64;
    uint32_t *hist = hist_sh[wv];
    uint16_t *order = order_sh[wv];
    const u64 nwaves = (u64)gridDim.x * (kBlock / 64);
    const uint32_t tile = a.light_tile, qn = tile / 64;
    Tally<R> t;
    for (u64 t0 = ((u64)blockIdx.x * (kBlock / 64) + wv) * tile; t0 < n; t0 += nwaves * tile) {
        hist[lane] = 0;
        __syncwarp();
        uint32_t kr[kTile / 64];  // key << 16 | rank
#pragma unroll
        for (int q = 0; q < kTile / 64; ++q) {
            const u64 i = t0 + q * 64 + lane;
            const uint32_t N = (uint32_t)q < qn && i < n ? a.nsub[s][i] : 0u;
            const uint32_t key = (N >= 1 && N <= lmax) ? kTileKeys - (N < kTileKeys - 1 ? N : kTileKeys - 1) : 0u;
            kr[q] = key ? (key << 16) | atomicAdd(&hist[key], 1u) : 0u;
        }
        __syncwarp();
        // exclusive prefix over keys 1..63 (key 0 is not in this pass)
        const uint32_t h = lane >= 1 ? hist[lane] : 0u;
        uint32_t incl = h;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o);
            if ((int)lane >= o) incl += v;
        }
        const uint32_t total = __shfl(incl, 63);
        __syncwarp();
        hist[lane] = incl - h;  // now the offset of each key
        __syncwarp();
#pragma unroll
        for (int q = 0; q < kTile / 64; ++q)
            if (kr[q]) order[hist[kr[q] >> 16] + (kr[q] & 0xFFFFu)] = (uint16_t)(q * 64 + lane);
        __syncwarp();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + lane;
            const bool has = p < total;
            const u64 i = has ? t0 + order[p] : 0;
            const uint32_t N = has ? a.nsub[s][i] : 0u;
            const Lepton<R> q = has ? load_lepton<R>(a, s, i) : Lepton<R>{0, 0, 0, 0, 0, 0, 0, 0, 0};
            LeptonRunner<R, SURR>::run(a, s, i, N, q, L, cb, t);
        }
        __syncwarp();
    }
    flush_children_block(L.cb, a.sp[2], a.seed, step_of(a));
    flush_tally(t, a.st, s);
}

// Tile-sorted scheduler (one pass, no pre-pass): each wave takes tiles of kTiledSlots
// consecutive slots, computes every particle's sub-step count, counting-sorts the
// tile by it in LDS (heaviest first) and runs the tile 64 particles at a time in
// that order, so the lanes of a wave carry nearly the same N.  The particle
// records are read twice, the second time from the cache.  Tiles hold a.tiled_slots
// slots, at most kTiledSlots.
constexpr int kTiledSlots = 256;  // largest wave tile of the tile-sorted scheduler (4 slots per lane)

template <class R, bool SURR>
__global__ __launch_bounds__(kBlock) void k_tiled(StepArgs a) {
    __shared__ LeptonLds<R, SURR> L;
    __shared__ uint32_t hist_sh[kBlock / 64][kTileKeys];
    __shared__ uint16_t order_sh[kBlock / 64][kTiledSlots];
    __shared__ uint32_t nsub_sh[kBlock / 64][kTiledSlots];
    auto &cb = lepton_lds_init<R, SURR>(a, L);
    const int s = blockIdx.y;
    const u64 n = a.st->n0[s];
    const uint32_t lane = __lane_id();
    const int wv = threadIdx.x / 64;
    uint32_t *hist = hist_sh[wv];
    uint16_t *order = order_sh[wv];
    uint32_t *nsub = nsub_sh[wv];
    const u64 nwaves = (u64)gridDim.x * (kBlock / 64);
    const uint32_t tile = a.tiled_slots, qn = tile / 64;
    Tally<R> t;
    for (u64 t0 = ((u64)blockIdx.x * (kBlock / 64) + wv) * tile; t0 < n; t0 += nwaves * tile) {
        hist[lane] = 0;
        __syncwarp();
        uint32_t kr[kTiledSlots / 64];  // key << 16 | rank
#pragma unroll
        for (int q = 0; q < kTiledSlots / 64; ++q) {
            const u64 i = t0 + q * 64 + lane;
            const bool in = (uint32_t)q < qn && i < n;
            Lepton<R> p;
            const uint32_t N = lepton_fetch(a, s, i, in, p, t, a.dt);
            if (in && N == 0 && a.sp[s].events) a.sp[s].events[i] = 0;
            nsub[q * 64 + lane] = N;
            const uint32_t key = N ? kTileKeys - (N < kTileKeys - 1 ? N : kTileKeys - 1) : 0u;
            kr[q] = key ? (key << 16) | atomicAdd(&hist[key], 1u) : 0u;
        }
        __syncwarp();
        const uint32_t h = lane >= 1 ? hist[lane] : 0u;
        uint32_t incl = h;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o);
            if ((int)lane >= o) incl += v;
        }
        const uint32_t total = __shfl(incl, 63);
        __syncwarp();
        hist[lane] = incl - h;
        __syncwarp();
#pragma unroll
        for (int q = 0; q < kTiledSlots / 64; ++q)
            if (kr[q]) order[hist[kr[q] >> 16] + (kr[q] & 0xFFFFu)] = (uint16_t)(q * 64 + lane);
        __syncwarp();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + lane;
            const bool has = p < total;
            const uint32_t idx = has ? order[p] : 0u;
            const u64 i = t0 + idx;
            const uint32_t N = has ? nsub[idx] : 0u;
            const Lepton<R> q = has ? load_lepton<R>(a, s, i) : Lepton<R>{0, 0, 0, 0, 0, 0, 0, 0, 0};
            LeptonRunner<R, SURR>::run(a, s, i, N, q, L, cb, t);
        }
        __syncwarp();
    }
    flush_children_block(L.cb, a.sp[2], a.seed, step_of(a));
    flush_tally(t, a.st, s);
}

// Persistent: each wave claims chunk consecutive queue entries at a time.  The
// optical-depth instance's LDS (the network, the rate table, the larger child
// buffers) fits two blocks per compute unit, so it is compiled for two waves per
// SIMD and may use the registers that allows.
template <class R, bool SURR>
__global__ __launch_bounds__(kBlock, SURR ? 2 : 3) void k_heavy(StepArgs a) {
    __shared__ LeptonLds<R, SURR> L;
    auto &cb = lepton_lds_init<R, SURR>(a, L);
    const int s = blockIdx.y;
    const u64 H = a.st->heavy[s];
    const uint32_t chunk = a.chunk;
    Tally<R> t;
    // the first chunk of every wave is assigned statically; later ones are
    // claimed from the queue, which starts after all static chunks
    const u64 nwaves = (u64)gridDim.x * (kBlock / 64);
    u64 base = ((u64)blockIdx.x * (kBlock / 64) + threadIdx.x / 64) * chunk;
    for (;;) {
        if (base >= H) break;
        const u64 end = base + chunk < H ? base + chunk : H;
        for (u64 j0 = base; j0 < end; j0 += 64) {
            const u64 j = j0 + __lane_id();
            const bool has = j < end;
            const u64 i = has ? a.queue[s][j] : 0;
            const uint32_t N = has ? a.nsub[s][i] : 0u;
            const Lepton<R> q = has ? load_lepton<R>(a, s, i) : Lepton<R>{0, 0, 0, 0, 0, 0, 0, 0, 0};
            LeptonRunner<R, SURR>::template run<SURR>(a, s, i, N, q, L, cb, t);
            t.particles += has;
        }
        u64 nb = 0;
        if (__lane_id() == 0) nb = nwaves * chunk + atomicAdd(&a.st->queue[s], (u64)chunk);
        base = __shfl(nb, 0);
    }
    flush_children_block(L.cb, a.sp[2], a.seed, step_of(a));
    flush_tally(t, a.st, s, 1);
}

// The sampling loop of one photon that can decay, from its queued step-start
// values.
template <class R>
__device__ __forceinline__ void photon_sample_one(const StepArgs &a, u64 i, R kx, R ky, R kz, double x0, double y0,
                                                  double z0, const PhotonStart &ps, const SynTable<R> &tab,
                                                  const PairTable &pt, Tally<R> &ts) {
    photon_sample<R>(a, i, kx, ky, kz, x0, y0, z0, ps, tab, pt, ts);
    ts.particles++;
}

// Algorithm 2 for every photon, in one pass.  Each lane loads kPhotonBatch
// photons per round (all loads issued before use; a uniform field, stride 0, is
// loaded once), computes the step-start bound and writes every photon's
// end-of-step position (the same float sum of sub-step moves the sampling loop
// takes), with coalesced stores.  Photons that cannot decay in this step
// (photon_quiet) are then done.  The others go to a wave-local LDS queue with
// their momentum and start position, which is drained 64 photons at a time, so
// the sampling loops run with all lanes busy and without reading the photon
// records again (only the id); a photon that decays leaves its children at its
// start position plus the moves up to the decay.  The pass covers the slots
// lo..hi of the device state; in a cascade pass (gen >= 1) each photon runs over
// the rest of the step from its birth time.
constexpr int kPhotonBatch = 2;
// The queue is drained after each group of 64 photons, so it holds at most 63 + 64
// entries; at 128 entries the kernel's LDS (35 KB per block) and registers allow 4
// waves per SIMD.
constexpr int kPhotonQueue = 128;

template <class R>
__global__ __launch_bounds__(kBlock) void k_photon(StepArgs a) {
    __shared__ SynTable<R> tab;
    __shared__ u64 queue_sh[kBlock / 64][kPhotonQueue];
    __shared__ double qchi_sh[kBlock / 64][kPhotonQueue], qeps_sh[kBlock / 64][kPhotonQueue];
    __shared__ double qx_sh[kBlock / 64][3][kPhotonQueue];
    __shared__ R qk_sh[kBlock / 64][3][kPhotonQueue];
    __shared__ uint32_t qn_sh[kBlock / 64][kPhotonQueue];
    __shared__ PairTable pt;
    pair_stage(pt);
    syn_stage(tab);
    const u64 lo = a.st->lo[2], n = a.st->hi[2];
    const SpeciesDev &sp = a.sp[2];
    const FieldDev &fl = a.fl[2];
    const bool uni = fl.stride == 0;
    const uint32_t lane = __lane_id();
    u64 *queue = queue_sh[threadIdx.x / 64];
    double *qchi = qchi_sh[threadIdx.x / 64], *qeps = qeps_sh[threadIdx.x / 64];
    double(*qx)[kPhotonQueue] = qx_sh[threadIdx.x / 64];
    R(*qk)[kPhotonQueue] = qk_sh[threadIdx.x / 64];
    uint32_t *qn = qn_sh[threadIdx.x / 64];
    uint32_t queued = 0;  // wave-uniform
    R fu[6] = {0, 0, 0, 0, 0, 0};
    if (uni) {
        fu[0] = ((const R *)fl.ex)[0];
        fu[1] = ((const R *)fl.ey)[0];
        fu[2] = ((const R *)fl.ez)[0];
        fu[3] = ((const R *)fl.bx)[0];
        fu[4] = ((const R *)fl.by)[0];
        fu[5] = ((const R *)fl.bz)[0];
    }
    Tally<R> tt[2];  // all photons; the sampled ones
    Tally<R> &t = tt[0], &ts = tt[1];
    const u64 G = (u64)gridDim.x * kBlock;
    // wave-uniform loop: photon b of this lane is slot wbase + lane + b G
    for (u64 wbase = lo + (u64)blockIdx.x * kBlock + (threadIdx.x & ~63u); wbase < n; wbase += G * kPhotonBatch) {
        const u64 i0 = wbase + lane;
        R k[kPhotonBatch][3], f[kPhotonBatch][6];
        double x[kPhotonBatch][3];
#pragma unroll
        for (int b = 0; b < kPhotonBatch; ++b) {
            const u64 i = i0 + b * G;
            const bool in = i < n;
            k[b][0] = in ? ((const R *)sp.ux)[i] : R(0);
            k[b][1] = in ? ((const R *)sp.uy)[i] : R(0);
            k[b][2] = in ? ((const R *)sp.uz)[i] : R(0);
            x[b][0] = in ? sp.x[i] : 0.0;
            x[b][1] = in ? sp.y[i] : 0.0;
            x[b][2] = in ? sp.z[i] : 0.0;
            const u64 fi = in ? i * fl.stride : 0;
#pragma unroll
            for (int c = 0; c < 6; ++c) f[b][c] = fu[c];
            if (!uni && in) {
                f[b][0] = ((const R *)fl.ex)[fi];
                f[b][1] = ((const R *)fl.ey)[fi];
                f[b][2] = ((const R *)fl.ez)[fi];
                f[b][3] = ((const R *)fl.bx)[fi];
                f[b][4] = ((const R *)fl.by)[fi];
                f[b][5] = ((const R *)fl.bz)[fi];
            }
        }
        uint32_t need = 0;  // bit b: photon b can decay
        PhotonStart pst[kPhotonBatch];
#pragma unroll
        for (int b = 0; b < kPhotonBatch; ++b) {
            const u64 i = i0 + b * G;
            if (i >= n) break;
            const R kx = k[b][0], ky = k[b][1], kz = k[b][2];
            if (!(finite3(kx, ky, kz) && finite3(f[b][0], f[b][1], f[b][2]) &&
                  finite3(f[b][3], f[b][4], f[b][5]))) {
                t.nonfinite++;
                a.alive[i] = 1;
                if (sp.events) sp.events[i] = 0;
                continue;
            }
            const double eps = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
            const double chi = chi_def(eps, kx, ky, kz, f[b][0], f[b][1], f[b][2], f[b][3], f[b][4], f[b][5]);
            const double t0 = a.gen ? sp.birth[i] : 0.0;
            const double dti = a.dt - t0;
            bool capped;
            uint32_t N = photon_nsub(a, chi, eps, dti, &capped);
            t.capped += capped;
            if (a.cells.n[1]) N = cell_nsub(a, 1, a.cells.slot[2][i], N);
            const double st = dti / (double)N;
            const R inv = eps > 0.0 ? (R)(1.0 / eps) : R(0);
            const R dirx = kx * inv, diry = ky * inv, dirz = kz * inv;
            const R str = (R)st;
            R dx = 0, dy = 0, dz = 0;
            for (uint32_t q = 0; q < N; ++q) {
                dx += dirx * str;
                dy += diry * str;
                dz += dirz * str;
            }
            sp.x[i] = x[b][0] + (double)dx;
            sp.y[i] = x[b][1] + (double)dy;
            sp.z[i] = x[b][2] + (double)dz;
            if (!photon_quiet<R>(chi, eps, st)) {
                need |= 1u << b;
                pst[b].eps = eps;
                pst[b].chi = chi;
                pst[b].t0 = t0;
                pst[b].N = N;
                continue;
            }
            a.alive[i] = 1;
            if (sp.events) sp.events[i] = 0u;
            t.substeps += N;
        }
        // queue the photons that can decay, group by group; sample 64 at a time
#pragma unroll
        for (int b = 0; b < kPhotonBatch; ++b) {
            const bool nb = (need >> b) & 1u;
            const u64 m = __ballot(nb);
            if (nb) {
                const uint32_t q = queued + (uint32_t)__popcll(m & lanemask_lt());
                queue[q] = i0 + b * G;
                qchi[q] = pst[b].chi;
                qeps[q] = pst[b].eps;
                qn[q] = pst[b].N;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    qx[c][q] = x[b][c];
                    qk[c][q] = k[b][c];
                }
            }
            queued += (uint32_t)__popcll(m);
            __syncwarp();
            if (queued >= 64) {  // at most 127 queued here, at most 63 after
                queued -= 64;
                const uint32_t q = queued + lane;
                const u64 iq = queue[q];
                const PhotonStart ps = {qeps[q], qchi[q], a.gen ? sp.birth[iq] : 0.0, qn[q]};
                photon_sample_one<R>(a, iq, qk[0][q], qk[1][q], qk[2][q], qx[0][q], qx[1][q], qx[2][q], ps, tab, pt,
                                     ts);
                __syncwarp();
            }
        }
    }
    if (lane < queued) {
        const u64 iq = queue[lane];
        const PhotonStart ps = {qeps[lane], qchi[lane], a.gen ? sp.birth[iq] : 0.0, qn[lane]};
        photon_sample_one<R>(a, iq, qk[0][lane], qk[1][lane], qk[2][lane], qx[0][lane], qx[1][lane], qx[2][lane], ps,
                             tab, pt, ts);
    }
    const int work[2] = {0, 2};
    flush_tallies<R, 2>(tt, work, a.st, 2);
}

// ---------------------------------------------------------------------------
// Photon optical-depth path (pair sampler = surrogate, mixed precision).  In the
// frozen field of a step a photon's chi and energy are constant, so its decay rate
// W = alpha (chi / eps) T(chi) is too, and the time of its decay follows from the
// optical depth without sub-steps: with tau left, it decays at t = tau / W if that
// falls inside the step (else tau -= W dt).  The electron's energy fraction is
// drawn from eq. (2) at that chi by rejection against the fitted envelope.
// ---------------------------------------------------------------------------
// Key tag of the photon path's random stream: the draws of photon id in step
// `step` are Philox blocks (id_lo, id_hi, step, j) under the seed key xor'ed with
// this tag, j counting the photon's draws within the step.
constexpr uint32_t kPairTagLo = 0x7F4A7C15u, kPairTagHi = 0xBB67AE85u;

// Electron energy fraction d in (0, 1) from the Baier-Katkov density at chi by
// rejection; every candidate costs one half of a Philox block.
__device__ __forceinline__ float pair_split_reject(float chi, const SynTable<float> &tab, const PairTable &pt,
                                                   uint32_t idlo, uint32_t idhi, uint32_t step, uint32_t klo,
                                                   uint32_t khi, uint32_t &j, Tally<float> &tl) {
    const float env = pair_envelope(chi, pt);
    u32x4 w = {0u, 0u, 0u, 0u};
    float d = 0.5f;
    for (uint32_t it = 0; it < kMaxRejections; ++it) {
        if ((it & 1u) == 0u) w = philox10(idlo, idhi, step, j++, klo, khi);
        const bool odd = (it & 1u) != 0u;
        d = u24(odd ? w.z : w.x);
        const float y = u24(odd ? w.w : w.y);
        const float dd = d * (1.0f - d);
        float F, G;
        syn_eval((2.0f / 3.0f) * rcp(chi * dd), tab, F, G);
        const float dens = 1.5f * chi * (G - dd * F);
        tl.fb_draws++;
        tl.env_clips += dens > env;
        if (y * env < dens) break;
    }
    return d;
}

// Network of the energy split in LDS (NET instance only).
template <bool NET>
struct PairNetLds {};
template <>
struct PairNetLds<true> {
    MlpLds M;
    MlpWave ws[kBlock / 64];
};

template <bool NET>
__global__ __launch_bounds__(kBlock) void k_photon_surr(StepArgs a) {
    __shared__ SynTable<float> tab;
    __shared__ PairTable pt;
    __shared__ PairNetLds<NET> net;
    if constexpr (NET) mlp_stage(a.pair_model, net.M);
    pair_stage(pt);
    syn_stage(tab);
    using R = float;
    const u64 n = a.st->hi[2];
    const SpeciesDev &sp = a.sp[2];
    const SpeciesDev &el = a.sp[0];
    const SpeciesDev &po = a.sp[1];
    const FieldDev &fl = a.fl[2];
    const uint32_t step = step_of(a);
    const uint32_t klo = (uint32_t)a.seed ^ kPairTagLo, khi = (uint32_t)(a.seed >> 32) ^ kPairTagHi;
    Tally<R> tt[2];  // all photons; those that decayed (their split draws)
    Tally<R> &t = tt[0], &ts = tt[1];
    for (u64 i0 = (u64)blockIdx.x * kBlock + (threadIdx.x & ~63u); i0 < n; i0 += (u64)gridDim.x * kBlock) {
        const u64 i = i0 + __lane_id();
        const bool in = i < n;
        bool decay = false, ok = false;
        double ts_move = 0.0, tau = 1.0, eps = 0.0;
        float chi = 0.0f;
        R kx = 0, ky = 0, kz = 0;
        uint64_t pid = 0;
        uint32_t j = 0;
        if (in) {
            kx = ((const R *)sp.ux)[i];
            ky = ((const R *)sp.uy)[i];
            kz = ((const R *)sp.uz)[i];
            const u64 f = i * fl.stride;
            const R ex = ((const R *)fl.ex)[f], ey = ((const R *)fl.ey)[f], ez = ((const R *)fl.ez)[f];
            const R bx = ((const R *)fl.bx)[f], by = ((const R *)fl.by)[f], bz = ((const R *)fl.bz)[f];
            ok = finite3(kx, ky, kz) && finite3(ex, ey, ez) && finite3(bx, by, bz);
            if (!ok) {
                t.nonfinite++;
                a.alive[i] = 1;
                if (sp.events) sp.events[i] = 0;
            } else {
                eps = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
                chi = (float)chi_def(eps, kx, ky, kz, ex, ey, ez, bx, by, bz);
                tau = sp.tau[i];
                // the id keys the random stream: only a photon that draws a new optical
                // depth or decays needs it (a few in a hundred), so it is loaded on demand
                const bool fresh = !(tau > 0.0);
                if (fresh) {
                    pid = sp.id[i];
                    const u32x4 w = philox10((uint32_t)pid, (uint32_t)(pid >> 32), step, j++, klo, khi);
                    tau = neg_ln(u53(w.x, w.y));
                }
                // rate per unit time; photons of zero energy do not decay
                const double W = eps > 0.0 ? kAlpha * (double)chi / eps * (double)pair_t(chi, pt) : 0.0;
                const double Wdt = W * a.dt;
                decay = tau <= Wdt;
                if (decay && !fresh) pid = sp.id[i];
                ts_move = decay ? tau / W : a.dt;
                tau = decay ? tau : tau - Wdt;
                t.substeps += 1;
                t.particles++;
            }
        }
        // the electron's energy fraction of the decaying photons: from the network
        // (batched over the wave's decaying lanes) where it serves this chi, else by
        // rejection
        float d = 0.5f;
        bool use_net = false;
        if constexpr (NET) {
            float sin = 0.0f, up = 0.0f;
            bool upper = false;
            if (decay) {
                const u32x4 w = philox10((uint32_t)pid, (uint32_t)(pid >> 32), step, j++, klo, khi);
                const float u = u24(w.x);
                upper = u >= 0.5f;
                up = fabsf(2.0f * u - 1.0f);
                bool in_range;
                int bin;
                sin = mlp_input_s(net.M, chi, in_range, bin);
                use_net = in_range && !net.M.fallback[bin];
            }
            if (__ballot(use_net)) {
                const float y = mlp_infer_wave(net.M, net.ws[threadIdx.x / 64], use_net, sin, mlp_input_v_pair(up));
                if (use_net) d = pair_d_of_y(y, chi, upper);
            }
        }
        if (decay) {
            if (use_net) {
                ts.learned++;
            } else {
                d = pair_split_reject(chi, tab, pt, (uint32_t)pid, (uint32_t)(pid >> 32), step, klo, khi, j, ts);
                ts.fallback++;
            }
            ts.particles++;
            t.events++;
        }
        // move (straight line over the time it lived in this step)
        double dirx = 0.0, diry = 0.0, dirz = 0.0;
        if (in && ok) {
            const double inv = eps > 0.0 ? 1.0 / eps : 0.0;
            dirx = kx * inv;
            diry = ky * inv;
            dirz = kz * inv;
            sp.x[i] += dirx * ts_move;
            sp.y[i] += diry * ts_move;
            sp.z[i] += dirz * ts_move;
            sp.tau[i] = tau;
            a.alive[i] = decay ? 0 : 1;
            if (sp.events) sp.events[i] = decay ? 1u : 0u;
        }
        // pair creation: electron with d eps, positron with (1 - d) eps, along k
        const u64 m = __ballot(decay);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            u64 be = 0, bp = 0, bd = 0;
            if (__lane_id() == leader) {
                const u64 c = (u64)__popcll(m);
                be = atomicAdd(el.n, c);
                bp = atomicAdd(po.n, c);
                bd = atomicAdd(&a.st->dead, c);
            }
            be = __shfl(be, leader);
            bp = __shfl(bp, leader);
            bd = __shfl(bd, leader);
            if (decay) {
                const u64 r = (u64)__popcll(m & lanemask_lt());
                a.dead_idx[bd + r] = i;
                const double px = sp.x[i], py = sp.y[i], pz = sp.z[i];
                const R w = ((const R *)sp.w)[i];
                const R epsr = (R)eps;
                const R ge = d * epsr, gp = (1.0f - d) * epsr;
                const R ue = sqrt_(fmaxf(ge * ge - 1.0f, 0.0f));
                const R up = sqrt_(fmaxf(gp * gp - 1.0f, 0.0f));
                const R fx = (R)dirx, fy = (R)diry, fz = (R)dirz;
                if (be + r < el.cap) {
                    const u64 q = be + r;
                    el.x[q] = px;
                    el.y[q] = py;
                    el.z[q] = pz;
                    ((R *)el.ux)[q] = ue * fx;
                    ((R *)el.uy)[q] = ue * fy;
                    ((R *)el.uz)[q] = ue * fz;
                    ((R *)el.w)[q] = w;
                    el.id[q] = child_id(a.seed, pid, step, 0, 0);
                    if (el.parent) el.parent[q] = pid;
                    if (el.tau) el.tau[q] = -1.0;
                }
                if (bp + r < po.cap) {
                    const u64 q = bp + r;
                    po.x[q] = px;
                    po.y[q] = py;
                    po.z[q] = pz;
                    ((R *)po.ux)[q] = up * fx;
                    ((R *)po.uy)[q] = up * fy;
                    ((R *)po.uz)[q] = up * fz;
                    ((R *)po.w)[q] = w;
                    po.id[q] = child_id(a.seed, pid, step, 0, 1);
                    if (po.parent) po.parent[q] = pid;
                    if (po.tau) po.tau[q] = -1.0;
                }
            }
        }
    }
    const int work[2] = {0, 2};
    flush_tallies<R, 2>(tt, work, a.st, 2);
}

// Elementwise T(chi) of the pair-rate fit.
__global__ __launch_bounds__(kBlock) void k_pair_rate(const float *__restrict__ chi, float *__restrict__ out, u64 n) {
    __shared__ PairTable t;
    pair_stage(t);
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock)
        out[i] = pair_t(chi[i], t);
}

// Sub-steps per cell, before the passes of a step: clear the counts, then raise each
// cell's count of a group to the largest own count among its particles present at the
// step start (the same own counts the passes compute), and record every slot's cell.
__global__ __launch_bounds__(kBlock) void k_cell_clear(StepArgs a) {
    const u64 nc = (u64)a.cells.nx * a.cells.ny * a.cells.nz;
    for (u64 c = (u64)blockIdx.x * kBlock + threadIdx.x; c < nc; c += (u64)gridDim.x * kBlock) {
        a.cells.n[0][c] = 0;
        a.cells.n[1][c] = 0;
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_cell_max(StepArgs a) {
    const int s = blockIdx.y;
    if (s < 2 ? !a.emission : !a.pairs) return;
    const u64 n = a.st->n0[s];
    const SpeciesDev &sp = a.sp[s];
    const FieldDev &fl = a.fl[s];
    uint32_t *cn = a.cells.n[s < 2 ? 0 : 1];
    Tally<R> t;  // not flushed: the passes count capping and non-finite input
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock) {
        uint32_t N = 0;
        if (s < 2) {
            N = lepton_nsub_own(a, load_lepton<R>(a, s, i), t, a.dt);
        } else {
            const R kx = ((const R *)sp.ux)[i], ky = ((const R *)sp.uy)[i], kz = ((const R *)sp.uz)[i];
            const u64 fi = i * fl.stride;
            const R f[6] = {((const R *)fl.ex)[fi], ((const R *)fl.ey)[fi], ((const R *)fl.ez)[fi],
                            ((const R *)fl.bx)[fi], ((const R *)fl.by)[fi], ((const R *)fl.bz)[fi]};
            if (finite3(kx, ky, kz) && finite3(f[0], f[1], f[2]) && finite3(f[3], f[4], f[5])) {
                const double eps = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
                const double chi = chi_def(eps, kx, ky, kz, f[0], f[1], f[2], f[3], f[4], f[5]);
                bool capped;
                N = photon_nsub(a, chi, eps, a.dt, &capped);
            }
        }
        uint32_t cell;
        const bool in = cell_of(a.cells, sp.x[i], sp.y[i], sp.z[i], cell);
        a.cells.slot[s][i] = in ? cell + 1 : 0u;
        // counts only grow during this kernel: a read that already shows N or more
        // (stale values are smaller) makes the atomic unnecessary; in crowded cells
        // this spares most of them
        if (N && in && cn[cell] < N) atomicMax(&cn[cell], N);
    }
}

__global__ void k_begin(StepArgs a) {
    DevState *st = a.st;
    for (int k = threadIdx.x; k < 2 * kBins; k += blockDim.x) st->hist[k / kBins][k % kBins] = 0;
    if (threadIdx.x == 0) {
        for (int s = 0; s < 3; ++s) {
            const u64 n = *a.sp[s].n;
            st->n0[s] = n < a.sp[s].cap ? n : a.sp[s].cap;
            st->lo[s] = 0;
            st->hi[s] = st->n0[s];
            if (s < 2 ? a.emission : a.pairs) st->particles[s] += st->n0[s];
        }
        st->dead = 0;
    }
}

// Cascade pass: the next pass covers the particles appended since the previous
// pass's range was fixed (clamped to capacity; an overflow is reported by k_end).
__global__ void k_gen(StepArgs a) {
    if (threadIdx.x == 0) {
        DevState *st = a.st;
        for (int s = 0; s < 3; ++s) {
            const u64 n = *a.sp[s].n;
            st->lo[s] = st->hi[s];
            st->hi[s] = n < a.sp[s].cap ? n : a.sp[s].cap;
            if (s < 2 ? a.emission : a.pairs) st->particles[s] += st->hi[s] - st->lo[s];
        }
    }
}

__global__ void k_end(StepArgs a) {
    if (threadIdx.x == 0) {
        DevState *st = a.st;
        for (int s = 0; s < 3; ++s) {
            const u64 n = *a.sp[s].n;
            if (n > a.sp[s].cap) {
                st->status_bits |= 1ull;
                if (n > st->required[s]) st->required[s] = n;
                *a.sp[s].n = a.sp[s].cap;
            }
        }
        const u64 ntot = *a.sp[2].n;
        st->ntot = ntot;
        st->S = ntot - st->dead;
        st->holes = 0;
        st->movers = 0;
        st->steps += 1;
        if (a.step_dev) *a.step_dev += 1u;
    }
}

// Holes: decayed slots below S (from the dead list).  Movers: live slots in
// [S, ntot) (a slot there is live if it survived the last pass that covered it,
// or if it was appended after that pass's range was fixed).
__global__ __launch_bounds__(kBlock) void k_fill(StepArgs a) {
    const DevState *st = a.st;
    const u64 D = st->dead;
    if (D == 0) return;
    const u64 S = st->S, done = st->hi[2];  // slots below done carry an alive flag
    // work items: D dead-list entries, then the D slots of [S, ntot)
    for (u64 t0 = (u64)blockIdx.x * kBlock; t0 < 2 * D; t0 += (u64)gridDim.x * kBlock) {
        const u64 t = t0 + threadIdx.x;
        bool hole = false, mover = false;
        u64 p = 0;
        if (t < D) {
            p = a.dead_idx[t];
            hole = p < S;
        } else if (t < 2 * D) {
            p = S + (t - D);
            mover = p >= done || a.alive[p] != 0;
        }
        const u64 mh = __ballot(hole), mm = __ballot(mover);
        u64 bh = 0, bm = 0;
        if (__lane_id() == 0) {
            if (mh) bh = atomicAdd(&a.st->holes, (u64)__popcll(mh));
            if (mm) bm = atomicAdd(&a.st->movers, (u64)__popcll(mm));
        }
        bh = __shfl(bh, 0);
        bm = __shfl(bm, 0);
        if (hole) a.hole_idx[bh + __popcll(mh & lanemask_lt())] = p;
        if (mover) a.mover_idx[bm + __popcll(mm & lanemask_lt())] = p;
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_move(StepArgs a) {
    const DevState *st = a.st;
    if (st->dead == 0) return;
    const u64 h = st->holes;  // equals st->movers
    const SpeciesDev &sp = a.sp[2];
    for (u64 r = (u64)blockIdx.x * kBlock + threadIdx.x; r < h; r += (u64)gridDim.x * kBlock) {
        const u64 d = a.hole_idx[r], s = a.mover_idx[r];
        sp.x[d] = sp.x[s];
        sp.y[d] = sp.y[s];
        sp.z[d] = sp.z[s];
        ((R *)sp.ux)[d] = ((const R *)sp.ux)[s];
        ((R *)sp.uy)[d] = ((const R *)sp.uy)[s];
        ((R *)sp.uz)[d] = ((const R *)sp.uz)[s];
        ((R *)sp.w)[d] = ((const R *)sp.w)[s];
        sp.id[d] = sp.id[s];
        if (sp.parent) sp.parent[d] = sp.parent[s];
        if (sp.birth) sp.birth[d] = sp.birth[s];
        if (sp.tau) sp.tau[d] = sp.tau[s];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *sp.n = st->S;
}

// ---------------------------------------------------------------------------
// Elementwise F, G.
// ---------------------------------------------------------------------------
// VEC: 16-byte loads of x and stores of F and G (4 floats or 2 doubles per lane and
// pass; the caller checks the pointers' alignment), which keeps more bytes in flight
// per wave than one element per lane; the elements past the last whole vector are
// done one per lane.
template <class R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_synchrotron(const R *__restrict__ x, R *__restrict__ F,
                                                        R *__restrict__ G, u64 n, DevState *st) {
    __shared__ SynTable<R> tab;
    syn_stage(tab);
    constexpr int V = VEC ? 16 / (int)sizeof(R) : 1;
    using Vec = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
    uint32_t bad = 0;
    const u64 stride = (u64)gridDim.x * kBlock;
    const u64 nv = VEC ? n / V : 0;   // whole vectors (none without the vector loop)
    auto one = [&](R z, R &f, R &g) {
        if (z >= R(0)) {
            syn_eval(z, tab, f, g);
        } else {
            f = g = (R)NAN;
            bad++;
        }
    };
    if constexpr (VEC) {
        for (u64 v = (u64)blockIdx.x * kBlock + threadIdx.x; v < nv; v += stride) {
            const Vec zv = reinterpret_cast<const Vec *>(x)[v];
            const R *z = reinterpret_cast<const R *>(&zv);
            Vec fv, gv;
            R *f = reinterpret_cast<R *>(&fv), *g = reinterpret_cast<R *>(&gv);
#pragma unroll
            for (int k = 0; k < V; ++k) one(z[k], f[k], g[k]);
            if (F) reinterpret_cast<Vec *>(F)[v] = fv;
            if (G) reinterpret_cast<Vec *>(G)[v] = gv;
        }
    }
    for (u64 i = nv * V + (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        R f, g;
        one(x[i], f, g);
        if (F) F[i] = f;
        if (G) G[i] = g;
    }
    const uint32_t b = wave_sum(bad);
    if (__lane_id() == 0 && b) {
        atomicAdd(&st->nonfinite, (u64)b);
        atomicOr(&st->status_bits, 2ull);
    }
}

// Elementwise chi q(chi) of the rate fit.
__global__ __launch_bounds__(kBlock) void k_rate(const float *__restrict__ chi, float *__restrict__ out, u64 n) {
    __shared__ RateTable t;
    rate_stage(t);
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock)
        out[i] = rate_chi_q(chi[i], t);
}

template <class R>
hipError_t launch_t(int id, const StepArgs &a, int blocks, hipStream_t s) {
    const dim3 blk(kBlock), g1(blocks), g2(blocks, 2);
    switch (id) {
        case K_BEGIN: hipLaunchKernelGGL(k_begin, dim3(1), dim3(256), 0, s, a); break;
        case K_PHOTON: hipLaunchKernelGGL(k_photon<R>, g1, blk, 0, s, a); break;
        case K_LEPTON:
            if constexpr (std::is_same<R, float>::value)
                if (a.sampler) {
                    hipLaunchKernelGGL((k_lepton<float, true>), g2, blk, 0, s, a);
                    break;
                }
            hipLaunchKernelGGL((k_lepton<R, false>), g2, blk, 0, s, a);
            break;
        case K_PREPASS:
            if constexpr (std::is_same<R, float>::value)
                if (a.sampler) {
                    hipLaunchKernelGGL((k_prepass<float, true>), g2, blk, 0, s, a);
                    break;
                }
            hipLaunchKernelGGL((k_prepass<R, false>), g2, blk, 0, s, a);
            break;
        case K_SCAN: hipLaunchKernelGGL(k_scan, dim3(1, 2), dim3(kBins), 0, s, a); break;
        case K_SCATTER: hipLaunchKernelGGL(k_scatter, g2, blk, 0, s, a); break;
        case K_LIGHT:
            if constexpr (std::is_same<R, float>::value)
                if (a.sampler) {
                    hipLaunchKernelGGL((k_light<float, true>), g2, blk, 0, s, a);
                    break;
                }
            hipLaunchKernelGGL((k_light<R, false>), g2, blk, 0, s, a);
            break;
        case K_HEAVY:
            if constexpr (std::is_same<R, float>::value)
                if (a.sampler) {
                    hipLaunchKernelGGL((k_heavy<float, true>), g2, blk, 0, s, a);
                    break;
                }
            hipLaunchKernelGGL((k_heavy<R, false>), g2, blk, 0, s, a);
            break;
        case K_TILED:
            if constexpr (std::is_same<R, float>::value)
                if (a.sampler) {
                    hipLaunchKernelGGL((k_tiled<float, true>), g2, blk, 0, s, a);
                    break;
                }
            hipLaunchKernelGGL((k_tiled<R, false>), g2, blk, 0, s, a);
            break;
        case K_END: hipLaunchKernelGGL(k_end, dim3(1), dim3(64), 0, s, a); break;
        case K_GEN: hipLaunchKernelGGL(k_gen, dim3(1), dim3(64), 0, s, a); break;
        case K_CELL_CLEAR: hipLaunchKernelGGL(k_cell_clear, g1, blk, 0, s, a); break;
        case K_CELL_MAX: hipLaunchKernelGGL(k_cell_max<R>, dim3(blocks, 3), blk, 0, s, a); break;
        case K_PHOTON_SURR:
            if constexpr (std::is_same<R, float>::value) {
                if (a.pair_model)
                    hipLaunchKernelGGL(k_photon_surr<true>, g1, blk, 0, s, a);
                else
                    hipLaunchKernelGGL(k_photon_surr<false>, g1, blk, 0, s, a);
                break;
            }
            return hipErrorInvalidValue;
        case K_FILL: hipLaunchKernelGGL(k_fill, g1, blk, 0, s, a); break;
        case K_MOVE: hipLaunchKernelGGL(k_move<R>, g1, blk, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_kernel(int id, const StepArgs &a, int precision, int blocks, hipStream_t s) {
    if (a.sampler && precision == 0) return hipErrorInvalidValue;  // surrogate: mixed precision only
    return precision == 0 ? launch_t<double>(id, a, blocks, s) : launch_t<float>(id, a, blocks, s);
}

hipError_t launch_rate(const float *chi, float *out, u64 n, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_rate, dim3(blocks), dim3(kBlock), 0, s, chi, out, n);
    return hipGetLastError();
}

hipError_t launch_pair_rate(const float *chi, float *out, u64 n, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_rate, dim3(blocks), dim3(kBlock), 0, s, chi, out, n);
    return hipGetLastError();
}

hipError_t launch_synchrotron(const void *x, void *F, void *G, u64 n, int dtype, DevState *st,
                              int blocks, hipStream_t s) {
    const bool vec = (((uintptr_t)x | (uintptr_t)F | (uintptr_t)G) & 15u) == 0;
    if (dtype == 0) {
        if (vec)
            hipLaunchKernelGGL((k_synchrotron<float, true>), dim3(blocks), dim3(kBlock), 0, s, (const float *)x,
                               (float *)F, (float *)G, n, st);
        else
            hipLaunchKernelGGL((k_synchrotron<float, false>), dim3(blocks), dim3(kBlock), 0, s, (const float *)x,
                               (float *)F, (float *)G, n, st);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_synchrotron<double, true>), dim3(blocks), dim3(kBlock), 0, s, (const double *)x,
                               (double *)F, (double *)G, n, st);
        else
            hipLaunchKernelGGL((k_synchrotron<double, false>), dim3(blocks), dim3(kBlock), 0, s,
                               (const double *)x, (double *)F, (double *)G, n, st);
    }
    return hipGetLastError();
}

}  // namespace qed
