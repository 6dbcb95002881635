// Kernels of the QED event generator for gfx950 (wave64).
//
// One global step (Sec. 2.2) is the sequence
//   k_begin   snapshot the live counts (particles appended later in the step wait
//             for the next step);
//   k_photon  Algorithm 2 for every photon: straight-line sub-steps, pair creation
//             with density eq. (2); pairs are appended to the e-/e+ buffers and the
//             photon is flagged dead;
//   k_lepton  Algorithm 1 for every electron and positron: Boris sub-steps,
//             emission with density eq. (1); photons are appended with recoil on
//             the parent;
//   k_end     clamp counts to capacity (reporting overflow) and size the
//             photon compaction;
//   k_fill / k_move  fill the holes left by decayed photons in [0, S) with the
//             survivors found in [S, n), so the photon buffer is dense again.
// Appends use one atomic per wavefront: the accepting lanes are found with a
// ballot, the lowest one reserves popcount slots and each lane takes its rank.
// The sub-step count of a particle comes from the bounds f(b) of Sec. 3.1.1,
// evaluated in double from the start-of-step momentum and field.
#include "qed_device.hpp"
#include "qed_internal.hpp"
#include "qed_synchro.hpp"

#include <type_traits>

namespace qed {

namespace {

constexpr int kBlock = 256;

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
    uint32_t events = 0, clips = 0, capped = 0, nonfinite = 0;
    R max_p = 0;
};

template <class R>
__device__ __forceinline__ void flush_tally(const Tally<R> &t, DevState *st, int species) {
    const u64 sub = wave_sum(t.substeps);
    const uint32_t ev = wave_sum(t.events), cl = wave_sum(t.clips), cp = wave_sum(t.capped),
                   nf = wave_sum(t.nonfinite);
    const double mp = wave_max((double)t.max_p);
    if (__lane_id() == 0) {
        if (sub) atomicAdd(&st->substeps[species], sub);
        if (ev) atomicAdd(species == 2 ? &st->pairs : &st->emissions, (u64)ev);
        if (cl) atomicAdd(&st->clips, (u64)cl);
        if (cp) atomicAdd(&st->capped, (u64)cp);
        if (nf) {
            atomicAdd(&st->nonfinite, (u64)nf);
            atomicOr(&st->status_bits, 2ull);
        }
        if (mp > 0.0) atomicMax(&st->max_p_bits, (u64)__double_as_longlong(mp));
    }
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
__device__ __forceinline__ float chi_sub(float ux, float uy, float uz, float g, float ex, float ey,
                                         float ez, float bx, float by, float bz, float e2) {
    return chi_lepton_f32(ux, uy, uz, g, ex, ey, ez, bx, by, bz, e2);
}
__device__ __forceinline__ double chi_sub(double ux, double uy, double uz, double g, double ex,
                                          double ey, double ez, double bx, double by, double bz,
                                          double) {
    return chi_def(g, ux, uy, uz, ex, ey, ez, bx, by, bz);
}

// ---------------------------------------------------------------------------
// Algorithm 1 for one electron (species 0, q = -1) or positron (species 1, q = +1).
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void lepton_one(const StepArgs &a, int s, u64 i, const SynTable<R> &tab,
                                           Tally<R> &tl) {
    const SpeciesDev &sp = a.sp[s];
    const FieldDev &fl = a.fl[s];
    const SpeciesDev &ph = a.sp[2];
    R ux = ((const R *)sp.ux)[i], uy = ((const R *)sp.uy)[i], uz = ((const R *)sp.uz)[i];
    const u64 f = i * fl.stride;
    const R ex = ((const R *)fl.ex)[f], ey = ((const R *)fl.ey)[f], ez = ((const R *)fl.ez)[f];
    const R bx = ((const R *)fl.bx)[f], by = ((const R *)fl.by)[f], bz = ((const R *)fl.bz)[f];
    if (!(finite3(ux, uy, uz) && finite3(ex, ey, ez) && finite3(bx, by, bz))) {
        tl.nonfinite++;
        if (sp.events) sp.events[i] = 0;
        return;
    }
    const uint64_t pid = sp.id[i];
    const R w = ((const R *)sp.w)[i];
    // Algorithm 1, line 1: sub-step from the bound at the step start (double).
    const double gd = sqrt(1.0 + (double)ux * ux + (double)uy * uy + (double)uz * uz);
    const double chi0 = chi_def(gd, ux, uy, uz, ex, ey, ez, bx, by, bz);
    bool capped;
    const uint32_t N = nsub(bound_emission(chi0, gd, a.dt), a.p_max, a.max_sub, &capped);
    tl.capped += capped;
    const double st = a.dt / (double)N;
    const R hq = (R)((s == 0 ? -0.5 : 0.5) * st);
    const R hex = hq * ex, hey = hq * ey, hez = hq * ez;
    const R e2 = ex * ex + ey * ey + ez * ez;
    const R str = (R)st;
    // c b = kcb * chi / gamma with c = sqrt(3) alpha st / (pi gamma), b = 3 chi / 2
    const R kcb = (R)(1.5 * kSqrt3 * kAlpha / kPi * st);
    const uint32_t idlo = (uint32_t)pid, idhi = (uint32_t)(pid >> 32);
    const uint32_t klo = (uint32_t)a.seed, khi = (uint32_t)(a.seed >> 32);
    R dx = 0, dy = 0, dz = 0;
    uint32_t nev = 0;
    Draw<R> draw;
    for (uint32_t k = 0; k < N; ++k) {
        // line 3: Boris push and move
        boris<R>(ux, uy, uz, hex, hey, hez, hq, bx, by, bz);
        const R u2 = ux * ux + uy * uy + uz * uz;
        const R g = sqrt_(R(1) + u2);
        const R ig = rcp(g);
        const R vs = str * ig;
        dx += ux * vs;
        dy += uy * vs;
        dz += uz * vs;
        // line 4
        const R chi = chi_sub(ux, uy, uz, g, ex, ey, ez, bx, by, bz, e2);
        // line 5
        R x, y;
        draw.get(k, idlo, idhi, a.step, klo, khi, x, y);
        // line 6: y < 3 x^2 P(x^3) = (c b / x) ((1 - x^3) F(z) + x^6 G(z)),
        //         z = x^3 / (b (1 - x^3))
        const R x2 = x * x, x3 = x2 * x;
        const R omx3 = (R(1) - x) * (R(1) + x + x2);
        const R b = R(1.5) * chi;
        const R z = x3 * rcp(b * omx3);
        R F, G;
        syn_eval(z, tab, F, G);
        const R pm = kcb * chi * ig * rcp(x) * (omx3 * F + x3 * x3 * G);
        tl.max_p = fmax(tl.max_p, pm);
        tl.clips += pm > R(1);
        const bool acc = y < pm;
        // line 7: append the photon (one atomic per wave)
        const u64 m = __ballot(acc);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            u64 base = 0;
            if (__lane_id() == leader) base = atomicAdd(ph.n, (u64)__popcll(m));
            base = __shfl(base, leader);
            if (acc) {
                const u64 slot = base + (u64)__popcll(m & lanemask_lt());
                const R umag = sqrt_(u2);
                const R inv = umag > R(0) ? rcp(umag) : R(0);
                const R eph = x3 * g * inv;
                if (slot < ph.cap) {
                    ph.x[slot] = sp.x[i] + (double)dx;
                    ph.y[slot] = sp.y[i] + (double)dy;
                    ph.z[slot] = sp.z[i] + (double)dz;
                    ((R *)ph.ux)[slot] = ux * eph;
                    ((R *)ph.uy)[slot] = uy * eph;
                    ((R *)ph.uz)[slot] = uz * eph;
                    ((R *)ph.w)[slot] = w;
                    ph.id[slot] = child_id(a.seed, pid, a.step, k, 0);
                    if (ph.parent) ph.parent[slot] = pid;
                }
                // recoil: gamma' = (1 - delta) gamma along the same direction
                const R g1 = omx3 * g;
                const R u1 = sqrt_(fmax(g1 * g1 - R(1), R(0)));
                const R sc = u1 * inv;
                ux *= sc;
                uy *= sc;
                uz *= sc;
                nev++;
            }
        }
    }
    ((R *)sp.ux)[i] = ux;
    ((R *)sp.uy)[i] = uy;
    ((R *)sp.uz)[i] = uz;
    sp.x[i] += (double)dx;
    sp.y[i] += (double)dy;
    sp.z[i] += (double)dz;
    if (sp.events) sp.events[i] = nev;
    tl.substeps += N;
    tl.events += nev;
}

// ---------------------------------------------------------------------------
// Algorithm 2 for one photon.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void photon_one(const StepArgs &a, u64 i, const SynTable<R> &tab,
                                           Tally<R> &tl, uint32_t &dead_out) {
    const SpeciesDev &sp = a.sp[2];
    const FieldDev &fl = a.fl[2];
    const SpeciesDev &el = a.sp[0];
    const SpeciesDev &po = a.sp[1];
    const R kx = ((const R *)sp.ux)[i], ky = ((const R *)sp.uy)[i], kz = ((const R *)sp.uz)[i];
    const u64 f = i * fl.stride;
    const R ex = ((const R *)fl.ex)[f], ey = ((const R *)fl.ey)[f], ez = ((const R *)fl.ez)[f];
    const R bx = ((const R *)fl.bx)[f], by = ((const R *)fl.by)[f], bz = ((const R *)fl.bz)[f];
    if (!(finite3(kx, ky, kz) && finite3(ex, ey, ez) && finite3(bx, by, bz))) {
        tl.nonfinite++;
        a.alive[i] = 1;
        if (sp.events) sp.events[i] = 0;
        return;
    }
    const uint64_t pid = sp.id[i];
    const R w = ((const R *)sp.w)[i];
    const double eps = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
    // the field and k are frozen, so chi_g is the same at every sub-step
    const double chi = chi_def(eps, kx, ky, kz, ex, ey, ez, bx, by, bz);
    uint32_t N = 1;
    if (eps > 0.0) {
        bool capped;
        N = nsub(bound_pair(chi, eps, a.dt, a.pair_coef), a.p_max, a.max_sub, &capped);
        tl.capped += capped;
    }
    const double st = a.dt / (double)N;
    const R inv = eps > 0.0 ? (R)(1.0 / eps) : R(0);
    const R dirx = kx * inv, diry = ky * inv, dirz = kz * inv;
    // P_p(x) = alpha st sqrt(3)/(2 pi) (chi/eps) (G(z) - x(1-x) F(z)),  z = 2/(3 chi x (1-x))
    const R A = eps > 0.0 ? (R)(kAlpha * st * kSqrt3 / (2.0 * kPi) * chi / eps) : R(0);
    const R chir = (R)chi;
    const R epsr = (R)eps;
    const R str = (R)st;
    const uint32_t idlo = (uint32_t)pid, idhi = (uint32_t)(pid >> 32);
    const uint32_t klo = (uint32_t)a.seed, khi = (uint32_t)(a.seed >> 32);
    R dx = 0, dy = 0, dz = 0;
    bool dead = false;
    uint32_t used = 0;
    Draw<R> draw;
    for (uint32_t k = 0; k < N && !dead; ++k) {
        used = k + 1;
        // line 3: move at the speed of light
        dx += dirx * str;
        dy += diry * str;
        dz += dirz * str;
        // lines 5-6
        R x, y;
        draw.get(k, idlo, idhi, a.step, klo, khi, x, y);
        const R xx = x * (R(1) - x);
        const R z = R(2.0 / 3.0) * rcp(chir * xx);
        R F, G;
        syn_eval(z, tab, F, G);
        const R pp = A * (G - xx * F);
        tl.max_p = fmax(tl.max_p, pp);
        tl.clips += pp > R(1);
        const bool acc = y < pp;
        // lines 7-8: electron with x eps, positron with (1-x) eps, along k
        const u64 m = __ballot(acc);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            u64 be = 0, bp = 0;
            if (__lane_id() == leader) {
                be = atomicAdd(el.n, (u64)__popcll(m));
                bp = atomicAdd(po.n, (u64)__popcll(m));
            }
            be = __shfl(be, leader);
            bp = __shfl(bp, leader);
            if (acc) {
                const u64 r = (u64)__popcll(m & lanemask_lt());
                const double px = sp.x[i] + (double)dx, py = sp.y[i] + (double)dy,
                             pz = sp.z[i] + (double)dz;
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
                    el.id[j] = child_id(a.seed, pid, a.step, k, 0);
                    if (el.parent) el.parent[j] = pid;
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
                    po.id[j] = child_id(a.seed, pid, a.step, k, 1);
                    if (po.parent) po.parent[j] = pid;
                }
                dead = true;
            }
        }
    }
    sp.x[i] += (double)dx;
    sp.y[i] += (double)dy;
    sp.z[i] += (double)dz;
    a.alive[i] = dead ? 0 : 1;
    if (sp.events) sp.events[i] = dead ? 1u : 0u;
    tl.substeps += used;
    tl.events += dead;
    dead_out += dead;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_lepton(StepArgs a) {
    __shared__ SynTable<R> tab;
    syn_stage(tab);
    const u64 ne = a.st->n0[0], np = a.st->n0[1], total = ne + np;
    Tally<R> t;
    u64 sub_pos = 0;  // positron share of t.substeps
    for (u64 g = (u64)blockIdx.x * kBlock + threadIdx.x; g < total; g += (u64)gridDim.x * kBlock) {
        const int s = g < ne ? 0 : 1;
        const u64 before = t.substeps;
        lepton_one<R>(a, s, s ? g - ne : g, tab, t);
        if (s) sub_pos += t.substeps - before;
    }
    const u64 sp = wave_sum(sub_pos);
    if (__lane_id() == 0 && sp) atomicAdd(&a.st->substeps[1], sp);
    t.substeps -= sub_pos;
    flush_tally(t, a.st, 0);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_photon(StepArgs a) {
    __shared__ SynTable<R> tab;
    syn_stage(tab);
    const u64 n = a.st->n0[2];
    Tally<R> t;
    uint32_t dead = 0;
    for (u64 g = (u64)blockIdx.x * kBlock + threadIdx.x; g < n; g += (u64)gridDim.x * kBlock)
        photon_one<R>(a, g, tab, t, dead);
    flush_tally(t, a.st, 2);
    const uint32_t d = wave_sum(dead);
    if (__lane_id() == 0 && d) atomicAdd(&a.st->dead, (u64)d);
}

__global__ void k_begin(StepArgs a) {
    if (threadIdx.x == 0) {
        for (int s = 0; s < 3; ++s) {
            const u64 n = *a.sp[s].n;
            a.st->n0[s] = n < a.sp[s].cap ? n : a.sp[s].cap;
            if (s < 2 ? a.emission : a.pairs) a.st->particles[s] += a.st->n0[s];
        }
        a.st->dead = 0;
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
    }
}

// Collect holes (decayed photons) below S and survivors at or above S.
__global__ __launch_bounds__(kBlock) void k_fill(StepArgs a) {
    const DevState *st = a.st;
    if (st->dead == 0) return;
    const u64 ntot = st->ntot, S = st->S, n0 = st->n0[2];
    for (u64 p0 = (u64)blockIdx.x * kBlock; p0 < ntot; p0 += (u64)gridDim.x * kBlock) {
        const u64 p = p0 + threadIdx.x;
        const bool in = p < ntot;
        const bool dead = in && p < n0 && a.alive[p] == 0;
        const bool hole = in && p < S && dead;
        const bool mover = in && p >= S && !dead;
        const u64 mh = __ballot(hole), mm = __ballot(mover);
        const int lane = __lane_id();
        u64 bh = 0, bm = 0;
        if (lane == 0) {
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
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *sp.n = st->S;
}

// ---------------------------------------------------------------------------
// Elementwise F, G.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k_synchrotron(const R *__restrict__ x, R *__restrict__ F,
                                                        R *__restrict__ G, u64 n, DevState *st) {
    __shared__ SynTable<R> tab;
    syn_stage(tab);
    uint32_t bad = 0;
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock) {
        const R z = x[i];
        R f, g;
        if (z >= R(0)) {
            syn_eval(z, tab, f, g);
        } else {
            f = g = (R)NAN;
            bad++;
        }
        if (F) F[i] = f;
        if (G) G[i] = g;
    }
    const uint32_t b = wave_sum(bad);
    if (__lane_id() == 0 && b) {
        atomicAdd(&st->nonfinite, (u64)b);
        atomicOr(&st->status_bits, 2ull);
    }
}

}  // namespace

hipError_t launch_kernel(int id, const StepArgs &a, int precision, int blocks, hipStream_t s) {
    const bool f64 = precision == 0;
    switch (id) {
        case K_BEGIN:
            hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, a);
            break;
        case K_PHOTON:
            if (f64)
                hipLaunchKernelGGL(k_photon<double>, dim3(blocks), dim3(kBlock), 0, s, a);
            else
                hipLaunchKernelGGL(k_photon<float>, dim3(blocks), dim3(kBlock), 0, s, a);
            break;
        case K_LEPTON:
            if (f64)
                hipLaunchKernelGGL(k_lepton<double>, dim3(blocks), dim3(kBlock), 0, s, a);
            else
                hipLaunchKernelGGL(k_lepton<float>, dim3(blocks), dim3(kBlock), 0, s, a);
            break;
        case K_END:
            hipLaunchKernelGGL(k_end, dim3(1), dim3(64), 0, s, a);
            break;
        case K_FILL:
            hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, s, a);
            break;
        case K_MOVE:
            if (f64)
                hipLaunchKernelGGL(k_move<double>, dim3(blocks), dim3(kBlock), 0, s, a);
            else
                hipLaunchKernelGGL(k_move<float>, dim3(blocks), dim3(kBlock), 0, s, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_synchrotron(const void *x, void *F, void *G, u64 n, int dtype, DevState *st,
                              int blocks, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_synchrotron<float>, dim3(blocks), dim3(kBlock), 0, s, (const float *)x,
                           (float *)F, (float *)G, n, st);
    else
        hipLaunchKernelGGL(k_synchrotron<double>, dim3(blocks), dim3(kBlock), 0, s,
                           (const double *)x, (double *)F, (double *)G, n, st);
    return hipGetLastError();
}

}  // namespace qed
