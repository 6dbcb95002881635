// Device-side building blocks of the QED event generator (gfx950).
//
// Counter-based random numbers, the quantum parameter chi, the sub-step bounds of
// Sec. 3.1.1, the Boris pusher and the synchrotron-function fits of Sec. 3.2.1.
// Everything is templated on the working real type R (float for the mixed path,
// double for the FP64 path); quantities that decide the sub-step count are always
// formed in double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qed {

constexpr double kAlpha = 7.2973525693e-3;  // fine-structure constant (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt3 = 1.7320508075688772935;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Round: with (hi, lo) the halves of the
// 32x32->64 products M0*c0 and M1*c2, the counter becomes
// (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key advances by the Weyl constants.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// (2k+1) 2^-24 with k the top 23 bits: exact in float, strictly inside (0, 1).
__device__ __forceinline__ float u24(uint32_t w) { return (float)(((w >> 9) << 1) | 1u) * 0x1p-24f; }

// (2k+1) 2^-53 with k the top 52 bits of (hi:lo): exact in double, inside (0, 1).
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
    const uint64_t k = ((((uint64_t)hi) << 32) | lo) >> 12;
    return (double)((k << 1) | 1u) * 0x1p-53;
}

// Id of a child: Philox under the seed key tagged with (0x5851F42D, 0x4C957F2D),
// counter (parent, step, 2 i + slot); slot 0 = photon or pair electron, 1 = positron.
__device__ __forceinline__ uint64_t child_id(uint64_t seed, uint64_t parent, uint32_t step,
                                             uint32_t sub, uint32_t slot) {
    const u32x4 w = philox10((uint32_t)parent, (uint32_t)(parent >> 32), step, 2u * sub + slot,
                             (uint32_t)seed ^ 0x5851F42Du, (uint32_t)(seed >> 32) ^ 0x4C957F2Du);
    return (((uint64_t)w.y) << 32) | w.x;
}

// ---------------------------------------------------------------------------
// chi = sqrt((energy E + p x B)^2 - (p . E)^2) (eq. (1) and eq. (2) text), in double.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double chi_def(double en, double px, double py, double pz, double ex,
                                          double ey, double ez, double bx, double by, double bz) {
    const double ax = en * ex + (py * bz - pz * by);
    const double ay = en * ey + (pz * bx - px * bz);
    const double az = en * ez + (px * by - py * bx);
    const double pe = px * ex + py * ey + pz * ez;
    const double s = ax * ax + ay * ay + az * az - pe * pe;
    return s > 0.0 ? sqrt(s) : 0.0;
}

// Lepton chi in float for the sub-step loop.  With gamma^2 = 1 + |u|^2 the
// definition rearranges to |E|^2 + |u x E|^2 + 2 gamma E.(u x B) + |u x B|^2
// (Lagrange's identity), which has no cancellation in a pure E field.  Only the
// cross term can cancel (crossed fields with u along E x B); then the value is
// recomputed in double from the definition, and guard counts it.
template <int FK = 0>
__device__ __forceinline__ float chi_lepton_f32(float ux, float uy, float uz, float gamma, float ex,
                                                float ey, float ez, float bx, float by, float bz,
                                                float e2, uint32_t &guard) {
    // FK = 1 (B = 0): |E|^2 + |u x E|^2;  FK = 2 (E = 0): |u x B|^2
    if constexpr (FK == 1) {
        const float cex = uy * ez - uz * ey, cey = uz * ex - ux * ez, cez = ux * ey - uy * ex;
        const float s = e2 + (cex * cex + cey * cey + cez * cez);
        return s > 0.0f ? __builtin_amdgcn_sqrtf(s) : 0.0f;
    }
    if constexpr (FK == 2) {
        const float cbx = uy * bz - uz * by, cby = uz * bx - ux * bz, cbz = ux * by - uy * bx;
        const float s = cbx * cbx + cby * cby + cbz * cbz;
        return s > 0.0f ? __builtin_amdgcn_sqrtf(s) : 0.0f;
    }
    const float cex = uy * ez - uz * ey, cey = uz * ex - ux * ez, cez = ux * ey - uy * ex;
    const float cbx = uy * bz - uz * by, cby = uz * bx - ux * bz, cbz = ux * by - uy * bx;
    const float t = e2 + (cex * cex + cey * cey + cez * cez) + (cbx * cbx + cby * cby + cbz * cbz);
    const float xt = 2.0f * gamma * (ex * cbx + ey * cby + ez * cbz);
    if (xt < -0.5f * t) {
        ++guard;
        const double gd = sqrt(1.0 + (double)ux * ux + (double)uy * uy + (double)uz * uz);
        return (float)chi_def(gd, ux, uy, uz, ex, ey, ez, bx, by, bz);
    }
    const float s = t + xt;
    return s > 0.0f ? __builtin_amdgcn_sqrtf(s) : 0.0f;
}

// ---------------------------------------------------------------------------
// ln b for finite b > 0 in double as hi + lo parts of e ln2 + ln m: b = m 2^e
// with m in [sqrt(1/2), sqrt(2)) from the exponent, ln m = 2 atanh(s) =
// 2 (s + s^3/3 + ... + s^23/23), s = (m - 1)/(m + 1), |s| < 0.172 (truncation
// below 1e-20); ln 2 split so that e ln2_hi is exact.
// ---------------------------------------------------------------------------
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;

struct Ln {
    double hi, e;  // ln b = hi + e ln2_lo
};

__device__ __forceinline__ Ln ln_pos(double b) {
    int e;
    double m = frexp(b, &e);  // b = m 2^e, m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double t = 1.0 / 23.0;
    t = fma(t, s2, 1.0 / 21.0);
    t = fma(t, s2, 1.0 / 19.0);
    t = fma(t, s2, 1.0 / 17.0);
    t = fma(t, s2, 1.0 / 15.0);
    t = fma(t, s2, 1.0 / 13.0);
    t = fma(t, s2, 1.0 / 11.0);
    t = fma(t, s2, 1.0 / 9.0);
    t = fma(t, s2, 1.0 / 7.0);
    t = fma(t, s2, 1.0 / 5.0);
    t = fma(t, s2, 1.0 / 3.0);
    const double lnm = 2.0 * s + 2.0 * s * s2 * t;
    const double ed = (double)e;
    return {fma(ed, kLn2Hi, lnm), ed};
}

// -ln u for u in (0, 1] (an exponentially distributed optical depth from a uniform).
__device__ __forceinline__ double neg_ln(double u) {
    const Ln l = ln_pos(u);
    return -(l.hi + l.e * kLn2Lo);
}

// ---------------------------------------------------------------------------
// b^p for finite b > 0 in double, relative error below 4e-15 for |p ln b| < 30
// (the rounding of y = p ln b dominates): ln b as above, then e^y = 2^k e^r with
// |r| <= ln(2)/2 and the Taylor series to r^14.  (One code path and about 60
// double operations, against a few hundred for the general pow, which also
// handles every special case.)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_pos(double b, double p) {
    constexpr double kLog2e = 1.44269504088896338700;
    const Ln l = ln_pos(b);
    // y = p ln b = p (e ln2 + ln m), kept as hi + lo
    const double yh = p * l.hi;
    const double yl = p * l.e * kLn2Lo;
    const double y = yh + yl;
    const double k = rint(y * kLog2e);
    double r = fma(-k, kLn2Hi, yh);
    r = fma(-k, kLn2Lo, r) + yl;
    double q = 1.0 / 87178291200.0;           // 1/14!
    q = fma(q, r, 1.0 / 6227020800.0);
    q = fma(q, r, 1.0 / 479001600.0);
    q = fma(q, r, 1.0 / 39916800.0);
    q = fma(q, r, 1.0 / 3628800.0);
    q = fma(q, r, 1.0 / 362880.0);
    q = fma(q, r, 1.0 / 40320.0);
    q = fma(q, r, 1.0 / 5040.0);
    q = fma(q, r, 1.0 / 720.0);
    q = fma(q, r, 1.0 / 120.0);
    q = fma(q, r, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    return ldexp(q, (int)k);
}

// ---------------------------------------------------------------------------
// Sub-step bounds (Sec. 3.1.1).  Emission: b = 3 chi/2, c = sqrt(3) alpha dt/(pi gamma),
// f(b) in four pieces; each printed breakpoint belongs to the piece above it.
// Pairs: f = coef c b with the photon energy in place of gamma.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bound_emission(double chi, double gamma, double dt) {
    const double b = 1.5 * chi;
    const double c = kSqrt3 * kAlpha * dt / (kPi * gamma);
    double coef, p;
    if (b < 0.1) {
        coef = 0.56;
        p = 1.0;
    } else if (b < 0.5) {
        coef = 0.45;
        p = 11.0 / 12.0;
    } else if (b < 10.0) {
        coef = 0.42;
        p = 19.0 / 24.0;
    } else {
        coef = 0.55;
        p = 2.0 / 3.0;
    }
    const double bp = p == 1.0 ? b : pow_pos(b, p);
    return coef * kPi * c * bp + 0.1 * c * b;
}

__device__ __forceinline__ double bound_pair(double chi, double eps, double dt, double coef) {
    return coef * (kSqrt3 * kAlpha * dt / (kPi * eps)) * (1.5 * chi);
}

// Smallest N >= 1 with f/N <= p_max, capped at cap (sets *capped).
__device__ __forceinline__ uint32_t nsub(double f, double p_max, uint32_t cap, bool *capped) {
    double r = ceil(f / p_max);
    if (!(r >= 1.0)) r = 1.0;
    *capped = r > (double)cap;
    if (*capped) r = (double)cap;
    return (uint32_t)r;
}

// Float reciprocal, square root and reciprocal square root from the hardware
// instructions (about 1 ulp); the double versions keep IEEE accuracy.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp(double v) { return 1.0 / v; }
__device__ __forceinline__ float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double sqrt_(double v) { return sqrt(v); }
__device__ __forceinline__ float rsqrt_(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_(double v) { return 1.0 / sqrt(v); }

// ---------------------------------------------------------------------------
// Boris pusher, du/dt = q (E + u x B / gamma), frozen fields.  hq = q dt / 2 and
// hex, hey, hez = hq E are precomputed per particle.
// ---------------------------------------------------------------------------
// FK selects a specialisation that gives the same result as the general form for
// the field it is used with: 0 general, 1 pure electric field (B = 0: the rotation
// is the identity and u <- (u + hE) + hE), 2 pure magnetic field (E = 0: the
// half kicks vanish exactly; see also Rot below).
template <class R>
__device__ __forceinline__ R inv_gamma(R ux, R uy, R uz, R &u2) {
    u2 = ux * ux + uy * uy + uz * uz;
    return rsqrt_(R(1) + u2);
}

template <class R, int FK = 0>
__device__ __forceinline__ void boris(R &ux, R &uy, R &uz, R hex, R hey, R hez, R hq, R bx, R by,
                                      R bz) {
    if constexpr (FK == 1) {
        ux = (ux + hex) + hex;
        uy = (uy + hey) + hey;
        uz = (uz + hez) + hez;
        return;
    }
    const R mx = FK == 2 ? ux : ux + hex, my = FK == 2 ? uy : uy + hey, mz = FK == 2 ? uz : uz + hez;
    const R ig = rsqrt_(R(1) + mx * mx + my * my + mz * mz);
    const R f = hq * ig;
    const R tx = f * bx, ty = f * by, tz = f * bz;
    const R s = R(2) * rcp(R(1) + tx * tx + ty * ty + tz * tz);
    const R px = mx + (my * tz - mz * ty);
    const R py = my + (mz * tx - mx * tz);
    const R pz = mz + (mx * ty - my * tx);
    const R sx = s * tx, sy = s * ty, sz = s * tz;
    if constexpr (FK == 2) {
        ux = mx + (py * sz - pz * sy);
        uy = my + (pz * sx - px * sz);
        uz = mz + (px * sy - py * sx);
    } else {
        ux = mx + (py * sz - pz * sy) + hex;
        uy = my + (pz * sx - px * sz) + hey;
        uz = mz + (px * sy - py * sx) + hez;
    }
}

// Pure magnetic field: the Boris rotation is exact, so |u|, hence gamma, the
// rotation vectors t = hq B / gamma and s = 2 t / (1 + t^2) and the move per
// sub-step u st / gamma keep their values from one sub-step to the next, and so do
// u . B and therefore chi = |u x B| (and the optical-depth rate, a function of chi
// and gamma).  They are set from u where gamma changes: at the start and after each
// emission's recoil (rot_of here; chi and rw by the lepton loops, which own the
// chi and rate code).
template <class R>
struct Rot {
    R ig, g, tx, ty, tz, sx, sy, sz, vs;
    R chi, rw;  // chi; rate of the optical depth per unit step, chi q(chi) / gamma (its path only)
};

template <class R>
__device__ __forceinline__ Rot<R> rot_of(R ux, R uy, R uz, R hq, R bx, R by, R bz, R str) {
    Rot<R> r;
    R u2;
    r.ig = inv_gamma(ux, uy, uz, u2);
    r.g = (R(1) + u2) * r.ig;
    const R f = hq * r.ig;
    r.tx = f * bx;
    r.ty = f * by;
    r.tz = f * bz;
    const R s = R(2) * rcp(R(1) + r.tx * r.tx + r.ty * r.ty + r.tz * r.tz);
    r.sx = s * r.tx;
    r.sy = s * r.ty;
    r.sz = s * r.tz;
    r.vs = str * r.ig;
    r.chi = R(0);
    r.rw = R(0);
    return r;
}

// The rotation of a Boris step in a pure magnetic field with the vectors of r.
template <class R>
__device__ __forceinline__ void rotate(R &ux, R &uy, R &uz, const Rot<R> &r) {
    const R px = ux + (uy * r.tz - uz * r.ty);
    const R py = uy + (uz * r.tx - ux * r.tz);
    const R pz = uz + (ux * r.ty - uy * r.tx);
    const R mx = ux, my = uy, mz = uz;
    ux = mx + (py * r.sz - pz * r.sy);
    uy = my + (pz * r.sx - px * r.sz);
    uz = mz + (px * r.sy - py * r.sx);
}

// m sub-steps of the held rotation at once: u <- R^m u and d <- d + vs sum_{j=1..m} R^j u,
// the result of m calls of rotate() with their moves, in closed form.  R turns u about
// n = t / |t| by theta, cos theta = (1 - t^2) / (1 + t^2), sin theta = 2 |t| / (1 + t^2): on the
// plane normal to n it multiplies u_perp + i w (w = u_perp x n) by z = e^{i theta}.  z^m = 1 + e
// comes from binary powering in that form ((1 + a)(1 + b) = 1 + a + b + ab), in double from the
// float t, so the turn m theta carries only the rounding of t itself (as m calls of rotate() do);
// then R^m u = u + Re(e) u_perp + Im(e) w and sum_{j=1..m} z^j = z e / (z - 1) with
// 1 / (z - 1) = -(1 + i / |t|) / 2 exactly.
__device__ __forceinline__ void rotate_many(float &ux, float &uy, float &uz, float &dx, float &dy, float &dz,
                                            const Rot<float> &r, uint32_t m) {
    const double tx = r.tx, ty = r.ty, tz = r.tz;
    const double t2 = tx * tx + ty * ty + tz * tz;
    const float fm = (float)m;
    if (!(t2 > 1e-60)) {   // no measurable turn: a straight line
        dx += fm * (ux * r.vs);
        dy += fm * (uy * r.vs);
        dz += fm * (uz * r.vs);
        return;
    }
    const double tn = sqrt(t2), it = 1.0 / tn;
    // z - 1 = h (-t^2 + i |t|), h = 2 / (1 + t^2)
    const double h = 2.0 / (1.0 + t2);
    const double cr = -t2 * h, ci = tn * h;
    double er = 0.0, ei = 0.0, br = cr, bi = ci;
    for (uint32_t q = m;;) {
        if (q & 1u) {
            const double nr = er + br + (er * br - ei * bi);
            const double ni = ei + bi + (er * bi + ei * br);
            er = nr;
            ei = ni;
        }
        q >>= 1;
        if (q == 0u) break;
        const double nr = br * (br + 2.0) - bi * bi;
        const double ni = 2.0 * bi * (br + 1.0);
        br = nr;
        bi = ni;
    }
    // z e, then times -(1 + i / |t|) / 2
    const double zr = 1.0 + cr, zi = ci;
    const double ar = zr * er - zi * ei, ai = zr * ei + zi * er;
    const float sr = (float)(-0.5 * (ar - ai * it)), si = (float)(-0.5 * (ai + ar * it));
    const float fer = (float)er, fei = (float)ei;
    const float fit = (float)it;
    const float nx = r.tx * fit, ny = r.ty * fit, nz = r.tz * fit;
    const float up = ux * nx + uy * ny + uz * nz;
    const float px = ux - up * nx, py = uy - up * ny, pz = uz - up * nz;
    const float wx = py * nz - pz * ny, wy = pz * nx - px * nz, wz = px * ny - py * nx;
    const float ms = fm * up;
    dx += r.vs * (ms * nx + sr * px + si * wx);
    dy += r.vs * (ms * ny + sr * py + si * wy);
    dz += r.vs * (ms * nz + sr * pz + si * wz);
    ux += fer * px + fei * wx;
    uy += fer * py + fei * wy;
    uz += fer * pz + fei * wz;
}

}  // namespace qed
