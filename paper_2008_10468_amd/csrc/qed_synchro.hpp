// Synchrotron functions F(x) = x int_x^inf K_{5/3} and G(x) = x K_{2/3} (Sec. 3.2.1)
// from the piecewise fits of synchro_coeffs.inc:
//   F(x) = t e^{-x} H_F(t),  G(x) = t e^{-x} H_G(t),  t = x^(1/3),
// with H_F, H_G analytic in t and tabulated as one polynomial per uniform segment
// of t.  F and G share t, e^{-x} and the segment index; the segment's
// coefficients are gathered from LDS with 128-bit loads (float: 2 loads per
// function, double: 6).  The tables live in constant memory and are staged into
// LDS once per block by syn_stage().
#pragma once

#include <hip/hip_runtime.h>

#define QED_SYN_STORAGE static __constant__ const
#include "synchro_coeffs.inc"
#undef QED_SYN_STORAGE

namespace qed {

template <class R>
struct SynTable;

template <>
struct SynTable<float> {
    static constexpr int kSeg = QED_SYN_F32_NSEG;
    static constexpr int kCoef = QED_SYN_F32_NCOEF;   // 8
    static constexpr float kTmax = (float)QED_SYN_F32_TMAX;
    static constexpr float kInvHalfWidth = 4.0f;       // 1 / (W/2), W = 0.5
    static constexpr int kWords = kSeg * 2 * kCoef;    // floats
    float4 v[kWords / 4];
};

template <>
struct SynTable<double> {
    static constexpr int kSeg = QED_SYN_F64_NSEG;
    static constexpr int kCoef = QED_SYN_F64_NCOEF;   // 12
    static constexpr double kTmax = QED_SYN_F64_TMAX;
    static constexpr double kInvHalfWidth = 8.0;       // 1 / (W/2), W = 0.25
    static constexpr int kWords = kSeg * 2 * kCoef;    // doubles
    double2 v[kWords / 2];
};

static_assert(QED_SYN_F32_NCOEF == 8, "float kernel assumes 8 coefficients");
static_assert(QED_SYN_F64_NCOEF == 12, "double kernel assumes 12 coefficients");

// Copy the constant table into the block's LDS copy.  All threads of the block
// must call it before any uses the table.
__device__ __forceinline__ void syn_stage(SynTable<float> &t) {
    const float4 *src = reinterpret_cast<const float4 *>(&qed_syn_f32_coef[0][0][0]);
    for (int i = threadIdx.x; i < SynTable<float>::kWords / 4; i += blockDim.x) t.v[i] = src[i];
    __syncthreads();
}

__device__ __forceinline__ void syn_stage(SynTable<double> &t) {
    const double2 *src = reinterpret_cast<const double2 *>(&qed_syn_f64_coef[0][0][0]);
    for (int i = threadIdx.x; i < SynTable<double>::kWords / 2; i += blockDim.x) t.v[i] = src[i];
    __syncthreads();
}

// Float z^(1/3) for 0 <= z <= 2^100: 2^(log2(z)/3) from the hardware log2 / exp2
// (relative error about 1e-6), then one Newton step t <- (2 t + z / t^2) / 3,
// which squares the error.  Inputs below 2^-90 are scaled by 2^90 (and the root
// by 2^-30) so that the hardware log2 never sees a denormal.  z = 0 gives 0.
__device__ __forceinline__ float syn_cbrt(float z) {
    const bool tiny = z < 0x1p-90f;
    const float zs = tiny ? z * 0x1p+90f : z;
    float t = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(zs) * (1.0f / 3.0f));
    const float r = __builtin_amdgcn_rcpf(t * t);
    t = t > 0.0f ? fmaf(t, 2.0f / 3.0f, zs * r * (1.0f / 3.0f)) : 0.0f;
    return tiny ? t * 0x1p-30f : t;
}
// Double z^(1/3) for z >= 0: z = m 2^(3q) with m in [0.5, 4) (from the exponent),
// then Newton's iteration for y = m^(-1/3), y <- y (4 - m y^3) / 3 (no division;
// the error squares each time), from the float seed 2^(-log2(m)/3) (about 1e-6):
// two steps leave about 1e-23, and m^(1/3) = m y^2 rounds to a few ulps.
// z = 0 gives 0, z = +inf gives +inf.
__device__ __forceinline__ double syn_cbrt(double z) {
    if (!(z > 0.0)) return 0.0;
    if (!(z <= 1.0e300)) return z;
    int e;
    const double m0 = frexp(z, &e);            // z = m0 2^e, m0 in [0.5, 1)
    const int q = (e + 3072) / 3 - 1024;       // floor(e / 3)
    const double m = ldexp(m0, e - 3 * q);     // in [0.5, 4)
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)m) * (-1.0f / 3.0f));
    y = y * fma(-m * y, y * y, 4.0) * (1.0 / 3.0);
    y = y * fma(-m * y, y * y, 4.0) * (1.0 / 3.0);
    return ldexp(m * y * y, q);
}

// Float e^{-z} for z >= 0: z = n ln2 + r with ln2 split in a 16-bit high part
// (n ln2_hi exact) and a low part, |r| <= ln2/2, e^{-r} = 2^(-r log2 e) from the
// hardware exp2 (the product's rounding is now tiny), scaled by 2^-n.  The
// argument is capped at 110 (e^-110 underflows to 0 in float).
__device__ __forceinline__ float syn_expm(float z) {
    const float zc = fminf(z, 110.0f);
    const float n = rintf(zc * 1.44269504088896341f);
    float r = fmaf(-n, 0.693145751953125f, zc);
    r = fmaf(-n, 1.42860682030941723e-6f, r);
    return ldexpf(__builtin_amdgcn_exp2f(-r * 1.44269504088896341f), -(int)n);
}
// Double e^{-z} for z >= 0: z = k ln2 + r (Cody-Waite: ln2 in a high part with
// trailing zeros, so k ln2_hi is exact, and a low part), |r| <= ln2/2, e^{-r} by
// its Taylor series to degree 13 (truncation below 1e-17), scaled by 2^-k.  Arguments
// above 746 give 0 (below the smallest double).
__device__ __forceinline__ double syn_expm(double z) {
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    constexpr double kLog2e = 1.44269504088896338700;
    const double zc = fmin(z, 746.0);
    const double k = rint(zc * kLog2e);
    double r = fma(-k, kLn2Hi, zc);
    r = -fma(-k, kLn2Lo, r);                   // e^{-z} = 2^-k e^{r}, r = -(z - k ln2)
    double p = 1.0 / 6227020800.0;             // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, -(int)k);
}

// F, G at z >= 0 (z = +inf gives 0).  Caller guarantees z is not NaN / negative.
__device__ __forceinline__ void syn_eval(float z, const SynTable<float> &tab, float &F, float &G) {
    const float t = syn_cbrt(fminf(z, 0x1p100f));
    const float tc = fminf(t, SynTable<float>::kTmax);
    const int seg = min((int)(tc * 2.0f), SynTable<float>::kSeg - 1);
    const float s = fmaf(tc, SynTable<float>::kInvHalfWidth, -(float)(2 * seg + 1));
    const float4 *c = &tab.v[seg * 4];
    const float4 f0 = c[0], f1 = c[1], g0 = c[2], g1 = c[3];
    float hf = f1.w, hg = g1.w;
    hf = fmaf(hf, s, f1.z);
    hg = fmaf(hg, s, g1.z);
    hf = fmaf(hf, s, f1.y);
    hg = fmaf(hg, s, g1.y);
    hf = fmaf(hf, s, f1.x);
    hg = fmaf(hg, s, g1.x);
    hf = fmaf(hf, s, f0.w);
    hg = fmaf(hg, s, g0.w);
    hf = fmaf(hf, s, f0.z);
    hg = fmaf(hg, s, g0.z);
    hf = fmaf(hf, s, f0.y);
    hg = fmaf(hg, s, g0.y);
    hf = fmaf(hf, s, f0.x);
    hg = fmaf(hg, s, g0.x);
    const float pre = tc * syn_expm(z);
    F = pre * hf;
    G = pre * hg;
}

__device__ __forceinline__ void syn_eval(double z, const SynTable<double> &tab, double &F, double &G) {
    const double t = syn_cbrt(z);
    const double tc = fmin(t, SynTable<double>::kTmax);
    const int seg = min((int)(tc * 4.0), SynTable<double>::kSeg - 1);
    const double s = fma(tc, SynTable<double>::kInvHalfWidth, -(double)(2 * seg + 1));
    const double2 *c = &tab.v[seg * 12];
    double hf = c[5].y, hg = c[11].y;
#pragma unroll
    for (int k = 10; k >= 0; --k) {
        const double2 cf = c[k >> 1], cg = c[6 + (k >> 1)];
        hf = fma(hf, s, (k & 1) ? cf.y : cf.x);
        hg = fma(hg, s, (k & 1) ? cg.y : cg.x);
    }
    const double pre = tc * syn_expm(z);
    F = pre * hf;
    G = pre * hg;
}

}  // namespace qed
