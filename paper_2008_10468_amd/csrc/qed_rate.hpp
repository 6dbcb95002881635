// Total photon-emission rate and the rejection envelope of eq. (1), for the
// surrogate event path.  Integrating eq. (1) over the candidate x in [0, 1]
// gives the emission probability of a sub-step of length s as
// alpha s chi q(chi) / gamma; q is tabulated by rate_coeffs.inc as one polynomial
// per unit segment of log2 chi (max relative error 1.1e-7 in float).
#pragma once

#include <hip/hip_runtime.h>

#define QED_RATE_STORAGE static __constant__ const
#include "rate_coeffs.inc"
#undef QED_RATE_STORAGE

namespace qed {

struct RateTable {
    static constexpr int kSeg = QED_RATE_NSEG;
    static constexpr int kL0 = QED_RATE_L0;
    float4 c[kSeg][2];   // 7 coefficients, padded to 8
    float env[kSeg];
};

static_assert(QED_RATE_NCOEF == 7, "rate kernel assumes 7 coefficients");

// Copy the tables into the block's LDS copy (every thread calls; ends with a barrier).
__device__ __forceinline__ void rate_stage(RateTable &t) {
    for (int i = threadIdx.x; i < RateTable::kSeg * 8; i += blockDim.x) {
        const int sg = i >> 3, k = i & 7;
        reinterpret_cast<float *>(&t.c[sg][0])[k] = k < 7 ? qed_rate_coef[sg][k] : 0.0f;
    }
    for (int i = threadIdx.x; i < RateTable::kSeg; i += blockDim.x) t.env[i] = qed_rate_env[i];
    __syncthreads();
}

// chi q(chi) for chi >= 0 (0 gives 0).  Below 2^L0, q is constant to float
// precision; above the table, q falls like chi^(-1/3) (its large-chi law).
__device__ __forceinline__ float rate_chi_q(float chi, const RateTable &t) {
    if (!(chi > 0.0f)) return 0.0f;
    constexpr float lo = (float)RateTable::kL0, hi = (float)(RateTable::kL0 + RateTable::kSeg);
    float l = __builtin_amdgcn_logf(fmaxf(chi, 0x1p-126f));
    float scale = 1.0f;
    if (l >= hi) {
        scale = __builtin_amdgcn_exp2f((hi - l) * (1.0f / 3.0f));
        l = hi;
    }
    l = fmaxf(l, lo);
    const int sg = min((int)(l - lo), RateTable::kSeg - 1);
    const float s = fmaf(2.0f, l - lo - (float)sg, -1.0f);
    const float4 a = t.c[sg][0], b = t.c[sg][1];
    float q = b.z;
    q = fmaf(q, s, b.y);
    q = fmaf(q, s, b.x);
    q = fmaf(q, s, a.w);
    q = fmaf(q, s, a.z);
    q = fmaf(q, s, a.y);
    q = fmaf(q, s, a.x);
    return chi * q * scale;
}

// Upper bound of ((1 - x^3) F(z) + x^6 G(z)) / x over x in (0, 1) at this chi
// (the emission density of eq. (1) divided by c b): env_j b^(-1/3) on the table,
// a constant above it.
__device__ __forceinline__ float rate_envelope(float chi, const RateTable &t) {
    constexpr float lo = (float)RateTable::kL0, hi = (float)(RateTable::kL0 + RateTable::kSeg);
    const float l = __builtin_amdgcn_logf(fmaxf(chi, 0x1p-126f));
    if (l >= hi) return QED_RATE_ENV_TOP;
    const int sg = max(0, min((int)(l - lo), RateTable::kSeg - 1));
    // b^(-1/3) = 2^(-log2(1.5 chi) / 3)
    const float bm13 = __builtin_amdgcn_exp2f(-(l + 0.58496250072f) * (1.0f / 3.0f));
    return t.env[sg] * bm13;
}

}  // namespace qed
