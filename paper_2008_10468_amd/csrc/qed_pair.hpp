// Total pair-creation rate and the rejection envelope of the energy split, for the
// photon optical-depth path.  Integrating eq. (2) over the electron's energy
// fraction gives the probability that a photon of energy eps decays in a time s as
// alpha s (chi / eps) T(chi); T(chi) e^{8/(3 chi)} is tabulated by pair_coeffs.inc
// as one polynomial per unit segment of log2 chi up to chi = 2^24 (max relative
// error 8.5e-8 in float).
#pragma once

#include <hip/hip_runtime.h>

#define QED_PAIR_STORAGE static __constant__ const
#include "pair_coeffs.inc"
#undef QED_PAIR_STORAGE

namespace qed {

struct PairTable {
    static constexpr int kSeg = QED_PAIR_NSEG;
    static constexpr int kL0 = QED_PAIR_L0;
    float4 c[kSeg][2];   // 7 coefficients, padded to 8
    float env[kSeg];
};

static_assert(QED_PAIR_NCOEF == 7, "pair-rate kernel assumes 7 coefficients");

// Copy the tables into the block's LDS copy (every thread calls; ends with a barrier).
__device__ __forceinline__ void pair_stage(PairTable &t) {
    for (int i = threadIdx.x; i < PairTable::kSeg * 8; i += blockDim.x) {
        const int sg = i >> 3, k = i & 7;
        reinterpret_cast<float *>(&t.c[sg][0])[k] = k < 7 ? qed_pair_coef[sg][k] : 0.0f;
    }
    for (int i = threadIdx.x; i < PairTable::kSeg; i += blockDim.x) t.env[i] = qed_pair_env[i];
    __syncthreads();
}

// T(chi) (0 for chi <= 0; the float result underflows to 0 below chi ~ 0.03, where
// no photon decays in any step).  Above the table T e^{8/(3 chi)} falls like chi^(-1/3).
__device__ __forceinline__ float pair_t(float chi, const PairTable &t) {
    if (!(chi > 0.0f)) return 0.0f;
    constexpr float lo = (float)PairTable::kL0, hi = (float)(PairTable::kL0 + PairTable::kSeg);
    float l = __builtin_amdgcn_logf(fmaxf(chi, 0x1p-126f));
    float scale = 1.0f;
    if (l >= hi) {
        scale = __builtin_amdgcn_exp2f((hi - l) * (1.0f / 3.0f));
        l = hi;
    }
    l = fmaxf(l, lo);
    const int sg = min((int)(l - lo), PairTable::kSeg - 1);
    const float s = fmaf(2.0f, l - lo - (float)sg, -1.0f);
    const float4 a = t.c[sg][0], b = t.c[sg][1];
    float q = b.z;
    q = fmaf(q, s, b.y);
    q = fmaf(q, s, b.x);
    q = fmaf(q, s, a.w);
    q = fmaf(q, s, a.z);
    q = fmaf(q, s, a.y);
    q = fmaf(q, s, a.x);
    // e^{-8/(3 chi)} in double: the exponent reaches about 90 before the float result
    // underflows, where a float exponent would cost 1e-5 of relative accuracy
    return q * scale * (float)exp(-8.0 / (3.0 * (double)chi));
}

// Upper bound over d of the Baier-Katkov density D(d) = (3/2) chi (G(z) - d (1-d) F(z)),
// z = 2/(3 chi d (1-d)), at this chi.
__device__ __forceinline__ float pair_envelope(float chi, const PairTable &t) {
    constexpr float lo = (float)PairTable::kL0;
    const float l = __builtin_amdgcn_logf(fmaxf(chi, 0x1p-126f));
    const int sg = max(0, min((int)(l - lo), PairTable::kSeg - 1));
    return t.env[sg] * __builtin_amdgcn_sqrtf(chi * (1.0f + chi)) *
           __builtin_amdgcn_exp2f(-3.8471867f * __builtin_amdgcn_rcpf(chi));
}

}  // namespace qed
