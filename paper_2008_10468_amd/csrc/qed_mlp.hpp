// Learned inverse CDF of the emitted photon energy (surrogate sampler): a
// 2 -> 64 -> 64 -> 64 -> 1 network evaluated on the matrix cores of gfx950.
//
// Inputs s = 2 (log10 chi - lo) / (hi - lo) - 1 and v = (-ln(1 - u))^(1/3) - 1 (the
// candidate's tail, x^3 ~ b ln(1/(1 - u)) at small chi, becomes linear in v); hidden
// activation a(t) = t / sqrt(1 + t^2) (smooth, bounded, three instructions, with
// derivative (1 + t^2)^(-3/2)); output y, from which x = delta^(1/3) = y (b / (1 +
// b))^(1/3).  Layer 1 and the output layer are float; the two 64 x 64 layers run
// on the matrix cores in bfloat16 with float accumulation
// (v_mfma_f32_16x16x32_bf16), with weights and input activations each held as
// the sum of two bfloat16 numbers (hi + lo) and the product formed as
// hi*hi + hi*lo + lo*hi (three passes), which keeps about 16 significant bits: a
// single bfloat16 rounding would leave errors of about 1e-3 in the output, the
// size of the accuracy the sampler needs.
//
// Matrix-core layouts used here (16 x 16 output tile, wave64): for lane l let
// r = l % 16 and g = l / 16.  The A operand (16 rows x K) supplies row r, the B
// operand (K x 16 columns) column r, and lane l holds the result rows 4g .. 4g+3
// of column r.  Which K indices a lane's 8 (or 4) elements stand for is a free
// choice as long as A and B make the same one: inference uses unit_of (below),
// training kidx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qed {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHid = 64;
constexpr int kMlpParams = 8577;
// offsets in the float parameter vector (W[out][in])
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352, kOffB3 = 8448,
              kOffW4 = 8512, kOffB4 = 8576;

// K index of element j of lane group g in a 32-wide K chunk (training layout).
__device__ __forceinline__ int kidx(int g, int j) { return 8 * g + j; }

// Hidden unit behind element j of lane group g in K chunk kk of the inference
// layout.  A product's result tile leaves lane (r, g) holding units 16 n + 4 g + q
// (n, q = 0..3) of batch row r; taking chunk kk = units of n = 2 kk and 2 kk + 1
// makes that exactly the lane's B-operand fragment for the next layer, so the
// activations never leave the registers between layers.
__device__ __forceinline__ int unit_of(int kk, int g, int j) { return 16 * (2 * kk + (j >> 2)) + 4 * g + (j & 3); }

__device__ __forceinline__ float mlp_act(float t) { return t * __builtin_amdgcn_rsqf(fmaf(t, t, 1.0f)); }
// a'(t) = (1 + t^2)^(-3/2)
__device__ __forceinline__ float mlp_dact(float t) {
    const float r = __builtin_amdgcn_rsqf(fmaf(t, t, 1.0f));
    return r * r * r;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ bf16x4 as_bf4(uint2 v) { return __builtin_bit_cast(bf16x4, v); }
// Two floats to packed bfloat16 (round to nearest even; one v_cvt_pk_bf16_f32).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    const bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint16_t bf_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
// the bfloat16 residual v - bf16(v)
__device__ __forceinline__ float bf_res(float v) { return v - (float)(__bf16)v; }
__device__ __forceinline__ uint32_t pack2_lo(float a, float b) { return pack2(bf_res(a), bf_res(b)); }

// Network in LDS, laid out for the matrix cores with the weights as the A
// operand: wf2[n][kk][lane] holds the 8 elements W2[16 n + r][unit_of(kk, g, j)]
// of lane (r, g) (high parts; wl2 the residuals), one 16-byte load per pass.
struct MlpLds {
    float w1[kHid][2];
    float b1[kHid], b2[kHid], b3[kHid], w4[kHid];
    float b4;
    float lo, inv_span;   // s = (log10 chi - lo) inv_span - 1
    int nbins;
    uint4 wf2[4][2][64];
    uint4 wf3[4][2][64];
    uint4 wl2[4][2][64];   // bf16 residuals of the same weights
    uint4 wl3[4][2][64];
    uint8_t fallback[256];
};

// Device copy of an installed model (same layout; staged into LDS per block).
typedef MlpLds MlpModel;

// Build the inference layout from float parameters (one block; every thread calls).
__device__ __forceinline__ void mlp_pack(const float *__restrict__ p, MlpLds &M) {
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        M.w1[i][0] = p[kOffW1 + 2 * i];
        M.w1[i][1] = p[kOffW1 + 2 * i + 1];
        M.b1[i] = p[kOffB1 + i];
        M.b2[i] = p[kOffB2 + i];
        M.b3[i] = p[kOffB3 + i];
        M.w4[i] = p[kOffW4 + i];
    }
    if (threadIdx.x == 0) M.b4 = p[kOffB4];
    for (int e = threadIdx.x; e < 2 * 4 * 2 * 64; e += blockDim.x) {
        const int lane = e & 63, kk = (e >> 6) & 1, n = (e >> 7) & 3, layer = e >> 9;
        const int r = lane & 15, g = lane >> 4;
        const float *row = p + (layer ? kOffW3 : kOffW2) + (16 * n + r) * kHid;
        float w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) w[j] = row[unit_of(kk, g, j)];
        const uint4 v = make_uint4(pack2(w[0], w[1]), pack2(w[2], w[3]), pack2(w[4], w[5]), pack2(w[6], w[7]));
        const uint4 l = make_uint4(pack2_lo(w[0], w[1]), pack2_lo(w[2], w[3]), pack2_lo(w[4], w[5]),
                                   pack2_lo(w[6], w[7]));
        (layer ? M.wf3 : M.wf2)[n][kk][lane] = v;
        (layer ? M.wl3 : M.wl2)[n][kk][lane] = l;
    }
}

// Copy an installed model into LDS (every thread calls; ends with a barrier).
__device__ __forceinline__ void mlp_stage(const MlpModel *__restrict__ src, MlpLds &M) {
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(&M);
    static_assert(sizeof(MlpLds) % 16 == 0, "MlpLds must be a multiple of 16 bytes");
    for (int i = threadIdx.x; i < (int)(sizeof(MlpLds) / 16); i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

// Per-wave scratch of the batched evaluation: the rows' inputs and outputs (up to
// two 16-row groups per pass).
struct MlpWave {
    float in_s[32], in_v[32], y[32];
};

// Activations of one batch row as B-operand fragments (high parts and residuals).
struct BFrag {
    uint32_t h[2][4], l[2][4];
};

// z = W x for the batch: acc[n][q] = sum_k W[16 n + 4 g + q][k] x[row r][k],
// as hi*hi + hi*lo + lo*hi, small terms first.
__device__ __forceinline__ void mlp_layer(const BFrag &x, const uint4 (*wh)[2][64], const uint4 (*wl)[2][64],
                                          int lane, f32x4 *acc) {
    const bf16x8 xh0 = as_bf8(make_uint4(x.h[0][0], x.h[0][1], x.h[0][2], x.h[0][3]));
    const bf16x8 xh1 = as_bf8(make_uint4(x.h[1][0], x.h[1][1], x.h[1][2], x.h[1][3]));
    const bf16x8 xl0 = as_bf8(make_uint4(x.l[0][0], x.l[0][1], x.l[0][2], x.l[0][3]));
    const bf16x8 xl1 = as_bf8(make_uint4(x.l[1][0], x.l[1][1], x.l[1][2], x.l[1][3]));
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const bf16x8 a0 = as_bf8(wh[n][0][lane]), a1 = as_bf8(wh[n][1][lane]);
        const bf16x8 c0 = as_bf8(wl[n][0][lane]), c1 = as_bf8(wl[n][1][lane]);
        f32x4 c = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xl0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xl1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, xh0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, xh1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xh0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xh1, c, 0, 0, 0);
        acc[n] = c;
    }
}

// The same products for two 16-row groups of one pass: each weight fragment is read
// from LDS once for both (the reads, 16 KB per layer and pass, are what a lone group
// waits on).  Every row goes through the same operations in the same order as in
// mlp_layer, so its result does not depend on the group it is evaluated in.
__device__ __forceinline__ void mlp_layer2(const BFrag &x, const BFrag &x2, const uint4 (*wh)[2][64],
                                           const uint4 (*wl)[2][64], int lane, f32x4 *acc, f32x4 *acc2) {
    const bf16x8 xh0 = as_bf8(make_uint4(x.h[0][0], x.h[0][1], x.h[0][2], x.h[0][3]));
    const bf16x8 xh1 = as_bf8(make_uint4(x.h[1][0], x.h[1][1], x.h[1][2], x.h[1][3]));
    const bf16x8 xl0 = as_bf8(make_uint4(x.l[0][0], x.l[0][1], x.l[0][2], x.l[0][3]));
    const bf16x8 xl1 = as_bf8(make_uint4(x.l[1][0], x.l[1][1], x.l[1][2], x.l[1][3]));
    const bf16x8 yh0 = as_bf8(make_uint4(x2.h[0][0], x2.h[0][1], x2.h[0][2], x2.h[0][3]));
    const bf16x8 yh1 = as_bf8(make_uint4(x2.h[1][0], x2.h[1][1], x2.h[1][2], x2.h[1][3]));
    const bf16x8 yl0 = as_bf8(make_uint4(x2.l[0][0], x2.l[0][1], x2.l[0][2], x2.l[0][3]));
    const bf16x8 yl1 = as_bf8(make_uint4(x2.l[1][0], x2.l[1][1], x2.l[1][2], x2.l[1][3]));
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const bf16x8 a0 = as_bf8(wh[n][0][lane]), a1 = as_bf8(wh[n][1][lane]);
        const bf16x8 c0 = as_bf8(wl[n][0][lane]), c1 = as_bf8(wl[n][1][lane]);
        f32x4 c = f32x4{0.0f, 0.0f, 0.0f, 0.0f}, d = c;
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xl0, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, yl0, d, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xl1, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, yl1, d, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, xh0, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, yh0, d, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, xh1, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, yh1, d, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xh0, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, yh0, d, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xh1, c, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, yh1, d, 0, 0, 0);
        acc[n] = c;
        acc2[n] = d;
    }
}

// a(z + b) of a layer's result, written as the next layer's B fragments.
__device__ __forceinline__ BFrag mlp_activate(const f32x4 *acc, const float *bias, int g) {
    BFrag x;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        float h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = mlp_act(acc[n][q] + bias[16 * n + 4 * g + q]);
        // units 16 n + 4 g + q sit in chunk n / 2, slots 4 (n % 2) + q
        x.h[n >> 1][2 * (n & 1)] = pack2(h[0], h[1]);
        x.h[n >> 1][2 * (n & 1) + 1] = pack2(h[2], h[3]);
        x.l[n >> 1][2 * (n & 1)] = pack2_lo(h[0], h[1]);
        x.l[n >> 1][2 * (n & 1) + 1] = pack2_lo(h[2], h[3]);
    }
    return x;
}

// Layer 1 (float) of batch row (s, v), straight into the B layout of layer 2.
__device__ __forceinline__ BFrag mlp_first(const MlpLds &M, float si, float vi, int g) {
    BFrag x;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
            const int u0 = unit_of(kk, g, j), u1 = unit_of(kk, g, j + 1);
            const float h0 = mlp_act(fmaf(M.w1[u0][0], si, fmaf(M.w1[u0][1], vi, M.b1[u0])));
            const float h1 = mlp_act(fmaf(M.w1[u1][0], si, fmaf(M.w1[u1][1], vi, M.b1[u1])));
            x.h[kk][j / 2] = pack2(h0, h1);
            x.l[kk][j / 2] = pack2_lo(h0, h1);
        }
    return x;
}

// Output layer: the row's value summed over the four lane groups (every lane gets it).
__device__ __forceinline__ float mlp_last(const MlpLds &M, const f32x4 *acc, int g) {
    float part = 0.0f;
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = 16 * n + 4 * g + q;
            part = fmaf(M.w4[u], mlp_act(acc[n][q] + M.b3[u]), part);
        }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + M.b4;
}

// y for every lane with act set.  Called by the whole wave in uniform control
// flow (all 64 lanes active); lanes without act get 0.  The active lanes are
// taken 16 at a time as the columns (batch rows) of one matrix-core pass; with
// DUAL, 32 at a time in two 16-row groups that share their weight reads while
// more than 16 wait (more registers: for kernels that have them to spare).  Each
// row's result is independent of the other rows and of its group.
template <bool DUAL = false>
__device__ __forceinline__ float mlp_infer_wave(const MlpLds &M, MlpWave &W, bool act, float s, float v) {
    const int lane = __lane_id(), r = lane & 15, g = lane >> 4;
    float out = 0.0f;
    uint64_t m = __ballot(act);
    while (m) {
        const bool two = DUAL && __popcll(m) > 16;   // uniform across the wave
        const uint32_t rows = two ? 32u : 16u;
        const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        const bool mine = ((m >> lane) & 1ull) && rank < rows;
        __syncwarp();
        if (lane < 32) {
            W.in_s[lane] = 0.0f;
            W.in_v[lane] = 0.0f;
        }
        __syncwarp();
        if (mine) {
            W.in_s[rank] = s;
            W.in_v[rank] = v;
        }
        __syncwarp();
        f32x4 acc[4];
        BFrag x = mlp_first(M, W.in_s[r], W.in_v[r], g);
        if (two) {
            f32x4 acc2[4];
            BFrag x2 = mlp_first(M, W.in_s[16 + r], W.in_v[16 + r], g);
            mlp_layer2(x, x2, M.wf2, M.wl2, lane, acc, acc2);
            x = mlp_activate(acc, M.b2, g);
            x2 = mlp_activate(acc2, M.b2, g);
            mlp_layer2(x, x2, M.wf3, M.wl3, lane, acc, acc2);
            const float y0 = mlp_last(M, acc, g), y1 = mlp_last(M, acc2, g);
            if (g == 0) {
                W.y[r] = y0;
                W.y[16 + r] = y1;
            }
        } else {
            mlp_layer(x, M.wf2, M.wl2, lane, acc);
            x = mlp_activate(acc, M.b2, g);
            mlp_layer(x, M.wf3, M.wl3, lane, acc);
            const float y0 = mlp_last(M, acc, g);
            if (g == 0) W.y[r] = y0;
        }
        __syncwarp();
        if (mine) out = W.y[rank];
        m &= ~__ballot(mine);
        __syncwarp();
    }
    return out;
}

// Network input s for a chi (float), and whether the model covers it.
__device__ __forceinline__ float mlp_input_s(const MlpLds &M, float chi, bool &in_range, int &bin) {
    const float l10 = __builtin_amdgcn_logf(fmaxf(chi, 0x1p-126f)) * 0.30102999566f;
    const float t = (l10 - M.lo) * M.inv_span;   // in [0, 1) on the model's range
    in_range = t >= 0.0f && t < 1.0f;
    bin = in_range ? min((int)(t * (float)M.nbins), M.nbins - 1) : 0;
    return 2.0f * t - 1.0f;
}

// Network input v of a uniform u in (0, 1): (-ln(1 - u))^(1/3) - 1.
__device__ __forceinline__ float mlp_input_v(float u) {
    const float L = -__builtin_amdgcn_logf(1.0f - u) * 0.69314718056f;   // -ln(1 - u) > 0
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fmaxf(L, 0x1p-100f)) * (1.0f / 3.0f)) - 1.0f;
}

// Pair creation's energy split (the network of the photon path): the electron's
// fraction d = 1/2 +- D, D = y w(chi) with the split's width w(chi) = sqrt(3 chi / 64) /
// sqrt(1 + 3 chi / 16) (the standard deviation of the Gaussian limit at small chi,
// 1/2 at large chi); input v = sqrt(-ln(1 - u')) - 1 of u' = |2u - 1|, the sign of
// d - 1/2 from u < 1/2 (the split is symmetric).
__device__ __forceinline__ float pair_width(float chi) {
    return __builtin_amdgcn_sqrtf(0.046875f * chi) * __builtin_amdgcn_rsqf(1.0f + 0.1875f * chi);
}

__device__ __forceinline__ float mlp_input_v_pair(float up) {
    const float L = -__builtin_amdgcn_logf(1.0f - up) * 0.69314718056f;   // -ln(1 - u') >= 0
    return __builtin_amdgcn_sqrtf(fmaxf(L, 0.0f)) - 1.0f;
}

__device__ __forceinline__ float pair_d_of_y(float y, float chi, bool upper) {
    const float D = fminf(fmaxf(y * pair_width(chi), 0.0f), 0.5f - 0x1p-24f);
    return upper ? 0.5f + D : 0.5f - D;
}

// x = y (b / (1 + b))^(1/3), b = 3 chi / 2, clamped to the open interval (0, 1).
__device__ __forceinline__ float mlp_x_of_y(float y, float chi) {
    const float b = 1.5f * chi;
    const float xs = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(b / (1.0f + b)) * (1.0f / 3.0f));
    return fminf(fmaxf(y * xs, 0x1p-24f), 1.0f - 0x1p-24f);
}

}  // namespace qed
