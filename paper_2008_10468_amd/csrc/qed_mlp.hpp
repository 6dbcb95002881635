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
// of column r.  Each lane's 8 (or 4) K-elements are K indices kidx(g, j); any
// fixed assignment works as long as A and B use the same one.
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

// K index of element j of lane group g in a 32-wide K chunk.
__device__ __forceinline__ int kidx(int g, int j) { return 8 * g + j; }

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf2f(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

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
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16);
}
// the bfloat16 residual v - bf16(v)
__device__ __forceinline__ float bf_res(float v) { return v - bf2f(f2bf(v)); }
__device__ __forceinline__ uint32_t pack2_lo(float a, float b) { return pack2(bf_res(a), bf_res(b)); }

// Network in LDS, laid out for the matrix cores: wf2[n][kk][lane] holds the 8
// B-operand elements W2[16 n + r][32 kk + kidx(g, j)] of lane (r, g), so each
// K chunk of each output tile is one 16-byte load per lane.
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

// Build the fragment layout from float parameters (one block; every thread calls).
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
        const float *W = p + (layer ? kOffW3 : kOffW2);
        const float *row = W + (16 * n + r) * kHid + 32 * kk;
        uint4 v, l;
        v.x = pack2(row[kidx(g, 0)], row[kidx(g, 1)]);
        v.y = pack2(row[kidx(g, 2)], row[kidx(g, 3)]);
        v.z = pack2(row[kidx(g, 4)], row[kidx(g, 5)]);
        v.w = pack2(row[kidx(g, 6)], row[kidx(g, 7)]);
        l.x = pack2_lo(row[kidx(g, 0)], row[kidx(g, 1)]);
        l.y = pack2_lo(row[kidx(g, 2)], row[kidx(g, 3)]);
        l.z = pack2_lo(row[kidx(g, 4)], row[kidx(g, 5)]);
        l.w = pack2_lo(row[kidx(g, 6)], row[kidx(g, 7)]);
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

// Per-wave scratch of the batched evaluation.
struct alignas(16) MlpWave {
    float in_s[16], in_v[16], y[16];
    uint16_t h[16][72];   // one layer's activations, bf16 high parts, rows padded to 144 bytes
    uint16_t l[16][72];   // and their bf16 residuals
};

// A-operand fragments (high and low parts) of row r, K chunks 0 and 1.
struct AFrag {
    bf16x8 h0, h1, l0, l1;
};

template <class Wv>
__device__ __forceinline__ AFrag load_a(const Wv &W, int r, int g) {
    AFrag a;
    a.h0 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][kidx(g, 0)]));
    a.h1 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][32 + kidx(g, 0)]));
    a.l0 = as_bf8(*reinterpret_cast<const uint4 *>(&W.l[r][kidx(g, 0)]));
    a.l1 = as_bf8(*reinterpret_cast<const uint4 *>(&W.l[r][32 + kidx(g, 0)]));
    return a;
}

// Store one value of a C-layout tile as high part and residual.
template <class Wv>
__device__ __forceinline__ void store_split(Wv &W, int row, int col, float v) {
    const uint16_t hb = f2bf(v);
    W.h[row][col] = hb;
    W.l[row][col] = f2bf(v - bf2f(hb));
}

// [16 x 64] x [64 x 64] product of split activations with split weight fragments
// (hi and lo): hi*hi + hi*lo + lo*hi, small terms first.
__device__ __forceinline__ void gemm_split(const AFrag &a, const uint4 (*fh)[2][64], const uint4 (*fl)[2][64],
                                           int lane, f32x4 *acc) {
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const bf16x8 b0 = as_bf8(fh[n][0][lane]), b1 = as_bf8(fh[n][1][lane]);
        const bf16x8 c0 = as_bf8(fl[n][0][lane]), c1 = as_bf8(fl[n][1][lane]);
        f32x4 c = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l0, b0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l1, b1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h0, c0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h1, c1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h0, b0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h1, b1, c, 0, 0, 0);
        acc[n] = c;
    }
}

// y for every lane with act set.  Called by the whole wave in uniform control
// flow (all 64 lanes active); lanes without act get 0.  The active lanes are
// taken 16 at a time as the rows of one matrix-core pass; each row's result is
// independent of the other rows.
__device__ __forceinline__ float mlp_infer_wave(const MlpLds &M, MlpWave &W, bool act, float s, float v) {
    const int lane = __lane_id(), r = lane & 15, g = lane >> 4;
    float out = 0.0f;
    uint64_t m = __ballot(act);
    while (m) {
        const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        const bool mine = ((m >> lane) & 1ull) && rank < 16;
        __syncwarp();
        if (lane < 16) {
            W.in_s[lane] = 0.0f;
            W.in_v[lane] = 0.0f;
        }
        __syncwarp();
        if (mine) {
            W.in_s[rank] = s;
            W.in_v[rank] = v;
        }
        __syncwarp();
        // layer 1, directly in the A layout of layer 2
        const float si = W.in_s[r], vi = W.in_v[r];
        uint32_t ph[2][4], pl[2][4];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
                const int u0 = 32 * kk + kidx(g, j), u1 = u0 + 1;
                const float h0 = mlp_act(fmaf(M.w1[u0][0], si, fmaf(M.w1[u0][1], vi, M.b1[u0])));
                const float h1 = mlp_act(fmaf(M.w1[u1][0], si, fmaf(M.w1[u1][1], vi, M.b1[u1])));
                ph[kk][j / 2] = pack2(h0, h1);
                pl[kk][j / 2] = pack2_lo(h0, h1);
            }
        AFrag a;
        a.h0 = as_bf8(make_uint4(ph[0][0], ph[0][1], ph[0][2], ph[0][3]));
        a.h1 = as_bf8(make_uint4(ph[1][0], ph[1][1], ph[1][2], ph[1][3]));
        a.l0 = as_bf8(make_uint4(pl[0][0], pl[0][1], pl[0][2], pl[0][3]));
        a.l1 = as_bf8(make_uint4(pl[1][0], pl[1][1], pl[1][2], pl[1][3]));
        // layer 2
        f32x4 acc[4];
        gemm_split(a, M.wf2, M.wl2, lane, acc);
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) store_split(W, 4 * g + q, 16 * n + r, mlp_act(acc[n][q] + M.b2[16 * n + r]));
        __syncwarp();
        a = load_a(W, r, g);
        // layer 3 and the output layer
        gemm_split(a, M.wf3, M.wl3, lane, acc);
        float part[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float sacc = 0.0f;
#pragma unroll
            for (int n = 0; n < 4; ++n) sacc = fmaf(M.w4[16 * n + r], mlp_act(acc[n][q] + M.b3[16 * n + r]), sacc);
            part[q] = sacc;
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) part[q] += __shfl_xor(part[q], o);
        if (r == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) W.y[4 * g + q] = part[q] + M.b4;
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

// x = y (b / (1 + b))^(1/3), b = 3 chi / 2, clamped to the open interval (0, 1).
__device__ __forceinline__ float mlp_x_of_y(float y, float chi) {
    const float b = 1.5f * chi;
    const float xs = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(b / (1.0f + b)) * (1.0f / 3.0f));
    return fminf(fmaxf(y * xs, 0x1p-24f), 1.0f - 0x1p-24f);
}

}  // namespace qed
