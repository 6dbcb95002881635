// Training of the optical-depth paths' networks on the GPU: the inverse CDF of the
// emitted energy (target 0) and of the pair's energy split (target 1, the
// half-distribution of |d - 1/2|), same network shape and kernels.
//
//   k_cdf_table    the normalised CDF of the emitted energy, eq. (1) integrated over
//                  the candidate x (or of the split, eq. (2) integrated over d), on a
//                  grid of chi (double, from the double fits of the synchrotron
//                  functions);
//   k_mlp_data     training samples (chi, u) -> x = CDF_chi^{-1}(u) from the table;
//   k_mlp_train    forward and backward passes on the matrix cores, gradients
//                  reduced per block;
//   k_mlp_reduce   sum of the block gradients and the Adam update (or only the sum,
//                  for gradient checks);
//   k_mlp_pack     float parameters -> the fragment layout the generator stages;
//   k_mlp_validate per chi bin, the largest CDF error |CDF_chi(x(chi, u)) - u| of
//                  the packed network over a grid of u;
//   k_mlp_infer    the packed network on given (chi, u) pairs.
#include "qed_device.hpp"
#include "qed_internal.hpp"
#include "qed_mlp.hpp"
#include "qed_synchro.hpp"

namespace qed {

namespace {

constexpr int kBlock = 256;

// Grid of the CDF table: x = 1 - (1 - xi)^2 with xi uniform, so points crowd
// towards x = 1, where the spectrum of large chi has its structure (1 - x ~ 1/b).
__device__ __forceinline__ double cdf_x_of_xi(double xi) { return 1.0 - (1.0 - xi) * (1.0 - xi); }
__device__ __forceinline__ double cdf_xi_of_x(double x) { return 1.0 - sqrt(fmax(1.0 - x, 0.0)); }

// ((1 - x^3) F(z) + x^6 G(z)) / x with z = x^3 / (b (1 - x^3)): eq. (1) over c b.
// x = 0 gives the limit 2^(2/3) Gamma(2/3) b^(-1/3).
__device__ __forceinline__ double emission_density(double x, double b, const SynTable<double> &tab) {
    if (x <= 0.0) return 2.1495282415344787 * cbrt(1.0 / b);
    const double x3 = x * x * x;
    const double omx3 = (1.0 - x) * (1.0 + x + x * x);
    if (omx3 <= 0.0) return 0.0;
    double F, G;
    syn_eval(x3 / (b * omx3), tab, F, G);
    return (omx3 * F + x3 * x3 * G) / x;
}

// Energy split of pair creation: the Baier-Katkov density (3/2) chi (G(z) - d(1-d) F(z)),
// z = 2/(3 chi d (1-d)), of the electron's fraction d (eq. (2) over its prefactor).
__device__ __forceinline__ double pair_density(double d, double chi, const SynTable<double> &tab) {
    const double dd = d * (1.0 - d);
    if (dd <= 0.0) return 0.0;
    double F, G;
    syn_eval(2.0 / (3.0 * chi * dd), tab, F, G);
    return 1.5 * chi * (G - dd * F);
}

// Density of the table's variable per unit of xi = k / nx at xi (kind 0: x(xi) with
// the grid's Jacobian; kind 1: D = xi / 2 of the half-distribution, d = 1/2 + D).
__device__ __forceinline__ double table_density(int kind, double xi, double l10, const SynTable<double> &tab) {
    if (kind == 0) return emission_density(cdf_x_of_xi(xi), 1.5 * exp10(l10), tab) * 2.0 * (1.0 - xi);
    return 0.5 * pair_density(0.5 + 0.5 * xi, exp10(l10), tab);
}

__global__ __launch_bounds__(kBlock) void k_cdf_table(CdfTableDev t) {
    __shared__ SynTable<double> tab;
    __shared__ double wsum[kBlock / 64];
    syn_stage(tab);
    const int c = blockIdx.x;
    const double l10 = t.lo10 + (t.hi10 - t.lo10) * (double)c / (double)(t.nchi - 1);
    const int per = t.nx / kBlock;  // intervals per thread
    const double h = 1.0 / (double)t.nx;
    const int k0 = threadIdx.x * per;
    double part = 0.0;
    double dprev = table_density(t.kind, k0 * h, l10, tab);
    for (int k = k0; k < k0 + per; ++k) {
        const double xi = (k + 1) * h;
        const double d = table_density(t.kind, xi, l10, tab);
        part += 0.5 * h * (dprev + d);
        dprev = d;
    }
    // block exclusive prefix of the thread sums
    double incl = part;
    const int lane = __lane_id(), wv = threadIdx.x / 64;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    double off = incl - part, total = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wv) off += wsum[w];
        total += wsum[w];
    }
    double *row = t.cdf + (u64)c * (t.nx + 1);
    if (threadIdx.x == 0) {
        row[0] = 0.0;
        t.total[c] = total;
    }
    // second pass: the running sum (same order of additions as above)
    double acc = off;
    dprev = table_density(t.kind, k0 * h, l10, tab);
    for (int k = k0; k < k0 + per; ++k) {
        const double xi = (k + 1) * h;
        const double d = table_density(t.kind, xi, l10, tab);
        acc += 0.5 * h * (dprev + d);
        dprev = d;
        row[k + 1] = k + 1 == t.nx ? 1.0 : fmin(acc / total, 1.0);
    }
}

// Table CDF at (log10 chi, x), linear in xi and in log10 chi between nodes (x: the
// candidate for kind 0, the distance D from 1/2 for kind 1).
__device__ __forceinline__ double cdf_lookup(const CdfTableDev &t, double l10, double x) {
    const double cpos = (l10 - t.lo10) / (t.hi10 - t.lo10) * (double)(t.nchi - 1);
    const int j = min(max((int)floor(cpos), 0), t.nchi - 2);
    const double w = fmin(fmax(cpos - j, 0.0), 1.0);
    const double xi = (t.kind == 0 ? cdf_xi_of_x(fmin(fmax(x, 0.0), 1.0)) : fmin(fmax(2.0 * x, 0.0), 1.0)) *
                      (double)t.nx;
    const int k = min((int)xi, t.nx - 1);
    const double f = xi - k;
    const double *r0 = t.cdf + (u64)j * (t.nx + 1), *r1 = r0 + (t.nx + 1);
    const double c0 = r0[k] + f * (r0[k + 1] - r0[k]);
    const double c1 = r1[k] + f * (r1[k + 1] - r1[k]);
    return c0 + w * (c1 - c0);
}

// Inverse of cdf_lookup at (log10 chi, u): x and the density dCDF/dx there.
__device__ __forceinline__ void cdf_invert(const CdfTableDev &t, double l10, double u, double &x,
                                           double &dens) {
    const double cpos = (l10 - t.lo10) / (t.hi10 - t.lo10) * (double)(t.nchi - 1);
    const int j = min(max((int)floor(cpos), 0), t.nchi - 2);
    const double w = fmin(fmax(cpos - j, 0.0), 1.0);
    const double *r0 = t.cdf + (u64)j * (t.nx + 1), *r1 = r0 + (t.nx + 1);
    int lo = 0, hi = t.nx;  // invariant: M(lo) <= u < M(hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const double m = r0[mid] + w * (r1[mid] - r0[mid]);
        if (m <= u)
            lo = mid;
        else
            hi = mid;
    }
    const double m0 = r0[lo] + w * (r1[lo] - r0[lo]);
    const double m1 = r0[hi] + w * (r1[hi] - r0[hi]);
    const double dm = m1 - m0;
    const double f = dm > 0.0 ? (u - m0) / dm : 0.5;
    const double xi = ((double)lo + f) / (double)t.nx;
    if (t.kind == 0) {
        x = cdf_x_of_xi(xi);
        dens = dm * (double)t.nx / fmax(2.0 * (1.0 - xi), 1e-300);
    } else {
        x = 0.5 * xi;
        dens = dm * (double)t.nx * 2.0;
    }
}

// Largest network input v: u = 1 - 2^-24, the largest float uniform, gives 1.55
// (emission) and 3.08 (pairs, v = sqrt(-ln(1 - u')) - 1).
constexpr double kVmax = 1.6;
constexpr double kVmaxPair = 3.1;

__global__ __launch_bounds__(kBlock) void k_mlp_data(CdfTableDev t, Sample *out, u64 n, uint64_t seed,
                                                     uint32_t step, double lo10, double hi10) {
    const uint32_t klo = (uint32_t)seed ^ 0x7F4A7C15u, khi = (uint32_t)(seed >> 32) ^ 0xF39CC060u;
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < n; i += (u64)gridDim.x * kBlock) {
        const u32x4 w = philox10((uint32_t)i, (uint32_t)(i >> 32), step, 0u, klo, khi);
        const double tl = u53(w.x, w.y);  // position in the chi range
        // the network input v = (-ln(1 - u))^(1/3) - 1 is drawn uniformly on
        // [-1, kVmax] (u = 1 - exp(-(v + 1)^3)), so the tails of the spectrum are
        // sampled as densely as its bulk
        const double vmax = t.kind == 0 ? kVmax : kVmaxPair;
        const double v = -1.0 + (vmax + 1.0) * u53(w.z, w.w);
        const double u = t.kind == 0 ? -expm1(-(v + 1.0) * (v + 1.0) * (v + 1.0)) : -expm1(-(v + 1.0) * (v + 1.0));
        const double l10 = lo10 + (hi10 - lo10) * tl;
        double x, dens;
        cdf_invert(t, l10, u, x, dens);
        // output scale: (b / (1 + b))^(1/3) of x (emission), the split's width (pairs)
        const double xs = t.kind == 0 ? cbrt(1.5 * exp10(l10) / (1.0 + 1.5 * exp10(l10)))
                                      : (double)pair_width((float)exp10(l10));
        Sample s;
        s.s = (float)(2.0 * tl - 1.0);
        s.v = (float)v;
        s.y = (float)(x / xs);
        // weight: squared density in units of the network output, so the loss
        // approximates the squared CDF error (capped to keep the scale moderate,
        // with a small floor for the far tail)
        const double dy = fmin(dens * xs, 5.0);
        s.w = (float)(dy * dy + 1e-4);
        out[i] = s;
    }
}

// ---------------------------------------------------------------------------
// Training step: forward and backward passes of 16-sample tiles per wave.
// ---------------------------------------------------------------------------
struct alignas(16) TrainWave {
    float s[16], v[16], yt[16], wt[16];
    uint16_t h[16][72];   // high parts (and single bf16 values of the backward pass)
    uint16_t l[16][72];   // residuals of the forward activations
};

struct TrainParams {
    float w1[kHid][2];
    float b1[kHid], b2[kHid], b3[kHid], w4[kHid];
    float b4;
};

// Training layout (activations as the A operand, weights as B): tf2[n][kk][lane]
// holds W2[16 n + r][32 kk + kidx(g, j)] (high parts; tl2 the residuals), and
// wt2 the transposed weights W2[32 kk + kidx(g, j)][16 n + r] for dZ W.
struct TrainLds {
    TrainParams P;
    uint4 tf2[4][2][64], tf3[4][2][64];
    uint4 tl2[4][2][64], tl3[4][2][64];
    uint4 wt2[4][2][64], wt3[4][2][64];
    TrainWave ws[kBlock / 64];
    float red[kMlpParams + 1];
};

__device__ __forceinline__ void pack_train(const float *__restrict__ p, TrainLds &L) {
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        L.P.w1[i][0] = p[kOffW1 + 2 * i];
        L.P.w1[i][1] = p[kOffW1 + 2 * i + 1];
        L.P.b1[i] = p[kOffB1 + i];
        L.P.b2[i] = p[kOffB2 + i];
        L.P.b3[i] = p[kOffB3 + i];
        L.P.w4[i] = p[kOffW4 + i];
    }
    if (threadIdx.x == 0) L.P.b4 = p[kOffB4];
    for (int e = threadIdx.x; e < 2 * 4 * 2 * 64; e += blockDim.x) {
        const int lane = e & 63, kk = (e >> 6) & 1, n = (e >> 7) & 3, layer = e >> 9;
        const int r = lane & 15, g = lane >> 4;
        const float *W = p + (layer ? kOffW3 : kOffW2);
        float f[8], t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            f[j] = W[(16 * n + r) * kHid + 32 * kk + kidx(g, j)];
            t[j] = W[(32 * kk + kidx(g, j)) * kHid + 16 * n + r];
        }
        (layer ? L.tf3 : L.tf2)[n][kk][lane] =
            make_uint4(pack2(f[0], f[1]), pack2(f[2], f[3]), pack2(f[4], f[5]), pack2(f[6], f[7]));
        (layer ? L.tl3 : L.tl2)[n][kk][lane] =
            make_uint4(pack2_lo(f[0], f[1]), pack2_lo(f[2], f[3]), pack2_lo(f[4], f[5]), pack2_lo(f[6], f[7]));
        (layer ? L.wt3 : L.wt2)[n][kk][lane] =
            make_uint4(pack2(t[0], t[1]), pack2(t[2], t[3]), pack2(t[4], t[5]), pack2(t[6], t[7]));
    }
}

// A-operand fragments (high and low parts) of row r, K chunks 0 and 1.
struct AFrag {
    bf16x8 h0, h1, l0, l1;
};

// [16 x 64] x [64 x 64] product of split activations (A) with split weights (B):
// hi*hi + hi*lo + lo*hi, small terms first.
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

typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ s16x4 pack4(const float *v) {
    const uint2 u = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
    return __builtin_bit_cast(s16x4, u);
}

// C-layout activations (rows 4g + q of column 16 n + r) -> split A-layout fragments.
__device__ __forceinline__ AFrag transpose_split(TrainWave &W, const float (*v)[4], int r, int g) {
    __syncwarp();
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const __bf16 hb = (__bf16)v[n][q];
            W.h[4 * g + q][16 * n + r] = __builtin_bit_cast(uint16_t, hb);
            W.l[4 * g + q][16 * n + r] = bf_bits(v[n][q] - (float)hb);
        }
    __syncwarp();
    AFrag a;
    a.h0 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][kidx(g, 0)]));
    a.h1 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][32 + kidx(g, 0)]));
    a.l0 = as_bf8(*reinterpret_cast<const uint4 *>(&W.l[r][kidx(g, 0)]));
    a.l1 = as_bf8(*reinterpret_cast<const uint4 *>(&W.l[r][32 + kidx(g, 0)]));
    __syncwarp();
    return a;
}

// C-layout tile values -> single bf16 A-layout fragments via LDS (backward pass).
__device__ __forceinline__ void transpose_to_a(TrainWave &W, const float (*v)[4], int r, int g, bf16x8 &a0,
                                               bf16x8 &a1) {
    __syncwarp();
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) W.h[4 * g + q][16 * n + r] = bf_bits(v[n][q]);
    __syncwarp();
    a0 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][kidx(g, 0)]));
    a1 = as_bf8(*reinterpret_cast<const uint4 *>(&W.h[r][32 + kidx(g, 0)]));
    __syncwarp();
}

__device__ __forceinline__ void gemm_64(bf16x8 a0, bf16x8 a1, const uint4 (*frag)[2][64], int lane,
                                        f32x4 *acc) {
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        acc[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, as_bf8(frag[n][0][lane]), acc[n], 0, 0, 0);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, as_bf8(frag[n][1][lane]), acc[n], 0, 0, 0);
    }
}

__global__ __launch_bounds__(kBlock) void k_mlp_train(TrainArgs ta) {
    __shared__ TrainLds L;
    for (int i = threadIdx.x; i <= kMlpParams; i += kBlock) L.red[i] = 0.0f;
    pack_train(ta.params, L);
    __syncthreads();
    const TrainParams &M = L.P;
    const int lane = __lane_id(), r = lane & 15, g = lane >> 4, wv = threadIdx.x / 64;
    TrainWave &W = L.ws[wv];
    f32x4 gw2[16], gw3[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gw2[k] = gw3[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float gw1[4][2] = {}, gb1[4] = {}, gb2[4] = {}, gb3[4] = {}, gw4[4] = {};
    float gb4 = 0.0f, loss = 0.0f;
    const u64 base = ((u64)blockIdx.x * (kBlock / 64) + wv) * (u64)ta.tiles * 16;
    for (uint32_t tile = 0; tile < ta.tiles; ++tile) {
        const u64 row0 = base + 16ull * tile;
        __syncwarp();
        if (lane < 16) {
            const Sample sm = ta.batch[row0 + lane];
            W.s[lane] = sm.s;
            W.v[lane] = sm.v;
            W.yt[lane] = sm.y;
            W.wt[lane] = sm.w;
        }
        __syncwarp();
        float sq[4], vq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sq[q] = W.s[4 * g + q];
            vq[q] = W.v[4 * g + q];
        }
        // layer 1 (C layout)
        float pre1[4][4], h1[4][4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int u = 16 * n + r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                pre1[n][q] = fmaf(M.w1[u][0], sq[q], fmaf(M.w1[u][1], vq[q], M.b1[u]));
                h1[n][q] = mlp_act(pre1[n][q]);
            }
        }
        bf16x8 a0, a1;
        f32x4 acc[4];
        gemm_split(transpose_split(W, h1, r, g), L.tf2, L.tl2, lane, acc);
        float pre2[4][4], h2[4][4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                pre2[n][q] = acc[n][q] + M.b2[16 * n + r];
                h2[n][q] = mlp_act(pre2[n][q]);
            }
        gemm_split(transpose_split(W, h2, r, g), L.tf3, L.tl3, lane, acc);
        float pre3[4][4], h3[4][4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                pre3[n][q] = acc[n][q] + M.b3[16 * n + r];
                h3[n][q] = mlp_act(pre3[n][q]);
            }
        float y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float sacc = 0.0f;
#pragma unroll
            for (int n = 0; n < 4; ++n) sacc = fmaf(M.w4[16 * n + r], h3[n][q], sacc);
            y[q] = sacc;
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) y[q] += __shfl_xor(y[q], o);
        // loss and output gradient
        float dy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float e = y[q] + M.b4 - W.yt[4 * g + q];
            const float wq = W.wt[4 * g + q];
            dy[q] = 2.0f * wq * e * ta.inv_batch;
            if (r == 0) {
                loss = fmaf(wq * e * e, ta.inv_batch, loss);
                gb4 += dy[q];
            }
        }
        float dz[4][4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const float w4 = M.w4[16 * n + r];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gw4[n] = fmaf(dy[q], h3[n][q], gw4[n]);
                dz[n][q] = dy[q] * w4 * mlp_dact(pre3[n][q]);
                gb3[n] += dz[n][q];
            }
        }
        // dW3 += dz3^T h2 (K = the 16 samples of the tile)
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) {
            const s16x4 ad = pack4(dz[ci]);
#pragma unroll
            for (int cj = 0; cj < 4; ++cj)
                gw3[ci * 4 + cj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ad, pack4(h2[cj]), gw3[ci * 4 + cj], 0, 0, 0);
        }
        // dh2 = dz3 W3
        transpose_to_a(W, dz, r, g, a0, a1);
        gemm_64(a0, a1, L.wt3, lane, acc);
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                dz[n][q] = acc[n][q] * mlp_dact(pre2[n][q]);
                gb2[n] += dz[n][q];
            }
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) {
            const s16x4 ad = pack4(dz[ci]);
#pragma unroll
            for (int cj = 0; cj < 4; ++cj)
                gw2[ci * 4 + cj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ad, pack4(h1[cj]), gw2[ci * 4 + cj], 0, 0, 0);
        }
        // dh1 = dz2 W2
        transpose_to_a(W, dz, r, g, a0, a1);
        gemm_64(a0, a1, L.wt2, lane, acc);
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float d1 = acc[n][q] * mlp_dact(pre1[n][q]);
                gw1[n][0] = fmaf(d1, sq[q], gw1[n][0]);
                gw1[n][1] = fmaf(d1, vq[q], gw1[n][1]);
                gb1[n] += d1;
            }
    }
    // per-column sums over the four lane groups, then the block reduction
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            gw1[n][0] += __shfl_xor(gw1[n][0], o);
            gw1[n][1] += __shfl_xor(gw1[n][1], o);
            gb1[n] += __shfl_xor(gb1[n], o);
            gb2[n] += __shfl_xor(gb2[n], o);
            gb3[n] += __shfl_xor(gb3[n], o);
            gw4[n] += __shfl_xor(gw4[n], o);
        }
    }
    // The block's sum: the four waves add their partial sums in a fixed order (one
    // wave at a time, its lanes writing distinct entries), so the float sums, and
    // with them a training run, are the same on every run.
    float *red = L.red;
    gb4 = wave_sum_f(gb4);
    loss = wave_sum_f(loss);
    for (int turn = 0; turn < kBlock / 64; ++turn) {
        __syncthreads();
        if ((int)(threadIdx.x / 64) != turn) continue;
        if (g == 0) {
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int u = 16 * n + r;
                red[kOffW1 + 2 * u] += gw1[n][0];
                red[kOffW1 + 2 * u + 1] += gw1[n][1];
                red[kOffB1 + u] += gb1[n];
                red[kOffB2 + u] += gb2[n];
                red[kOffB3 + u] += gb3[n];
                red[kOffW4 + u] += gw4[n];
            }
        }
        if (lane == 0) {
            red[kOffB4] += gb4;
            red[kMlpParams] += loss;
        }
#pragma unroll
        for (int ci = 0; ci < 4; ++ci)
#pragma unroll
            for (int cj = 0; cj < 4; ++cj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int idx = (16 * ci + 4 * g + q) * kHid + 16 * cj + r;
                    red[kOffW2 + idx] += gw2[ci * 4 + cj][q];
                    red[kOffW3 + idx] += gw3[ci * 4 + cj][q];
                }
    }
    __syncthreads();
    float *dst = ta.partials + (u64)blockIdx.x * (kMlpParams + 1);
    for (int i = threadIdx.x; i <= kMlpParams; i += kBlock) dst[i] = red[i];
}

// Sum of the block gradients; then Adam (grad_out == nullptr) or a plain copy of
// the sum (gradient checks).  One thread per parameter, plus one for the loss.
__global__ __launch_bounds__(kBlock) void k_mlp_reduce(ReduceArgs ra) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p > kMlpParams) return;
    float gsum = 0.0f;
    for (int b = 0; b < ra.blocks; ++b) gsum += ra.partials[(u64)b * (kMlpParams + 1) + p];
    if (p == kMlpParams) {
        if (ra.loss_out) *ra.loss_out = gsum;
        return;
    }
    if (ra.grad_out) {
        ra.grad_out[p] = gsum;
        return;
    }
    const float m = ra.beta1 * ra.m[p] + (1.0f - ra.beta1) * gsum;
    const float v = ra.beta2 * ra.v[p] + (1.0f - ra.beta2) * gsum * gsum;
    ra.m[p] = m;
    ra.v[p] = v;
    ra.params[p] -= ra.lr * (m * ra.c1) / (sqrtf(v * ra.c2) + ra.eps);
}

__global__ __launch_bounds__(kBlock) void k_mlp_pack(const float *params, MlpModel *out) {
    __shared__ MlpLds M;
    mlp_pack(params, M);
    __syncthreads();
    // weights only: lo, inv_span, nbins and the fallback flags are set by the host
    const uint4 *s = reinterpret_cast<const uint4 *>(&M);
    uint4 *d = reinterpret_cast<uint4 *>(out);
    constexpr int kHead = offsetof(MlpLds, b4) / 16;   // whole 16-byte words before b4
    for (int i = threadIdx.x; i < (int)(sizeof(MlpLds) / 16); i += kBlock) {
        if (i < kHead || (i >= (int)(offsetof(MlpLds, wf2) / 16) && i < (int)(offsetof(MlpLds, fallback) / 16)))
            d[i] = s[i];
    }
    if (threadIdx.x == 0) out->b4 = M.b4;
}

// x of the packed network for (chi, u) (kind 1: the electron's fraction d); NaN
// where the model does not sample.
__device__ __forceinline__ float infer_one(const MlpLds &M, MlpWave &W, bool valid, float chi, float u, int kind) {
    bool in_range;
    int bin;
    const float s = mlp_input_s(M, chi, in_range, bin);
    const bool use = valid && in_range && !M.fallback[bin];
    const float v = kind == 0 ? mlp_input_v(u) : mlp_input_v_pair(fabsf(2.0f * u - 1.0f));
    const float y = mlp_infer_wave(M, W, use, s, v);
    if (!use) return __builtin_nanf("");
    return kind == 0 ? mlp_x_of_y(y, chi) : pair_d_of_y(y, chi, u >= 0.5f);
}

__global__ __launch_bounds__(kBlock) void k_mlp_infer(const MlpModel *model, const float *chi, const float *u,
                                                      float *x, u64 n, int kind) {
    __shared__ MlpLds M;
    __shared__ MlpWave ws[kBlock / 64];
    mlp_stage(model, M);
    MlpWave &W = ws[threadIdx.x / 64];
    // wave-uniform trip count: every lane takes part in the matrix-core passes
    for (u64 i0 = (u64)blockIdx.x * kBlock; i0 < n; i0 += (u64)gridDim.x * kBlock) {
        const u64 i = i0 + threadIdx.x;
        const bool valid = i < n;
        const float xi = infer_one(M, W, valid, valid ? chi[i] : 1.0f, valid ? u[i] : 0.5f, kind);
        if (valid) x[i] = xi;
    }
}

// One block per (bin, position in the bin); 1024 values of u per chi.
__global__ __launch_bounds__(kBlock) void k_mlp_validate(const MlpModel *model, CdfTableDev t, int per_bin,
                                                         float *bin_err) {
    __shared__ MlpLds M;
    __shared__ MlpWave ws[kBlock / 64];
    __shared__ float wmax[kBlock / 64];
    mlp_stage(model, M);
    MlpWave &W = ws[threadIdx.x / 64];
    const int bin = blockIdx.x / per_bin, q = blockIdx.x % per_bin;
    const double span = 1.0 / (double)M.inv_span;
    const double l10 = (double)M.lo + span * ((double)bin + (double)q / (double)(per_bin - 1)) / (double)M.nbins;
    const double l10c = fmin(l10, (double)M.lo + span * (1.0 - 1e-7));   // stay inside [lo, hi)
    const float chi = (float)exp10(l10c);
    float emax = 0.0f;
    for (int k = threadIdx.x; k < 1024; k += kBlock) {
        const float u = ((float)k + 0.5f) / 1024.0f;
        bool in_range;
        int b;
        const float s = mlp_input_s(M, chi, in_range, b);
        const float y = mlp_infer_wave(M, W, true, s, t.kind == 0 ? mlp_input_v(u) : mlp_input_v_pair(u));
        // kind 1: u is u' of the half-distribution, the network gives D
        const float x = t.kind == 0 ? mlp_x_of_y(y, chi) : fminf(fmaxf(y * pair_width(chi), 0.0f), 0.5f);
        const double c = cdf_lookup(t, log10((double)chi), (double)x);
        emax = fmaxf(emax, (float)fabs(c - (double)u));
    }
    for (int o = 32; o > 0; o >>= 1) emax = fmaxf(emax, __shfl_xor(emax, o));
    if (__lane_id() == 0) wmax[threadIdx.x / 64] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w) m = fmaxf(m, wmax[w]);
        atomicMax(reinterpret_cast<unsigned int *>(&bin_err[bin]), __float_as_uint(m));
    }
}

}  // namespace

hipError_t launch_cdf_table(const CdfTableDev &t, hipStream_t s) {
    if (t.nx % kBlock != 0 || t.nchi < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cdf_table, dim3(t.nchi), dim3(kBlock), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_mlp_data(const CdfTableDev &t, Sample *out, u64 n, uint64_t seed, uint32_t step,
                           double lo10, double hi10, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_data, dim3(blocks), dim3(kBlock), 0, s, t, out, n, seed, step, lo10, hi10);
    return hipGetLastError();
}

hipError_t launch_mlp_train(const TrainArgs &ta, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train, dim3(blocks), dim3(kBlock), 0, s, ta);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const ReduceArgs &ra, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, ra);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *params, MlpModel *out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(kBlock), 0, s, params, out);
    return hipGetLastError();
}

hipError_t launch_mlp_validate(const MlpModel *model, const CdfTableDev &t, int nbins, int per_bin, float *bin_err,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_validate, dim3(nbins * per_bin), dim3(kBlock), 0, s, model, t, per_bin, bin_err);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpModel *model, const float *chi, const float *u, float *x, u64 n, int blocks,
                            hipStream_t s, int kind) {
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(kBlock), 0, s, model, chi, u, x, n, kind);
    return hipGetLastError();
}

}  // namespace qed
