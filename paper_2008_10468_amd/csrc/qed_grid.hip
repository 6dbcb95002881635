// Grid coupling: the PIC stages around the particle push (Sec. 2.1: stage 2, field
// interpolation from the grid to the particles; stage 4, deposition of the
// particles' currents to the grid), on a periodic Cartesian Yee grid.
//
// Each component lives on its own lattice, shifted by half a cell in some
// directions (Ex and Jx by (1/2, 0, 0), Ey, Jy (0, 1/2, 0), Ez, Jz (0, 0, 1/2),
// Bx (0, 1/2, 1/2), By (1/2, 0, 1/2), Bz (1/2, 1/2, 0)); both stages use linear
// (cloud-in-cell) weights on that lattice, computed in double from the double
// positions.  One lane per particle; the grid arrays are read through the cache
// (neighbouring particles share cells), the currents are added with the hardware's
// double-precision atomic add (ordinary device memory; the default compare-and-swap
// loop of atomicAdd on doubles is several times slower), combined first across the
// lanes of a wave that share a cell.
#include <hip/hip_runtime.h>
#include <math.h>

#include "qed_internal.hpp"

namespace qed {
namespace {

constexpr int kGridBlock = 256;

struct Corners {
    uint32_t idx[8];
    double w[8];
};

// Periodic index in [0, n) of the lattice point at or below f = floor(s), computed in
// double (exact while |f| < 2^53 / n; beyond that only kept in range).  Callers pass
// finite s.
__device__ __forceinline__ uint32_t wrap_index(double f, uint32_t n) {
    double r = f - (double)n * floor(f / (double)n);
    r = r < 0.0 ? 0.0 : (r > (double)(n - 1) ? (double)(n - 1) : r);
    return (uint32_t)r;
}

// A position whose lattice coordinates are finite (the others are skipped).
__device__ __forceinline__ bool on_grid(const GridDev &g, double x, double y, double z) {
    return isfinite((x - g.x0) * g.idx) && isfinite((y - g.y0) * g.idy) && isfinite((z - g.z0) * g.idz);
}

// The 8 lattice points around (x, y, z) on the lattice shifted by (ox, oy, oz) cells,
// with their weights (periodic).  The position must be on_grid.
__device__ __forceinline__ Corners corners(const GridDev &g, double x, double y, double z, double ox, double oy,
                                           double oz) {
    const double sx = (x - g.x0) * g.idx - ox, sy = (y - g.y0) * g.idy - oy, sz = (z - g.z0) * g.idz - oz;
    const double fx0 = floor(sx), fy0 = floor(sy), fz0 = floor(sz);
    const double fx = sx - fx0, fy = sy - fy0, fz = sz - fz0;
    // periodic wrap of the lower corner (positions may lie outside the box)
    const uint32_t i0 = wrap_index(fx0, g.nx), j0 = wrap_index(fy0, g.ny), k0 = wrap_index(fz0, g.nz);
    const uint32_t i1 = i0 + 1 == g.nx ? 0 : i0 + 1, j1 = j0 + 1 == g.ny ? 0 : j0 + 1,
                   k1 = k0 + 1 == g.nz ? 0 : k0 + 1;
    Corners c;
    int q = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx, ++q) {
                const uint32_t i = cx ? i1 : i0, j = cy ? j1 : j0, k = cz ? k1 : k0;
                c.idx[q] = (k * g.ny + j) * g.nx + i;
                c.w[q] = (cx ? fx : 1.0 - fx) * (cy ? fy : 1.0 - fy) * (cz ? fz : 1.0 - fz);
            }
    return c;
}

__device__ __constant__ const double kStagger[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},   // Ex, Ey, Ez (and Jx, Jy, Jz)
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};  // Bx, By, Bz

template <class R>
__global__ __launch_bounds__(kGridBlock) void k_gather(GridDev g, GatherArgs a) {
    const u64 n0 = *a.n;
    const u64 n = n0 < a.cap ? n0 : a.cap;
    for (u64 p = (u64)blockIdx.x * kGridBlock + threadIdx.x; p < n; p += (u64)gridDim.x * kGridBlock) {
        const double x = a.x[p], y = a.y[p], z = a.z[p];
        if (!on_grid(g, x, y, z)) {
#pragma unroll
            for (int c = 0; c < 6; ++c) ((R *)a.out[c])[p] = (R)NAN;
            continue;
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const Corners cr = corners(g, x, y, z, kStagger[c][0], kStagger[c][1], kStagger[c][2]);
            const R *f = (const R *)g.f[c];
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) v += cr.w[q] * (double)f[cr.idx[q]];
            ((R *)a.out[c])[p] = (R)v;
        }
    }
}

// Deposition.  Lanes whose particles share a component's lattice cell (the usual case
// when particles are stored in cell order, as PIC codes keep them) have the same eight
// corners: the wave then sums their contributions per distinct cell with cross-lane
// reductions and one lane adds the eight sums, so same-address atomics do not
// serialise.  A wave whose lanes fall into many different cells (particles in random
// order) adds directly.  The choice is made per wave from the number of changes of the
// particles' node cell between neighbouring lanes (each node cell spans at most two
// cells of a staggered lattice per axis); kMaxRuns is the largest count for which the
// wave combines first.
constexpr int kMaxRuns = 12;

// Node cell (i, j, k) of an on_grid position, flattened, wrapped as corners() wraps.
__device__ __forceinline__ uint32_t node_cell(const GridDev &g, double x, double y, double z) {
    const uint32_t i = wrap_index(floor((x - g.x0) * g.idx), g.nx), j = wrap_index(floor((y - g.y0) * g.idy), g.ny),
                   k = wrap_index(floor((z - g.z0) * g.idz), g.nz);
    return (k * g.ny + j) * g.nx + i;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <class R>
__global__ __launch_bounds__(kGridBlock) void k_deposit(GridDev g, DepositArgs a) {
    const u64 n0 = *a.n;
    const u64 n = n0 < a.cap ? n0 : a.cap;
    const double scale = a.charge * g.idx * g.idy * g.idz;   // q / cell volume
    const uint32_t lane = __lane_id();
    // wave-uniform loop: lane l of the wave takes particle p0 + l
    for (u64 p0 = (u64)blockIdx.x * kGridBlock + (threadIdx.x & ~63u); p0 < n; p0 += (u64)gridDim.x * kGridBlock) {
        const u64 p = p0 + lane;
        const bool has = p < n;
        double cur[3] = {0.0, 0.0, 0.0};
        double x = g.x0, y = g.y0, z = g.z0;
        if (has) {
            const double ux = (double)((const R *)a.ux)[p], uy = (double)((const R *)a.uy)[p],
                         uz = (double)((const R *)a.uz)[p];
            const double w = (double)((const R *)a.w)[p];
            const double gi = 1.0 / sqrt(1.0 + ux * ux + uy * uy + uz * uz);
            const double px = a.x[p], py = a.y[p], pz = a.z[p];
            if (on_grid(g, px, py, pz) && isfinite(w * gi * (ux + uy + uz))) {
                cur[0] = scale * w * ux * gi;
                cur[1] = scale * w * uy * gi;
                cur[2] = scale * w * uz * gi;
                x = px;
                y = py;
                z = pz;
            }
        }
        const uint32_t node = node_cell(g, x, y, z);
        const uint32_t prev_node = __shfl_up(node, 1);
        const bool prev_has = __shfl_up(has ? 1 : 0, 1) != 0;
        const bool combine = __popcll(__ballot(has && (lane == 0 || !prev_has || prev_node != node))) <= kMaxRuns;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool act = has && cur[c] != 0.0;
            const Corners cr = corners(g, x, y, z, kStagger[c][0], kStagger[c][1], kStagger[c][2]);
            const uint32_t key = cr.idx[0];   // the corners follow from the first one
            if (!combine) {
                if (act)
#pragma unroll
                    for (int q = 0; q < 8; ++q) unsafeAtomicAdd(&a.j[c][cr.idx[q]], cr.w[q] * cur[c]);
                continue;
            }
            u64 pending = __ballot(act);
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const uint32_t lk = __shfl(key, leader);
                const bool mine = ((pending >> lane) & 1ull) && key == lk;
                pending &= ~__ballot(mine);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double v = wave_sum_d(mine ? cr.w[q] * cur[c] : 0.0);
                    if ((int)lane == leader) unsafeAtomicAdd(&a.j[c][cr.idx[q]], v);
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_gather(const GridDev &g, const GatherArgs &a, int dtype, int blocks, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_deposit(const GridDev &g, const DepositArgs &a, int dtype, int blocks, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_deposit<float>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    else
        hipLaunchKernelGGL(k_deposit<double>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    return hipGetLastError();
}

}  // namespace qed
