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

// Deposition.  Particles stored in cell order (as PIC codes keep them) put neighbouring
// lanes into the same node cell.  Relative to its node cell a particle's contribution
// to current component c falls on 12 lattice points: three along the axis on which
// the component's lattice is shifted by half a cell (offsets -1, 0, +1) and two along
// each other axis (0, +1).  The wave sums those 12 values over each run of lanes in
// the same node cell with a segmented scan, and the run's last lane adds the 12 sums
// with the hardware's double atomic add, so same-address atomics do not serialise.
// A wave with more than kMaxRuns runs (particles in random order, or sparser than
// about two per cell) adds each particle's 8 corners directly.
constexpr int kMaxRuns = 32;

template <class R>
__global__ __launch_bounds__(kGridBlock) void k_deposit(GridDev g, DepositArgs a) {
    const u64 n0 = *a.n;
    const u64 n = n0 < a.cap ? n0 : a.cap;
    const double scale = a.charge * g.idx * g.idy * g.idz;   // q / cell volume
    const uint32_t lane = __lane_id();
    const uint32_t dims[3] = {g.nx, g.ny, g.nz};
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
        // node cell and the fractions within it (lanes without a particle sit at the
        // origin with zero current)
        const double s3[3] = {(x - g.x0) * g.idx, (y - g.y0) * g.idy, (z - g.z0) * g.idz};
        uint32_t nd[3];
        double ph[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double f = floor(s3[d]);
            nd[d] = wrap_index(f, dims[d]);
            ph[d] = s3[d] - f;
        }
        const uint32_t node = (nd[2] * g.ny + nd[1]) * g.nx + nd[0];
        const uint32_t prev = __shfl_up(node, 1);
        const u64 starts = __ballot(lane == 0 || prev != node);
        if (__popcll(starts) > kMaxRuns) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!(has && cur[c] != 0.0)) continue;
                const Corners cr = corners(g, x, y, z, kStagger[c][0], kStagger[c][1], kStagger[c][2]);
#pragma unroll
                for (int q = 0; q < 8; ++q) unsafeAtomicAdd(&a.j[c][cr.idx[q]], cr.w[q] * cur[c]);
            }
            continue;
        }
        // run of this lane (1-based count of run starts up to it) and scan masks
        const uint32_t rid = (uint32_t)__popcll(starts & ((2ull << lane) - 1ull));
        bool same[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const uint32_t o = 1u << t;
            const uint32_t r = __shfl_up(rid, o);   // every lane takes part in the shuffle
            same[t] = lane >= o && r == rid;
        }
        const bool last = lane == 63 || (((starts >> lane) >> 1) & 1ull);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // weights along each axis: the shifted axis c over offsets -1, 0, +1
            double wa[3][3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double f = ph[d];
                if (d == c) {
                    const bool up = f >= 0.5;
                    wa[d][0] = up ? 0.0 : 0.5 - f;
                    wa[d][1] = up ? 1.5 - f : f + 0.5;
                    wa[d][2] = up ? f - 0.5 : 0.0;
                } else {
                    wa[d][0] = 1.0 - f;
                    wa[d][1] = f;
                    wa[d][2] = 0.0;
                }
            }
            // the 12 values: shifted axis slot a (0..2), the other two axes slots b, e
            const int d1 = c == 0 ? 1 : 0, d2 = c == 2 ? 1 : 2;
            double v[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) v[q] = cur[c] * wa[c][q / 4] * wa[d1][(q / 2) & 1] * wa[d2][q & 1];
#pragma unroll
            for (int t = 0; t < 6; ++t) {
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const double o = __shfl_up(v[q], 1u << t);
                    if (same[t]) v[q] += o;
                }
            }
            if (last) {
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    if (v[q] == 0.0) continue;
                    int off[3];
                    off[c] = q / 4 - 1;
                    off[d1] = (q / 2) & 1;
                    off[d2] = q & 1;
                    uint32_t id[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const int ii = (int)nd[d] + off[d];
                        id[d] = ii < 0 ? (uint32_t)(ii + (int)dims[d]) : ((uint32_t)ii >= dims[d] ? (uint32_t)ii - dims[d] : (uint32_t)ii);
                    }
                    unsafeAtomicAdd(&a.j[c][(id[2] * g.ny + id[1]) * g.nx + id[0]], v[q]);
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
