// Grid coupling: the PIC stages around the particle push (Sec. 2.1: stage 2, field
// interpolation from the grid to the particles; stage 4, deposition of the
// particles' currents to the grid), on a periodic Cartesian Yee grid.
//
// Each component lives on its own lattice, shifted by half a cell in some
// directions (Ex and Jx by (1/2, 0, 0), Ey, Jy (0, 1/2, 0), Ez, Jz (0, 0, 1/2),
// Bx (0, 1/2, 1/2), By (1/2, 0, 1/2), Bz (1/2, 1/2, 0)); both stages use linear
// (cloud-in-cell) weights on that lattice, computed in double from the double
// positions.  The gather takes one lane per particle and reads the grid arrays
// through the cache (neighbouring particles share cells).  The deposition sorts the
// particles by tile of cells and sums each tile in LDS, so that every grid point is
// written once whatever the particles' order and density; without its scratch it
// adds with the hardware's double-precision atomic add (ordinary device memory; the
// default compare-and-swap loop of atomicAdd on doubles is several times slower),
// combined first across the lanes of a wave that share a cell.
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

// Node cell of an on-grid position (periodic) and the fractions within it along x, y, z.
__device__ __forceinline__ void node_cell(const GridDev &g, double x, double y, double z, uint32_t nd[3],
                                          double ph[3]) {
    const double s3[3] = {(x - g.x0) * g.idx, (y - g.y0) * g.idy, (z - g.z0) * g.idz};
    const uint32_t dims[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = floor(s3[d]);
        nd[d] = wrap_index(f, dims[d]);
        ph[d] = s3[d] - f;
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
        uint32_t nd[3];
        double ph[3];
        node_cell(g, x, y, z, nd, ph);
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

// ---------------------------------------------------------------------------
// Deposition sorted by tile, for particles in any order and at any density, without
// atomic adds on the grid.  The grid's node cells are grouped into tiles of
// kTileEdge^3 cells; a tile's particles touch the lattice points of its region, node
// offsets -1 .. kTileEdge (6^3 points per current component).  Five kernels:
//   k_dep_bin      tile of every particle; its rank among the tile's particles (each
//                  block counts its particles per tile in LDS and reserves a range of
//                  every tile it touches with one atomic add; beyond kBinLdsTiles
//                  tiles every particle reserves its own place)
//   k_dep_scan     exclusive sums over the tiles of their particles and of their
//                  parts (a part: up to kPart particles of one tile), the tile of each
//                  part; clears the counts for the next call
//   k_dep_scatter  one 64-byte record per particle at its place in tile order: the
//                  three fractions, the three current components, the node within
//                  the tile
//   k_dep_accum    one block per part (every np-th particle of a tile of np parts):
//                  its particles' 24 values each summed over the region in LDS, the
//                  region stored to the part's staging slot
//   k_dep_reduce   one thread per grid point and component: the sum of the staged
//                  regions that cover the point (periodic images included), added to
//                  the current array
// The record holds the same node cell and fractions as the wave-run kernel above
// computes, so both give the same current up to the order of the additions.
// ---------------------------------------------------------------------------
constexpr uint32_t kTileEdge = kDepTileEdge;
constexpr uint32_t kRegionEdge = kTileEdge + 2;
constexpr uint32_t kRegionPts = kRegionEdge * kRegionEdge * kRegionEdge;   // per component
constexpr uint32_t kStage = 3 * kRegionPts;          // doubles per part
constexpr uint32_t kBinItems = 8;                    // particles per thread in k_dep_bin
constexpr uint32_t kPart = kDepPart;
constexpr uint32_t kNoTile = 0xffffffffu;
static_assert(kTileEdge == 4, "the record packs the node within its tile in 2 bits per axis");

// Tile of a node cell and the node's place in it (x + 4 y + 16 z).
__device__ __forceinline__ uint32_t tile_of(const DepSortArgs &a, const uint32_t nd[3], uint32_t &local) {
    local = (nd[0] % kTileEdge) | (nd[1] % kTileEdge) << 2 | (nd[2] % kTileEdge) << 4;
    return ((nd[2] / kTileEdge) * a.tiles[1] + nd[1] / kTileEdge) * a.tiles[0] + nd[0] / kTileEdge;
}

template <bool LDS>
__global__ __launch_bounds__(kGridBlock) void k_dep_bin(GridDev g, DepSortArgs a) {
    __shared__ uint32_t hist[LDS ? kBinLdsTiles : 1], base[LDS ? kBinLdsTiles : 1];
    const u64 n0 = *a.n;
    const u64 n = n0 < a.cap ? n0 : a.cap;
    const u64 p0 = (u64)blockIdx.x * (kGridBlock * kBinItems);
    if (p0 >= n) return;   // whole block
    if (LDS) {
        for (uint32_t i = threadIdx.x; i < a.ntiles; i += kGridBlock) hist[i] = 0;
        __syncthreads();
    }
    uint32_t t[kBinItems], r[kBinItems];
#pragma unroll
    for (uint32_t k = 0; k < kBinItems; ++k) {
        const u64 p = p0 + k * kGridBlock + threadIdx.x;
        t[k] = kNoTile;
        r[k] = 0;
        if (p >= n) continue;
        const double x = a.x[p], y = a.y[p], z = a.z[p];
        if (!on_grid(g, x, y, z)) continue;
        uint32_t nd[3], local;
        double ph[3];
        node_cell(g, x, y, z, nd, ph);
        t[k] = tile_of(a, nd, local);
        r[k] = LDS ? atomicAdd(&hist[t[k]], 1u) : atomicAdd(&a.count[t[k]], 1u);
    }
    if (LDS) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < a.ntiles; i += kGridBlock) {
            const uint32_t c = hist[i];
            if (c) base[i] = atomicAdd(&a.count[i], c);
        }
        __syncthreads();
    }
#pragma unroll
    for (uint32_t k = 0; k < kBinItems; ++k) {
        const u64 p = p0 + k * kGridBlock + threadIdx.x;
        if (p < n) a.pos[p] = t[k] == kNoTile ? kNoTile : (LDS ? base[t[k]] + r[k] : r[k]);
    }
}

// Inclusive sum over a block of kScanBlock threads (16 waves); total: the block's sum.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ uint32_t block_incl(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o);
        if ((int)lane >= o) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (uint32_t w = 0; w < kScanBlock / 64; ++w) {
        before += w < wv ? wsum[w] : 0u;
        total += wsum[w];
    }
    __syncthreads();   // wsum is reused by the next call
    return before + v;
}

// One block; four tiles per thread per round.
__global__ __launch_bounds__(kScanBlock) void k_dep_scan(DepSortArgs a) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    uint32_t carry = 0, pcarry = 0;   // the same in every thread
    for (uint32_t b0 = 0; b0 < a.ntiles; b0 += 4 * kScanBlock) {
        const uint32_t i = b0 + 4 * threadIdx.x;
        uint32_t v[4], pc[4], s = 0, ps = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i + k < a.ntiles ? a.count[i + k] : 0u;
            if (i + k < a.ntiles) a.count[i + k] = 0;   // zero for the next deposit
            pc[k] = (v[k] + kPart - 1) / kPart;
            s += v[k];
            ps += pc[k];
        }
        uint32_t tot, ptot;
        uint32_t e = carry + block_incl(s, wsum, tot) - s;
        uint32_t pe = pcarry + block_incl(ps, wsum, ptot) - ps;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i + k < a.ntiles) {
                a.off[i + k] = e;
                a.part_off[i + k] = pe;
                for (uint32_t q = 0; q < pc[k]; ++q) a.part_tile[pe + q] = i + k;
            }
            e += v[k];
            pe += pc[k];
        }
        carry += tot;
        pcarry += ptot;
    }
    if (threadIdx.x == 0) {
        a.off[a.ntiles] = carry;
        a.part_off[a.ntiles] = pcarry;
    }
}

template <class R>
__global__ __launch_bounds__(kGridBlock) void k_dep_scatter(GridDev g, DepSortArgs a) {
    const u64 n0 = *a.n;
    const u64 n = n0 < a.cap ? n0 : a.cap;
    const double scale = a.charge * g.idx * g.idy * g.idz;
    for (u64 p = (u64)blockIdx.x * kGridBlock + threadIdx.x; p < n; p += (u64)gridDim.x * kGridBlock) {
        const uint32_t rank = a.pos[p];
        if (rank == kNoTile) continue;
        const double x = a.x[p], y = a.y[p], z = a.z[p];
        const double ux = (double)((const R *)a.ux)[p], uy = (double)((const R *)a.uy)[p],
                     uz = (double)((const R *)a.uz)[p];
        const double w = (double)((const R *)a.w)[p];
        const double gi = 1.0 / sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        const bool ok = isfinite(w * gi * (ux + uy + uz));
        uint32_t nd[3], local;
        double ph[3];
        node_cell(g, x, y, z, nd, ph);
        const uint32_t t = tile_of(a, nd, local);
        // one 64-byte line per record, written as four 16-byte stores
        DepRecord *r = a.rec + ((u64)a.off[t] + rank);
        double2 *v = reinterpret_cast<double2 *>(r);
        v[0] = make_double2(ph[0], ph[1]);
        v[1] = make_double2(ph[2], ok ? scale * w * ux * gi : 0.0);
        v[2] = make_double2(ok ? scale * w * uy * gi : 0.0, ok ? scale * w * uz * gi : 0.0);
        reinterpret_cast<uint4 *>(r)[3] = make_uint4(local, 0u, 0u, 0u);
    }
}

// The 8 lattice points and weights of current component c: along axis c (the
// lattice shifted by half a cell) the two points at offsets (-1, 0) or (0, +1) from
// the node cell, along the others (0, +1).  lo[d] is the lower offset.
__device__ __forceinline__ void comp_weights(int c, const double ph[3], int lo[3], double wl[3], double wh[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = ph[d];
        if (d == c) {
            const bool up = f >= 0.5;
            lo[d] = up ? 0 : -1;
            wl[d] = up ? 1.5 - f : 0.5 - f;
            wh[d] = up ? f - 0.5 : f + 0.5;
        } else {
            lo[d] = 0;
            wl[d] = 1.0 - f;
            wh[d] = f;
        }
    }
}

__global__ __launch_bounds__(kGridBlock) void k_dep_accum(DepSortArgs a) {
    __shared__ double acc[kStage];
    const uint32_t part = blockIdx.x;
    if (part >= a.part_off[a.ntiles]) return;   // whole block
    const uint32_t t = a.part_tile[part];
    // part k of a tile's np parts takes every np-th of its records from the k-th on,
    // and the lanes of a wave take records `rows` apart within the part (read as a
    // 64 x rows matrix, transposed): particles stored in cell order then spread over
    // the tile's cells instead of adding to the same LDS points together
    const uint32_t np = a.part_off[t + 1] - a.part_off[t], k0 = part - a.part_off[t];
    const uint32_t r0 = a.off[t] + k0, tile_cnt = a.off[t + 1] - a.off[t];
    const uint32_t cnt = (tile_cnt - k0 + np - 1) / np, rows = (cnt + 63) / 64;
    for (uint32_t e = threadIdx.x; e < kStage; e += kGridBlock) acc[e] = 0.0;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < 64 * rows; k += kGridBlock) {
        const uint32_t kk = (k % 64) * rows + k / 64;
        if (kk >= cnt) continue;
        const DepRecord *rp = a.rec + (r0 + (u64)kk * np);
        const double2 v0 = reinterpret_cast<const double2 *>(rp)[0], v1 = reinterpret_cast<const double2 *>(rp)[1],
                      v2 = reinterpret_cast<const double2 *>(rp)[2];
        const uint32_t key = reinterpret_cast<const uint4 *>(rp)[3].x;
        const double ph[3] = {v0.x, v0.y, v1.x};
        const double cur[3] = {v1.y, v2.x, v2.y};
        const uint32_t loc[3] = {key & 3u, (key >> 2) & 3u, (key >> 4) & 3u};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int lo[3];
            double wl[3], wh[3];
            comp_weights(c, ph, lo, wl, wh);
            // region point (c, lz, ly, lx) is node offset l - 1 from the tile's corner
            const uint32_t b = ((c * kRegionEdge + loc[2] + lo[2] + 1) * kRegionEdge + loc[1] + lo[1] + 1) *
                                   kRegionEdge + loc[0] + lo[0] + 1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double v = cur[c] * ((q & 4) ? wh[2] : wl[2]) * ((q & 2) ? wh[1] : wl[1]) * ((q & 1) ? wh[0] : wl[0]);
                unsafeAtomicAdd(&acc[b + ((q >> 2) & 1) * kRegionEdge * kRegionEdge + ((q >> 1) & 1) * kRegionEdge +
                                     (q & 1)],
                                v);
            }
        }
    }
    __syncthreads();
    double *st = a.stage + (u64)part * kStage;
    for (uint32_t e = threadIdx.x; e < kStage; e += kGridBlock) st[e] = acc[e];
}

// Tiles along one axis whose region holds grid coordinate gi (0 <= gi < n): pairs
// (tile, region coordinate l in [0, kRegionEdge)) over the periodic images gi - n, gi,
// gi + n.  A region point further than one cell from the tile's nodes is never
// touched, so the images beyond these hold nothing.  Returns the number of pairs.
constexpr int kMaxCover = 5;

__device__ __forceinline__ int cover(int gi, int n, int ntile, int T[kMaxCover], int L[kMaxCover]) {
    int c = 0;
#pragma unroll
    for (int im = -1; im <= 1; ++im) {
        const int h = gi + im * n;
        // l = h - kTileEdge * tile + 1 in [0, kRegionEdge)
        const int hi = (h + 1) >= 0 ? (h + 1) / (int)kTileEdge : -1;   // largest tile with l >= 0
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int tt = hi - k;
            const int l = h - (int)kTileEdge * tt + 1;
            if (tt >= 0 && tt < ntile && l >= 0 && l < (int)kRegionEdge && c < kMaxCover) {
                T[c] = tt;
                L[c] = l;
                ++c;
            }
        }
    }
    return c;
}

__global__ __launch_bounds__(kGridBlock) void k_dep_reduce(GridDev g, DepSortArgs a) {
    const u64 ncell = (u64)g.nx * g.ny * g.nz;
    for (u64 q = (u64)blockIdx.x * kGridBlock + threadIdx.x; q < 3 * ncell; q += (u64)gridDim.x * kGridBlock) {
        const uint32_t c = (uint32_t)(q / ncell);
        const u64 gq = q - c * ncell;
        const int gx = (int)(gq % g.nx), gy = (int)((gq / g.nx) % g.ny), gz = (int)(gq / ((u64)g.nx * g.ny));
        int Tx[kMaxCover], Lx[kMaxCover], Ty[kMaxCover], Ly[kMaxCover], Tz[kMaxCover], Lz[kMaxCover];
        const int cx = cover(gx, (int)g.nx, (int)a.tiles[0], Tx, Lx);
        const int cy = cover(gy, (int)g.ny, (int)a.tiles[1], Ty, Ly);
        const int cz = cover(gz, (int)g.nz, (int)a.tiles[2], Tz, Lz);
        double sum = 0.0;
        if (cx <= 2 && cy <= 2 && cz <= 2) {
            // at most 8 regions: their part ranges first, then the staged values
            uint32_t p0[8], p1[8], e[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ix = q & 1, iy = (q >> 1) & 1, iz = q >> 2;
                p0[q] = p1[q] = 0;
                e[q] = 0;
                if (ix < cx && iy < cy && iz < cz) {
                    const uint32_t t = ((uint32_t)Tz[iz] * a.tiles[1] + (uint32_t)Ty[iy]) * a.tiles[0] + (uint32_t)Tx[ix];
                    p0[q] = a.part_off[t];
                    p1[q] = a.part_off[t + 1];
                    e[q] = c * kRegionPts + ((uint32_t)Lz[iz] * kRegionEdge + (uint32_t)Ly[iy]) * kRegionEdge +
                           (uint32_t)Lx[ix];
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (p1[q] > p0[q]) sum += a.stage[(u64)p0[q] * kStage + e[q]];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                for (uint32_t p = p0[q] + 1; p < p1[q]; ++p) sum += a.stage[(u64)p * kStage + e[q]];
        } else {
            for (int iz = 0; iz < cz; ++iz)
                for (int iy = 0; iy < cy; ++iy)
                    for (int ix = 0; ix < cx; ++ix) {
                        const uint32_t t =
                            ((uint32_t)Tz[iz] * a.tiles[1] + (uint32_t)Ty[iy]) * a.tiles[0] + (uint32_t)Tx[ix];
                        const uint32_t e = c * kRegionPts +
                                           ((uint32_t)Lz[iz] * kRegionEdge + (uint32_t)Ly[iy]) * kRegionEdge +
                                           (uint32_t)Lx[ix];
                        for (uint32_t p = a.part_off[t]; p < a.part_off[t + 1]; ++p)
                            sum += a.stage[(u64)p * kStage + e];
                    }
        }
        if (sum != 0.0) a.j[c][gq] += sum;
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

hipError_t launch_deposit_sorted(const GridDev &g, const DepSortArgs &a, int dtype, int blocks, hipStream_t s) {
    const u64 per_bin = (u64)kGridBlock * kBinItems;
    const int bin_blocks = (int)((a.cap + per_bin - 1) / per_bin);
    if (bin_blocks == 0) return hipSuccess;
    if (a.ntiles <= kBinLdsTiles)
        hipLaunchKernelGGL(k_dep_bin<true>, dim3(bin_blocks), dim3(kGridBlock), 0, s, g, a);
    else
        hipLaunchKernelGGL(k_dep_bin<false>, dim3(bin_blocks), dim3(kGridBlock), 0, s, g, a);
    hipLaunchKernelGGL(k_dep_scan, dim3(1), dim3(kScanBlock), 0, s, a);
    if (dtype == 0)
        hipLaunchKernelGGL(k_dep_scatter<float>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    else
        hipLaunchKernelGGL(k_dep_scatter<double>, dim3(blocks), dim3(kGridBlock), 0, s, g, a);
    hipLaunchKernelGGL(k_dep_accum, dim3((uint32_t)a.max_parts), dim3(kGridBlock), 0, s, a);
    const u64 pts = 3ull * g.nx * g.ny * g.nz;
    const u64 rblocks = (pts + kGridBlock - 1) / kGridBlock;
    hipLaunchKernelGGL(k_dep_reduce, dim3((uint32_t)(rblocks < 65536 ? rblocks : 65536)), dim3(kGridBlock), 0, s, g, a);
    return hipGetLastError();
}

}  // namespace qed
