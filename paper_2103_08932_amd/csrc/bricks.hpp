// bricks.hpp -- brick geometry shared by setup, the per-pair passes and the damping pass.
//
// A brick is a run of `zb` consecutive cells along the fastest cell axis (z in 3D, y in 2D):
// cells (cx, cy, cz0 .. cz0 + zb - 1) in 3D, (cx, cy0 .. cy0 + zb - 1) in 2D.  Because particles
// are sorted by cell id, the brick's own particles are one contiguous range, and its neighbourhood
// (every cell within one cell of the brick) is 3^(dim-1) contiguous "runs" of particles: for each
// offset of the slow axes, the zb + 2 cells along the fast axis.  A workgroup stages the
// neighbourhood in LDS run after run; the halo slot of particle j is its position in that
// concatenation.  Per-pair halo slots (uint16) are precomputed at setup, so the per-pair passes
// read 2 bytes per neighbour instead of a 4-byte particle index and never search the runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlsph {

// Compact brick neighbourhoods (pass B of large bodies): per brick and 64-slot group of its
// neighbourhood, the slots its own rows read (mask) and the read slots of the groups before
// (prefix).  A brick then stages only those slots, at their rank among them; its rows' pass-B slots
// hold those ranks.
struct CMapWord {
    uint64_t mask;
    int32_t prefix;
    int32_t pad;
};

struct BrickGeom {
    int dim;
    int32_t nc[3];
    int zb;        // cells per brick along the fast axis
    int nbf;       // bricks along the fast axis = ceil(nfast / zb)
    int tile[3];   // 3D: brick order in tiles of tile[0] x tile[1] columns x tile[2] bricks (0: column order)
    const CMapWord *cmap;   // compact neighbourhoods: [bricks][cmap_words] (null: full neighbourhoods)
    int cmap_words;
    const int32_t *runs;    // [bricks][run_words] run descriptors (pair-pass geometries; set at setup)
};

__host__ __device__ inline int fast_cells(const BrickGeom &g) { return g.dim == 3 ? g.nc[2] : g.nc[1]; }

__host__ __device__ inline int64_t brick_count(const BrickGeom &g)
{
    return g.dim == 3 ? (int64_t)g.nc[0] * g.nc[1] * g.nbf : (int64_t)g.nc[0] * g.nbf;
}

__host__ __device__ inline int64_t cell_lin(const BrickGeom &g, int x, int y, int z)
{
    return g.dim == 2 ? (int64_t)x * g.nc[1] + y : ((int64_t)x * g.nc[1] + y) * g.nc[2] + z;
}

// brick index -> slow-axis cell coordinates and first fast-axis cell.  Column order: fast axis
// fastest, then cy, then cx.  Tiled order (3D bodies with tile[0] > 0): tiles of tile[0] x tile[1]
// columns x tile[2] bricks (clipped at the grid's edges), tiles in column order, bricks inside a tile
// in column order, so that the bricks one XCD runs at a time (consecutive indices) share one
// L2-sized neighbourhood.
__device__ inline void brick_coords(const BrickGeom &g, int64_t b, int &cx, int &cy, int &f0)
{
    if (g.dim == 3 && g.tile[0] > 0) {
        const int TX = g.tile[0], TY = g.tile[1], TZ = g.tile[2];
        const int ny = g.nc[1], nz = g.nbf;
        int r = (int)b;                          // bodies with tiled order hold fewer than 2^31 bricks
        const int tx = r / (TX * ny * nz);
        r -= tx * TX * ny * nz;
        const int wx = g.nc[0] - tx * TX < TX ? g.nc[0] - tx * TX : TX;
        const int ty = r / (wx * TY * nz);
        r -= ty * wx * TY * nz;
        const int wy = ny - ty * TY < TY ? ny - ty * TY : TY;
        const int tz = r / (wx * wy * TZ);
        r -= tz * wx * wy * TZ;
        const int wz = nz - tz * TZ < TZ ? nz - tz * TZ : TZ;
        const int ix = r / (wy * wz);
        r -= ix * wy * wz;
        const int iy = r / wz, iz = r - iy * wz;
        cx = tx * TX + ix;
        cy = ty * TY + iy;
        f0 = (tz * TZ + iz) * g.zb;
        return;
    }
    const int64_t bf = b % g.nbf;
    const int64_t t = b / g.nbf;
    if (g.dim == 3) {
        cy = (int)(t % g.nc[1]);
        cx = (int)(t / g.nc[1]);
    } else {
        cx = (int)t;
        cy = 0;
    }
    f0 = (int)bf * g.zb;
}

template <int D>
struct BrickRuns {
    static constexpr int NR = (D == 3) ? 9 : 3;
    static constexpr int CR = (D == 3) ? 4 : 1;   // run that holds the brick itself
    int start[NR];
    int len[NR];
    int off[NR];
    int total;
    int own0, own1;      // the brick's own particles [own0, own1)
};

// Runs of the neighbourhood of the brick (cx, cy, f0): 3D cells (cx+dx, cy+dy, f0-1 .. f0+zb),
// 2D cells (cx+dx, f0-1 .. f0+zb), clipped to the grid; runs ordered by (dx, dy) ascending, which
// is ascending particle index.
template <int D>
__device__ inline void brick_runs(const BrickGeom &g, const int32_t *__restrict__ cell_start, int cx, int cy, int f0,
                                  BrickRuns<D> &R)
{
    const int nf = fast_cells(g);
    const int fa = f0 > 0 ? f0 - 1 : 0;
    const int fb = (f0 + g.zb < nf) ? f0 + g.zb : nf - 1;
    const int oa = f0, ob = (f0 + g.zb - 1 < nf) ? f0 + g.zb - 1 : nf - 1;
    int tot = 0;
#pragma unroll
    for (int r = 0; r < BrickRuns<D>::NR; ++r) {
        int s0 = 0, l0 = 0;
        if constexpr (D == 3) {
            const int x = cx + r / 3 - 1, y = cy + r % 3 - 1;
            if (x >= 0 && x < g.nc[0] && y >= 0 && y < g.nc[1]) {
                s0 = cell_start[cell_lin(g, x, y, fa)];
                l0 = cell_start[cell_lin(g, x, y, fb) + 1] - s0;
            }
        } else {
            const int x = cx + r - 1;
            if (x >= 0 && x < g.nc[0]) {
                s0 = cell_start[cell_lin(g, x, fa, 0)];
                l0 = cell_start[cell_lin(g, x, fb, 0) + 1] - s0;
            }
        }
        R.start[r] = s0;
        R.len[r] = l0;
        R.off[r] = tot;
        tot += l0;
    }
    R.total = tot;
    if constexpr (D == 3) {
        R.own0 = cell_start[cell_lin(g, cx, cy, oa)];
        R.own1 = cell_start[cell_lin(g, cx, cy, ob) + 1];
    } else {
        R.own0 = cell_start[cell_lin(g, cx, oa, 0)];
        R.own1 = cell_start[cell_lin(g, cx, ob, 0) + 1];
    }
}

// Run descriptors: a brick's runs are fixed once the cells are sorted (neighbourhoods live in the
// reference configuration), so setup stores them per brick and the pair passes read one record
// (three scalar loads) instead of decoding the brick index and looking up 2 NR + 2 cell starts.
// Record of a brick: start[NR], off[NR], total, own0, own1, padded to run_words<D>() words.
template <int D> constexpr int run_words() { return D == 3 ? 24 : 12; }

template <int D>
__device__ __forceinline__ void store_runs(const BrickRuns<D> &R, int32_t *__restrict__ d)
{
    constexpr int NR = BrickRuns<D>::NR;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        d[r] = R.start[r];
        d[NR + r] = R.off[r];
    }
    d[2 * NR] = R.total;
    d[2 * NR + 1] = R.own0;
    d[2 * NR + 2] = R.own1;
#pragma unroll
    for (int k = 2 * NR + 3; k < run_words<D>(); ++k) d[k] = 0;
}

// The runs of brick `blk` (the index after the XCD remap) from its record; the geometry must carry
// the records (both pair-pass geometries do once the body is set up).
template <int D>
__device__ __forceinline__ void brick_runs_of(const BrickGeom &g, int64_t blk, BrickRuns<D> &R)
{
    constexpr int NR = BrickRuns<D>::NR;
    const int32_t *__restrict__ d = g.runs + blk * run_words<D>();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        R.start[r] = d[r];
        R.off[r] = r == 0 ? 0 : d[NR + r];   // the first run starts the neighbourhood (a known zero
    }                                        // keeps the staging loop's run search short)
    R.total = d[2 * NR];
    R.own0 = d[2 * NR + 1];
    R.own1 = d[2 * NR + 2];
#pragma unroll
    for (int r = 0; r < NR; ++r) R.len[r] = (r + 1 < NR ? R.off[r + 1] : R.total) - R.off[r];
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Launching
// 8 * ceil(nb / 8) workgroups and mapping workgroup w to logical block (w % 8) * per + w / 8 gives
// every XCD one contiguous range of blocks, so neighbouring blocks, which read overlapping
// neighbourhoods, share an L2.  Returns -1 for the padding workgroups.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t xcd_grid(int64_t nb) { return kXcds * ((nb + kXcds - 1) / kXcds); }
__device__ inline int64_t xcd_block(int64_t w, int64_t nb)
{
    const int64_t per = (nb + kXcds - 1) / kXcds;
    const int64_t l = (w % kXcds) * per + w / kXcds;
    return l < nb ? l : -1;
}

// Particle index of position `idx` of the concatenated neighbourhood (0 <= idx < R.total).  Run
// offsets ascend, so the last run whose offset is <= idx holds it (empty runs are skipped because
// the next run starts at the same offset).
template <int D>
__device__ __forceinline__ int halo_particle(const BrickRuns<D> &R, int idx)
{
    int j = 0;
#pragma unroll
    for (int r = 0; r < BrickRuns<D>::NR; ++r)
        if (idx >= R.off[r]) j = R.start[r] + (idx - R.off[r]);
    return j;
}

}  // namespace tlsph
