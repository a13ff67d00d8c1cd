// setup.hip -- once-per-body construction on the GPU: cell binning (cell size = cut-off,
// Sec. 3.4), cell-sorted internal order, CSR neighbour rows of the reference configuration and
// the kernel-correction matrices B0 (Eq. 9).
//
// This translation unit is compiled with -ffp-contract=off: the cell index floor((X - Xmin) / r_c)
// and the squared distance ((dx dx + dy dy) + dz dz) < r_c^2 are rounded operation by operation,
// so the neighbour lists and the colouring are reproducible bit for bit on any IEEE machine.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bricks.hpp"
#include "internal.hpp"

namespace tlsph {
size_t passB_lds_bytes(int dim, int precision, int hcap);
size_t passA_lds_bytes(int dim, int precision, int hcap, int zb);
namespace {

struct Grid {
    int dim;
    int32_t nc[3];
    double xmin[3];
    double rc, rc2;
};

__device__ __forceinline__ int64_t lin_of(const Grid &g, int cx, int cy, int cz)
{
    return g.dim == 2 ? (int64_t)cx * g.nc[1] + cy : ((int64_t)cx * g.nc[1] + cy) * g.nc[2] + cz;
}

__device__ __forceinline__ void coords_of(const Grid &g, int64_t lin, int c[3])
{
    if (g.dim == 2) {
        c[0] = (int)(lin / g.nc[1]);
        c[1] = (int)(lin % g.nc[1]);
        c[2] = 0;
    } else {
        c[2] = (int)(lin % g.nc[2]);
        int64_t t = lin / g.nc[2];
        c[1] = (int)(t % g.nc[1]);
        c[0] = (int)(t / g.nc[1]);
    }
}

// Cell of every input particle; per-cell counts.
__global__ void k_bin(Grid g, const double *__restrict__ X0, int64_t n, int32_t *__restrict__ cell_in,
                      int32_t *__restrict__ count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3] = {0, 0, 0};
    for (int k = 0; k < g.dim; ++k) {
        double x = X0[i * g.dim + k];
        int ck = (int)floor((x - g.xmin[k]) / g.rc);
        c[k] = ck < 0 ? 0 : (ck >= g.nc[k] ? g.nc[k] - 1 : ck);
    }
    int32_t lin = (int32_t)lin_of(g, c[0], c[1], c[2]);
    cell_in[i] = lin;
    atomicAdd(&count[lin], 1);
}

__global__ void k_scatter(const int32_t *__restrict__ cell_in, int64_t n, const int32_t *__restrict__ cell_start,
                          int32_t *__restrict__ fill, int32_t *__restrict__ perm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = cell_in[i];
    int32_t pos = cell_start[c] + atomicAdd(&fill[c], 1);
    perm[pos] = (int32_t)i;
}

// Particles of a cell in ascending input index (the atomic scatter left them in arbitrary order).
__global__ void k_sort_cells(const int32_t *__restrict__ cell_start, int64_t ncell, int32_t *__restrict__ perm)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int32_t lo = cell_start[c], hi = cell_start[c + 1];
    for (int32_t a = lo + 1; a < hi; ++a) {
        int32_t key = perm[a];
        int32_t b = a - 1;
        while (b >= lo && perm[b] > key) {
            perm[b + 1] = perm[b];
            --b;
        }
        perm[b + 1] = key;
    }
}

__global__ void k_gather(const int32_t *__restrict__ perm, int64_t n, int dim, const double *__restrict__ X0,
                         const uint8_t *__restrict__ cl_in, double *__restrict__ X, uint8_t *__restrict__ clamped)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t i = perm[p];
    for (int k = 0; k < dim; ++k) X[k * n + p] = X0[i * dim + k];
    clamped[p] = cl_in ? (cl_in[i] != 0) : 0;
}

// Neighbour search of internal particle p over the 3^dim adjacent cells in ascending cell id,
// particles of a cell ascending: count (col == nullptr) or write the row.
template <int D>
__device__ int64_t scan_row(const Grid &g, const double *__restrict__ X, int64_t n,
                            const int32_t *__restrict__ cell_start, int64_t p, int32_t cellp,
                            int32_t *__restrict__ col)
{
    int c[3];
    coords_of(g, cellp, c);
    double xp[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xp[k] = X[k * n + p];
    int64_t cnt = 0;
    const int zlo = (D == 3) ? -1 : 0, zhi = (D == 3) ? 1 : 0;
    for (int dx = -1; dx <= 1; ++dx) {
        int cx = c[0] + dx;
        if (cx < 0 || cx >= g.nc[0]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = c[1] + dy;
            if (cy < 0 || cy >= g.nc[1]) continue;
            for (int dz = zlo; dz <= zhi; ++dz) {
                int cz = c[2] + dz;
                if (D == 3 && (cz < 0 || cz >= g.nc[2])) continue;
                int64_t lin = lin_of(g, cx, cy, cz);
                for (int32_t j = cell_start[lin]; j < cell_start[lin + 1]; ++j) {
                    if (j == p) continue;
                    double d0 = X[j] - xp[0];
                    double d1 = X[n + j] - xp[1];
                    double r2 = d0 * d0 + d1 * d1;
                    if constexpr (D == 3) {
                        double d2 = X[2 * n + j] - xp[2];
                        r2 = r2 + d2 * d2;
                    }
                    if (r2 < g.rc2) {
                        if (col) col[cnt] = j;
                        ++cnt;
                    }
                }
            }
        }
    }
    return cnt;
}

template <int D>
__global__ void k_row_count(Grid g, const double *__restrict__ X, int64_t n, const int32_t *__restrict__ cell_start,
                            const int32_t *__restrict__ cell_of, int64_t *__restrict__ cnt, int *__restrict__ rowmax)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t c = scan_row<D>(g, X, n, cell_start, p, cell_of[p], nullptr);
    cnt[p] = c;
    atomicMax(rowmax, (int)c);
}

template <int D>
__global__ void k_row_fill(Grid g, const double *__restrict__ X, int64_t n, const int32_t *__restrict__ cell_start,
                           const int32_t *__restrict__ cell_of, const int64_t *__restrict__ row_ptr,
                           int32_t *__restrict__ col)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    scan_row<D>(g, X, n, cell_start, p, cell_of[p], col + row_ptr[p]);
}

// Cell id of each internal particle, and the size of each cell's 3^dim neighbourhood.
__global__ void k_cell_of(const int32_t *__restrict__ cell_start, int64_t ncell, int32_t *__restrict__ cell_of)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int32_t p = cell_start[c]; p < cell_start[c + 1]; ++p) cell_of[p] = (int32_t)c;
}

__global__ void k_halo_max(Grid g, const int32_t *__restrict__ cell_start, int64_t ncell, int *__restrict__ hmax)
{
    int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lin >= ncell) return;
    if (cell_start[lin] == cell_start[lin + 1]) return;
    int c[3];
    coords_of(g, lin, c);
    int tot = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = (g.dim == 3 ? -1 : 0); dz <= (g.dim == 3 ? 1 : 0); ++dz) {
                int cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                if (cx < 0 || cy < 0 || cx >= g.nc[0] || cy >= g.nc[1]) continue;
                if (g.dim == 3 && (cz < 0 || cz >= g.nc[2])) continue;
                int64_t l2 = lin_of(g, cx, cy, cz);
                tot += cell_start[l2 + 1] - cell_start[l2];
            }
    atomicMax(hmax, tot);
}

// Eq. 9:  B0_p = ( - sum_j V (X_p - X_j) (x) grad0_p W_pj )^-1  in FP64, stored as Real.
// grad0_p W_pj = (dW/dr) (X_p - X_j) / r with the Wendland C2 kernel.  Also the row sum of the
// kernel gradient, which the reference configuration fixes: gsum_p = sum_j (1 - q/2)^3 (X_p - X_j)
// = sum_j grad0_p W_pj / kfac (kfac = -5 a_D / h^2), the factor of T_p in the force of Eq. 12.
template <int D, typename R>
__global__ void k_B0(const double *__restrict__ X, int64_t n, const int64_t *__restrict__ row_ptr,
                     const int32_t *__restrict__ col, double h, double aD, double vol, R *__restrict__ B0,
                     R *__restrict__ gsum, int *__restrict__ singular)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double M[D * D], G[D];
    for (int k = 0; k < D * D; ++k) M[k] = 0.0;
    for (int k = 0; k < D; ++k) G[k] = 0.0;
    double xp[D];
    for (int k = 0; k < D; ++k) xp[k] = X[k * n + p];
    for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
        int32_t j = col[e];
        double d[D];
        double r2 = 0.0;
        for (int k = 0; k < D; ++k) {
            d[k] = xp[k] - X[k * n + j];
            r2 += d[k] * d[k];
        }
        double r = sqrt(r2);
        double q = r / h;
        double t = 1.0 - 0.5 * q;
        double dW = aD / h * (-5.0 * q) * t * t * t;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) M[a * D + b] -= vol * d[a] * (dW * d[b] / r);
        const double t3 = t * t * t;
        for (int k = 0; k < D; ++k) G[k] += t3 * d[k];
    }
    for (int k = 0; k < D; ++k) gsum[k * n + p] = (R)G[k];
    double nrm = 0.0;
    for (int k = 0; k < D * D; ++k) nrm = fmax(nrm, fabs(M[k]));
    double Bi[D * D];
    double det;
    if constexpr (D == 2) {
        det = M[0] * M[3] - M[1] * M[2];
        Bi[0] = M[3] / det; Bi[1] = -M[1] / det; Bi[2] = -M[2] / det; Bi[3] = M[0] / det;
    } else {
        double c00 = M[4] * M[8] - M[5] * M[7];
        double c01 = M[5] * M[6] - M[3] * M[8];
        double c02 = M[3] * M[7] - M[4] * M[6];
        det = M[0] * c00 + M[1] * c01 + M[2] * c02;
        Bi[0] = c00 / det;
        Bi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
        Bi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
        Bi[3] = c01 / det;
        Bi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
        Bi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
        Bi[6] = c02 / det;
        Bi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
        Bi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    }
    double scale = (D == 2) ? nrm * nrm : nrm * nrm * nrm;
    if (!(fabs(det) > 1e-12 * scale) || nrm == 0.0) {
        atomicMax(singular, 1);
        for (int k = 0; k < D * D; ++k) Bi[k] = 0.0;
    }
    for (int k = 0; k < D * D; ++k) B0[k * n + p] = (R)Bi[k];
}

// Largest brick neighbourhood (particles) for a brick depth.
template <int D>
__global__ void k_brick_halo(BrickGeom g, const int32_t *__restrict__ cell_start, int *__restrict__ hmax)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= brick_count(g)) return;
    int cx, cy, f0;
    brick_coords(g, b, cx, cy, f0);
    BrickRuns<D> R;
    brick_runs<D>(g, cell_start, cx, cy, f0, R);
    if (R.own1 > R.own0) atomicMax(hmax, R.total);
}

// Compact damping neighbourhoods.  Of the slots of a cell's 3^D-cell neighbourhood, its particles'
// damping visits read only the cell's own particles and the entries of their rows (on a lattice at
// h = 1.3 dp about half of the neighbourhood: a 3 x 3 x 3-particle cell reads 275 of 512 slots).
// Sixteen lanes per cell mark those slots in a mask (slot s < 1024 is bit s >> 4 of lane s & 15, the
// lane that stages slot s), number them consecutively in slot order, and rewrite the damping slots
// of the cell's CSR entries in place with those numbers (the clamp-class bits kept).  out_own gets
// the compact slot of the cell's first own particle (own particles are consecutive slots, all
// read, so their compact slots are consecutive too), hmax the largest compact neighbourhood.
template <int D>
__global__ void k_compact(BrickGeom g, const int32_t *__restrict__ cell_start, const int64_t *__restrict__ row_ptr,
                          uint16_t *__restrict__ dslot, int64_t ncell, uint64_t *__restrict__ out_mask,
                          int32_t *__restrict__ out_own, int *__restrict__ hmax)
{
    __shared__ unsigned long long m[16][16];
    __shared__ unsigned int colbits[16][64];   // bit l of column k: slot 16 k + l is read
    __shared__ int colrank[16][64];            // compact slots before column k
    const int grp = threadIdx.x / 16, sl = threadIdx.x % 16;
    const int64_t lin = (int64_t)blockIdx.x * 16 + grp;
    const bool ok = lin < ncell;
    m[grp][sl] = 0;
    __syncthreads();
    BrickRuns<D> R;
    int cbase = 0;
    if (ok) {
        if constexpr (D == 3) {
            const int cz = (int)(lin % g.nc[2]), cy = (int)((lin / g.nc[2]) % g.nc[1]),
                      cx = (int)(lin / g.nc[2] / g.nc[1]);
            brick_runs<D>(g, cell_start, cx, cy, cz, R);
        } else {
            const int cy = (int)(lin % g.nc[1]), cx = (int)(lin / g.nc[1]);
            brick_runs<D>(g, cell_start, cx, 0, cy, R);
        }
        cbase = R.off[BrickRuns<D>::CR] - R.start[BrickRuns<D>::CR];
        for (int q = R.own0 + sl; q < R.own1; q += 16) {
            const int slot = q + cbase;
            atomicOr(&m[grp][slot & 15], 1ull << (slot >> 4));
        }
        const int64_t e1 = row_ptr[R.own1];
        for (int64_t e = row_ptr[R.own0] + sl; e < e1; e += 16) {
            const int slot = dslot[e] & 0x3fff;
            atomicOr(&m[grp][slot & 15], 1ull << (slot >> 4));
        }
    }
    __syncthreads();
    for (int k = sl; k < 64; k += 16) {
        unsigned int w = 0;
        for (int l = 0; l < 16; ++l) w |= (unsigned int)((m[grp][l] >> k) & 1ull) << l;
        colbits[grp][k] = w;
    }
    __syncthreads();
    if (sl == 0) {
        int acc = 0;
        for (int k = 0; k < 64; ++k) {
            colrank[grp][k] = acc;
            acc += __popc(colbits[grp][k]);
        }
        if (ok) atomicMax(hmax, acc);
    }
    __syncthreads();
    if (!ok) return;
    auto rank = [&](int slot) {
        const int k = slot >> 4;
        return colrank[grp][k] + __popc(colbits[grp][k] & ((1u << (slot & 15)) - 1u));
    };
    const int64_t e1 = row_ptr[R.own1];
    for (int64_t e = row_ptr[R.own0] + sl; e < e1; e += 16) {
        const int raw = dslot[e];
        dslot[e] = (uint16_t)((raw & 0xc000) | rank(raw & 0x3fff));
    }
    out_mask[lin * 16 + sl] = m[grp][sl];
    if (sl == 0) out_own[lin] = R.own1 > R.own0 ? rank(R.own0 + cbase) : 0;
}

// The run descriptor of every brick of geometry g (bricks.hpp), one thread per brick.
template <int D>
__global__ void k_brick_runs(BrickGeom g, const int32_t *__restrict__ cell_start, int32_t *__restrict__ out)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= brick_count(g)) return;
    int cx, cy, f0;
    brick_coords(g, b, cx, cy, f0);
    BrickRuns<D> R;
    brick_runs<D>(g, cell_start, cx, cy, f0, R);
    store_runs<D>(R, out + b * run_words<D>());
}

// Compact brick neighbourhoods (pass B): of a brick's neighbourhood its own rows read only part (on
// the lattice at h = 1.3 dp 590 of a 4-cell brick's 1024 slots).
// One workgroup per brick marks the slots its own particles and their rows read, writes the brick's
// map (per 64-slot group: mask, read slots before the group) and rewrites its rows' slots in place
// with their rank among the read slots; hmax gets the largest count.
template <int D>
__global__ void k_compact_brick(BrickGeom g, const int32_t *__restrict__ cell_start,
                                const int64_t *__restrict__ row_ptr, uint16_t *__restrict__ hslot, int words,
                                CMapWord *__restrict__ out, int *__restrict__ hmax)
{
    __shared__ unsigned long long m[32];
    __shared__ int pre[32];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    if (t < 32) m[t] = 0;
    __syncthreads();
    int cx, cy, f0;
    brick_coords(g, b, cx, cy, f0);
    BrickRuns<D> R;
    brick_runs<D>(g, cell_start, cx, cy, f0, R);
    const int cbase = R.off[BrickRuns<D>::CR] - R.start[BrickRuns<D>::CR];
    for (int q = R.own0 + t; q < R.own1; q += blockDim.x) {
        const int sl = q + cbase;
        atomicOr(&m[sl >> 6], 1ull << (sl & 63));
    }
    const int64_t e0 = row_ptr[R.own0], e1 = row_ptr[R.own1];
    for (int64_t e = e0 + t; e < e1; e += blockDim.x) {
        const int sl = hslot[e];
        atomicOr(&m[sl >> 6], 1ull << (sl & 63));
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int w = 0; w < words; ++w) {
            pre[w] = acc;
            acc += __popcll(m[w]);
        }
        atomicMax(hmax, acc);
    }
    __syncthreads();
    if (t < words) {
        CMapWord c;
        c.mask = m[t];
        c.prefix = pre[t];
        c.pad = 0;
        out[b * words + t] = c;
    }
    for (int64_t e = e0 + t; e < e1; e += blockDim.x) {
        const int sl = hslot[e];
        hslot[e] = (uint16_t)(pre[sl >> 6] + __popcll(m[sl >> 6] & ((1ull << (sl & 63)) - 1ull)));
    }
}

// Longest row among the own particles of every brick (the row-loop bound of passes A and B).
template <int D>
__global__ void k_brick_lmax(BrickGeom g, const int32_t *__restrict__ cell_start, const int64_t *__restrict__ row_ptr,
                             int32_t *__restrict__ lmax)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= brick_count(g)) return;
    int cx, cy, f0;
    brick_coords(g, b, cx, cy, f0);
    BrickRuns<D> R;
    brick_runs<D>(g, cell_start, cx, cy, f0, R);
    int m = 0;
    for (int64_t p = R.own0; p < R.own1; ++p) m = max(m, (int)(row_ptr[p + 1] - row_ptr[p]));
    lmax[b] = m;
}

// Halo slot (position in its brick's neighbourhood) of every CSR entry of particle p.
// With `clamped` non-null (single-cell bricks of the damping pass) the top two bits carry the
// clamp class of the pair: bit 15 = i clamped, bit 14 = j clamped (slots must then be < 2^14).
template <int D>
__global__ void k_slots(BrickGeom g, const int32_t *__restrict__ cell_start, const int32_t *__restrict__ cell_of,
                        const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, int64_t n,
                        const uint8_t *__restrict__ clamped, uint16_t *__restrict__ slot, int *__restrict__ bad)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int c[3];
    const int64_t lin = cell_of[p];
    if (D == 3) {
        c[2] = (int)(lin % g.nc[2]);
        const int64_t t = lin / g.nc[2];
        c[1] = (int)(t % g.nc[1]);
        c[0] = (int)(t / g.nc[1]);
    } else {
        c[1] = (int)(lin % g.nc[1]);
        c[0] = (int)(lin / g.nc[1]);
        c[2] = 0;
    }
    const int cf = D == 3 ? c[2] : c[1];
    const int f0 = (cf / g.zb) * g.zb;
    BrickRuns<D> R;
    brick_runs<D>(g, cell_start, c[0], D == 3 ? c[1] : 0, f0, R);
    for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
        const int j = col[e];
        int s = -1;
#pragma unroll
        for (int r = 0; r < BrickRuns<D>::NR; ++r)
            if (j >= R.start[r] && j < R.start[r] + R.len[r]) s = R.off[r] + (j - R.start[r]);
        const int lim = clamped ? 16383 : 65535;
        if (s < 0 || s > lim) {
            atomicMax(bad, 1);
            s = 0;
        }
        if (clamped) s |= (clamped[p] ? 0x8000 : 0) | (clamped[j] ? 0x4000 : 0);
        slot[e] = (uint16_t)s;
    }
}

// Damping factor of every CSR entry: g_ij = 2 V^2 (dW/dr) / r (the pair coefficient of Eq. 27
// without eta and dt), FP64 arithmetic stored in the working precision.
template <int D, typename R>
__global__ void k_gdamp(const double *__restrict__ X, int64_t n, const int64_t *__restrict__ row_ptr,
                        const int32_t *__restrict__ col, double h, double aD, double vol, R *__restrict__ gd)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double xp[D];
    for (int k = 0; k < D; ++k) xp[k] = X[k * n + p];
    for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
        const int32_t j = col[e];
        double r2 = 0.0;
        for (int k = 0; k < D; ++k) {
            const double d = xp[k] - X[k * n + j];
            r2 += d * d;
        }
        const double r = sqrt(r2);
        const double q = r / h;
        const double t = 1.0 - 0.5 * q;
        const double dW = aD / h * (-5.0 * q) * t * t * t;
        gd[e] = (R)(2.0 * vol * vol * dW / r);
    }
}

// Largest particle count and largest CSR-entry count of one cell.
__global__ void k_cell_stats(const int32_t *__restrict__ cell_start, const int64_t *__restrict__ row_ptr,
                             int64_t ncell, int *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int32_t a = cell_start[c], b = cell_start[c + 1];
    atomicMax(&out[0], b - a);
    atomicMax(&out[1], (int)(row_ptr[b] - row_ptr[a]));
}

// ---------------------------------------------------------------------------------------------
// Device-wide exclusive scan (three phases: per-block scan, scan of block sums, add offsets).
// ---------------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename TI, typename TO>
__global__ void k_scan_local(const TI *__restrict__ in, TO *__restrict__ out, TO *__restrict__ bsum, int64_t n)
{
    __shared__ TO s[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO tsum = 0;
    for (int t = 0; t < kScanItems; ++t) {
        int64_t idx = base + t;
        v[t] = idx < n ? (TO)in[idx] : (TO)0;
        tsum += v[t];
    }
    s[threadIdx.x] = tsum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        TO x = (int)threadIdx.x >= off ? s[threadIdx.x - off] : (TO)0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    TO excl = s[threadIdx.x] - tsum;
    for (int t = 0; t < kScanItems; ++t) {
        int64_t idx = base + t;
        if (idx < n) out[idx] = excl;
        excl += v[t];
    }
    if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = s[kScanThreads - 1];
}

template <typename TO>
__global__ void k_scan_add(TO *__restrict__ out, const TO *__restrict__ boff, int64_t n)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += boff[idx / kScanTile];
}

struct Alloc {
    void *(*alloc)(size_t, void *);
    void (*dfree)(void *, void *);
    void *ctx;
    void *get(size_t bytes) const { return alloc(bytes ? bytes : 256, ctx); }
    void put(void *p) const { if (p) dfree(p, ctx); }
};

// out[0..n) = exclusive prefix sums of in[0..n).  Returns false on allocation failure.
template <typename TI, typename TO>
bool scan_exclusive(const TI *in, TO *out, int64_t n, const Alloc &A, hipStream_t s)
{
    if (n <= 0) return true;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    TO *bsum = (TO *)A.get(sizeof(TO) * nb);
    if (!bsum) return false;
    hipLaunchKernelGGL((k_scan_local<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, bsum, n);
    bool ok = true;
    if (nb > 1) {
        TO *boff = (TO *)A.get(sizeof(TO) * nb);
        if (!boff) ok = false;
        if (ok) ok = scan_exclusive<TO, TO>(bsum, boff, nb, A, s);
        if (ok)
            hipLaunchKernelGGL((k_scan_add<TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, boff, n);
        if (boff) {
            (void)hipStreamSynchronize(s);
            A.put(boff);
        }
    }
    (void)hipStreamSynchronize(s);
    A.put(bsum);
    return ok;
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Chooses the brick depth of each per-pair pass, the largest (up to a default) whose LDS tile fits
// in 64 KiB: pass A holds positions and half-step displacements of the neighbourhood plus the
// reduced sums of the own rows, pass B positions and T.  Pass A gains from long bricks (fewer halo
// particles staged per own particle), pass B from the occupancy of shorter ones (its tile is twice
// as wide).  Builds the slot arrays: bricks of pass A, of pass B (pass A's at equal depth), single
// cells for the damping pass.
int build_slots(DeviceBody &db, int precision, const int32_t *cell_of, int *flags, const Alloc &A, hipStream_t s,
                char *errmsg, size_t errlen)
{
    const int D = db.dim;
    auto geom = [&](int zb) {
        BrickGeom g;
        g.dim = D;
        for (int k = 0; k < 3; ++k) g.nc[k] = db.nc[k];
        g.zb = zb;
        const int nf = D == 3 ? db.nc[2] : db.nc[1];
        g.nbf = (nf + zb - 1) / zb;
        g.tile[0] = g.tile[1] = g.tile[2] = 0;
        g.cmap = nullptr;
        g.cmap_words = 0;
        g.runs = nullptr;
        return g;
    };
    auto halo_of = [&](int zb) -> int {
        BrickGeom g = geom(zb);
        int h = 0;
        (void)hipMemsetAsync(flags + 3, 0, sizeof(int), s);
        const int64_t nb = brick_count(g);
        if (D == 2)
            hipLaunchKernelGGL(k_brick_halo<2>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, flags + 3);
        else
            hipLaunchKernelGGL(k_brick_halo<3>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, flags + 3);
        (void)hipMemcpyAsync(&h, flags + 3, sizeof(int), hipMemcpyDeviceToHost, s);
        (void)hipStreamSynchronize(s);
        return h;
    };
    auto lds_a = [&](int zb, int h) { return passA_lds_bytes(D, precision, h, zb); };
    auto lds_b = [&](int, int h) { return passB_lds_bytes(D, precision, h); };
    // depth from `zb` down by halving until the tile fits; h = its largest neighbourhood
    auto pick = [&](int zb, auto lds_of, int &h) {
        h = halo_of(zb);
        while (zb > 1 && lds_of(zb, h) > 64 * 1024) {
            zb /= 2;
            h = halo_of(zb);
        }
        return zb;
    };
#ifndef TLSPH_BRICK_CELLS_A_3D
#define TLSPH_BRICK_CELLS_A_3D 5
#endif
#ifndef TLSPH_BRICK_CELLS_B_3D
#define TLSPH_BRICK_CELLS_B_3D 3
#endif
    // Pass B's short bricks stage more halo per own particle: measured faster on a 1.26M-particle
    // body, slower on a 40M-particle one, where pass B's halo re-reads already reach HBM (2.5x its
    // algorithmic bytes), so bodies above 8M particles (TLSPH_PASSB_LONG_BRICK_N in the environment
    // at body creation overrides the threshold) keep 4 cells.  Those bodies take 4-cell bricks for
    // pass A too (1.6 % faster per step on the 40M-particle body than 5 cells), so both passes share
    // one slot array.
    int64_t long_brick_n = 8000000;
    if (const char *e = getenv("TLSPH_PASSB_LONG_BRICK_N")) {
        char *end = nullptr;
        const long long v = strtoll(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0) long_brick_n = v;
    }
    const int zbb3 = db.n > long_brick_n ? 4 : TLSPH_BRICK_CELLS_B_3D;
    const int zba3 = db.n > long_brick_n ? 4 : TLSPH_BRICK_CELLS_A_3D;
    int ha = 0, hb = 0;
    const int zba = pick(D == 3 ? (precision == 32 ? zba3 : 2) : 8, lds_a, ha);
    const int zbb = pick(D == 3 ? (precision == 32 ? zbb3 : 2) : 8, lds_b, hb);
    db.ga = geom(zba);
    db.halo_a = ha;
    db.gb = geom(zbb);
    db.halo_b = hb;
    db.gd = geom(1);
    // 3D bodies above 8M particles take their pair-pass bricks in tiles of 4 x 4 columns x 16
    // bricks, so that the bricks in flight on one XCD share one L2-sized neighbourhood; in column
    // order a column's halo comes back from HBM when the next row of columns comes round.  On the
    // 40M-particle column, FP32: 22.13-22.19 ms per step against 22.90 in column order (4 x 4 x 8:
    // 22.21, 6 x 6 x 16: 22.14, 4 x 4 x 32: 22.22, 2 x 2 x 16: 22.38, 4 x 4 x 4: 22.51, 8 x 8 x 4:
    // 22.62); FP64: 54.4 against 55.3.  On the 1.26M-particle cantilever tiles are 1 % slower.
    // TLSPH_BRICK_TILE_N (threshold) and TLSPH_BRICK_TILE ("0": column order, "X,Y,Z": the tile)
    // in the environment at body creation override the choice.
    int64_t tile_n = long_brick_n;
    if (const char *e = getenv("TLSPH_BRICK_TILE_N")) {
        char *end = nullptr;
        const long long v = strtoll(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0) tile_n = v;
    }
    if (D == 3 && db.n > tile_n && brick_count(db.ga) < (1ll << 31) && brick_count(db.gb) < (1ll << 31)) {
        int t[3] = {4, 4, 16};
        if (const char *e = getenv("TLSPH_BRICK_TILE")) {
            int a = 0, b = 0, c = 0;
            if (sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0) {
                t[0] = a;
                t[1] = b;
                t[2] = c;
            } else {
                t[0] = t[1] = t[2] = 0;
            }
        }
        for (int k = 0; k < 3; ++k) db.ga.tile[k] = db.gb.tile[k] = t[k];
    }
    if (lds_a(zba, ha) > 64 * 1024 || lds_b(zbb, hb) > 64 * 1024 || ha > 65535 || hb > 65535) {
        snprintf(errmsg, errlen, "a cell neighbourhood holds %d particles, too many for the LDS tiles of this build",
                 std::max(ha, hb));
        return -8;
    }
    const int64_t nnz = db.nnz > 0 ? db.nnz : 1;
    const bool shared = zbb == zba;
    const int64_t nba = brick_count(db.ga), nbb = brick_count(db.gb);
    // pass A / B slot arrays end with kSlotPad padding entries: the row prologue of those passes
    // loads a fixed number of entries per row (kPre, fewer than kSlotPad) without clamping them
    db.hslot_a = (uint16_t *)A.get(sizeof(uint16_t) * (nnz + kSlotPad));
    db.dslot = (uint16_t *)A.get(sizeof(uint16_t) * nnz);
    db.brick_lmax_a = (int32_t *)A.get(sizeof(int32_t) * (nba > 0 ? nba : 1));
    db.hslot_b = shared ? db.hslot_a : (uint16_t *)A.get(sizeof(uint16_t) * (nnz + kSlotPad));
    db.brick_lmax_b = shared ? db.brick_lmax_a : (int32_t *)A.get(sizeof(int32_t) * (nbb > 0 ? nbb : 1));
    if (!db.hslot_a || !db.dslot || !db.brick_lmax_a || !db.hslot_b || !db.brick_lmax_b) {
        snprintf(errmsg, errlen, "device allocation of the halo-slot arrays failed");
        return -2;
    }
    auto lmax_of = [&](const BrickGeom &g, int64_t nb, int32_t *out) {
        if (nb <= 0) return;
        if (D == 2)
            hipLaunchKernelGGL(k_brick_lmax<2>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, db.row_ptr, out);
        else
            hipLaunchKernelGGL(k_brick_lmax<3>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, db.row_ptr, out);
    };
    auto slots_of = [&](const BrickGeom &g, const uint8_t *cl, uint16_t *out) {
        if (D == 2)
            hipLaunchKernelGGL(k_slots<2>, dim3(nblk(db.n)), dim3(256), 0, s, g, db.cell_start, cell_of, db.row_ptr,
                               db.col, db.n, cl, out, flags);
        else
            hipLaunchKernelGGL(k_slots<3>, dim3(nblk(db.n)), dim3(256), 0, s, g, db.cell_start, cell_of, db.row_ptr,
                               db.col, db.n, cl, out, flags);
    };
    lmax_of(db.ga, nba, db.brick_lmax_a);
    if (!shared) lmax_of(db.gb, nbb, db.brick_lmax_b);
    (void)hipMemsetAsync(flags, 0, sizeof(int), s);
    slots_of(db.ga, nullptr, db.hslot_a);
    if (!shared) slots_of(db.gb, nullptr, db.hslot_b);
    slots_of(db.gd, db.clamped, db.dslot);
    int bad = 0;
    (void)hipMemcpyAsync(&bad, flags, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error while building halo slots");
        return -7;
    }
    if (bad) {
        snprintf(errmsg, errlen, "a neighbour lies outside the adjacent cells");
        return -4;
    }
    // Compact pass-B neighbourhoods for bodies above TLSPH_BRICK_COMPACT_N particles (default 1M): pass
    // B's LDS tile then holds only the slots its rows read, and more of its bricks fit on a CU (it is
    // bound by the bricks in flight per CU: its launch takes 8.6 instead of 9.6 ms on the 40M-particle
    // column, 963 instead of 1024 us on a 4.2M-particle block, 277 instead of 285 us on a 1.26M-particle
    // cantilever).  Where both passes share one slot array pass B gets its own copy; pass A, VALU-bound,
    // keeps the full layout (compact it ran 3 % slower).  The server's small bodies keep the full one.
    int64_t compact_n = 1000000;
    if (const char *e = getenv("TLSPH_BRICK_COMPACT_N")) {
        char *end = nullptr;
        const long long v = strtoll(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0) compact_n = v;
    }
    if (db.n > compact_n && db.halo_b <= 2048 && nbb > 0) {
        const int words = (db.halo_b + 63) / 64;
        db.cmap = (CMapWord *)A.get(sizeof(CMapWord) * (size_t)words * (size_t)nbb);
        if (!db.cmap) {
            snprintf(errmsg, errlen, "device allocation of the compact pass-B maps failed");
            return -2;
        }
        if (shared) {   // pass B's own copy of the slots, compacted below
            uint16_t *hb = (uint16_t *)A.get(sizeof(uint16_t) * (nnz + kSlotPad));
            if (!hb) {
                snprintf(errmsg, errlen, "device allocation of the compact pass-B slots failed");
                return -2;
            }
            (void)hipMemcpyAsync(hb, db.hslot_a, sizeof(uint16_t) * (nnz + kSlotPad), hipMemcpyDeviceToDevice, s);
            db.hslot_b = hb;
        }
        (void)hipMemsetAsync(flags, 0, sizeof(int), s);
        if (D == 2)
            hipLaunchKernelGGL(k_compact_brick<2>, dim3((unsigned)nbb), dim3(256), 0, s, db.gb, db.cell_start,
                               db.row_ptr, db.hslot_b, words, db.cmap, flags);
        else
            hipLaunchKernelGGL(k_compact_brick<3>, dim3((unsigned)nbb), dim3(256), 0, s, db.gb, db.cell_start,
                               db.row_ptr, db.hslot_b, words, db.cmap, flags);
        int h = 0;
        if (hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            snprintf(errmsg, errlen, "HIP error while compacting the pass-B neighbourhoods");
            return -7;
        }
        db.gb.cmap = db.cmap;
        db.gb.cmap_words = words;
        db.halo_b = h;
    }
    // run descriptors of both pair passes (one array where they share a geometry)
    const int rw = D == 3 ? run_words<3>() : run_words<2>();
    db.runs_a = (int32_t *)A.get(sizeof(int32_t) * (size_t)rw * (size_t)(nba > 0 ? nba : 1));
    db.runs_b = shared ? db.runs_a : (int32_t *)A.get(sizeof(int32_t) * (size_t)rw * (size_t)(nbb > 0 ? nbb : 1));
    if (!db.runs_a || !db.runs_b) {
        snprintf(errmsg, errlen, "device allocation of the brick run descriptors failed");
        return -2;
    }
    auto runs_of = [&](const BrickGeom &g, int64_t nb, int32_t *out) {
        if (nb <= 0) return;
        if (D == 2)
            hipLaunchKernelGGL(k_brick_runs<2>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, out);
        else
            hipLaunchKernelGGL(k_brick_runs<3>, dim3(nblk(nb)), dim3(256), 0, s, g, db.cell_start, out);
    };
    runs_of(db.ga, nba, db.runs_a);
    if (!shared) runs_of(db.gb, nbb, db.runs_b);
    if (hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error while building the brick run descriptors");
        return -7;
    }
    db.ga.runs = db.runs_a;
    db.gb.runs = db.runs_b;
    return 0;
}

// The order in which the damping launches take each colour's cells: the colour's cells in the
// enumeration cz fastest, then cy, then cx, then, within windows of kOrderWindow consecutive cells
// (neighbouring cells, so one wavefront's staged neighbourhoods stay close in memory), sorted by
// particle count, most first.  A wavefront serves four consecutive cells and runs as long as its
// longest chain, so similar counts in a wavefront waste fewer issue slots.  Colours follow one
// another, colour c starting at colour_offset(nc, dim, c).
constexpr int kOrderWindow = 64;

int build_damp_order(DeviceBody &db, const Alloc &A, hipStream_t s, char *errmsg, size_t errlen)
{
    const int D = db.dim;
    const int64_t ncell = db.ncell;
    std::vector<int32_t> cs((size_t)ncell + 1);
    if (hipMemcpyAsync(cs.data(), db.cell_start, sizeof(int32_t) * (ncell + 1), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error during setup (damping order)");
        return -7;
    }
    std::vector<int32_t> order;
    order.reserve((size_t)ncell);
    for (int c = 0; c < (D == 3 ? 27 : 9); ++c) {
        int kx, ky, kz, nby, nbz, ncells;
        colour_axes(D, c, kx, ky, kz);
        colour_cells(db.nc, D, kx, ky, kz, nby, nbz, ncells);
        const size_t first = order.size();
        for (int ci = 0; ci < ncells; ++ci) {
            int b = ci, bz = 0;
            if (D == 3) {
                bz = b % nbz;
                b /= nbz;
            }
            const int cx = kx + 3 * (b / nby), cy = ky + 3 * (b % nby), cz = kz + 3 * bz;
            order.push_back(D == 3 ? (cx * db.nc[1] + cy) * db.nc[2] + cz : cx * db.nc[1] + cy);
        }
        for (size_t w = first; w < order.size(); w += kOrderWindow) {
            const size_t e = std::min(order.size(), w + kOrderWindow);
            std::stable_sort(order.begin() + w, order.begin() + e,
                             [&](int32_t a, int32_t b) { return cs[a + 1] - cs[a] > cs[b + 1] - cs[b]; });
        }
    }
    if ((int64_t)order.size() != ncell) {
        snprintf(errmsg, errlen, "damping order covers %zu of %lld cells", order.size(), (long long)ncell);
        return -1;
    }
    db.dorder = (int32_t *)A.get(sizeof(int32_t) * (ncell > 0 ? ncell : 1));
    if (!db.dorder) {
        snprintf(errmsg, errlen, "device allocation of the damping order failed");
        return -2;
    }
    if (hipMemcpyAsync(db.dorder, order.data(), sizeof(int32_t) * ncell, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error during setup (damping order upload)");
        return -7;
    }
    return 0;
}

// Compact damping neighbourhoods (k_compact) for bodies above TLSPH_DAMP_COMPACT_N particles
// (default 2M; the environment at body creation overrides it) whose neighbourhoods hold at most 1024
// particles: a cell's LDS then holds about half as many slots, and twice as many cells fit on a CU
// (the colour launches of large bodies are bound by the chains in flight per CU).  Per colour launch:
// 560 -> 487 us on a 40M-particle column, 97.6 -> 80.6 us on a 4.2M-particle block, but 42.4 -> 47.2
// us on a 1.26M-particle cantilever, whose launches hold fewer wavefronts than the chip has SIMDs
// (the ranking costs issue slots there and buys nothing), so smaller bodies keep the full layout.
int build_damp_compact(DeviceBody &db, const Alloc &A, int *flags, hipStream_t s, char *errmsg, size_t errlen)
{
    db.halo_damp = db.halo_max;
    int64_t min_n = 2000000;
    if (const char *e = getenv("TLSPH_DAMP_COMPACT_N")) {
        char *end = nullptr;
        const long long v = strtoll(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0) min_n = v;
    }
    if (db.n <= min_n || db.ncell <= 0 || db.halo_max > 1024) return 0;
    db.dtouch = (uint64_t *)A.get(sizeof(uint64_t) * 16 * (size_t)db.ncell);
    db.downr = (int32_t *)A.get(sizeof(int32_t) * (size_t)db.ncell);
    if (!db.dtouch || !db.downr) {
        snprintf(errmsg, errlen, "device allocation of the compact damping neighbourhoods failed");
        return -2;
    }
    (void)hipMemsetAsync(flags, 0, sizeof(int), s);
    const dim3 grid((unsigned)((db.ncell + 15) / 16));
    if (db.dim == 2)
        hipLaunchKernelGGL(k_compact<2>, grid, dim3(256), 0, s, db.gd, db.cell_start, db.row_ptr, db.dslot, db.ncell,
                           db.dtouch, db.downr, flags);
    else
        hipLaunchKernelGGL(k_compact<3>, grid, dim3(256), 0, s, db.gd, db.cell_start, db.row_ptr, db.dslot, db.ncell,
                           db.dtouch, db.downr, flags);
    int h = 0;
    if (hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error while compacting the damping neighbourhoods");
        return -7;
    }
    db.halo_damp = h;
    return 0;
}

}  // namespace

int setup_topology(DeviceBody &db, int precision, const double *X0_in, const uint8_t *cl_in, const double xmin[3],
                   double rc, double rc2, double h, double vol, int32_t *perm, void *(*alloc)(size_t, void *),
                   void (*dfree)(void *, void *), void *actx, hipStream_t s, char *errmsg, size_t errlen)
{
    Alloc A{alloc, dfree, actx};
    const int64_t n = db.n;
    const int D = db.dim;
    Grid g;
    g.dim = D;
    for (int k = 0; k < 3; ++k) { g.nc[k] = db.nc[k]; g.xmin[k] = xmin[k]; }
    g.rc = rc;
    g.rc2 = rc2;
    const int64_t ncell = db.ncell;

    int status = 0;
    int32_t *cell_in = (int32_t *)A.get(sizeof(int32_t) * n);
    int32_t *count = (int32_t *)A.get(sizeof(int32_t) * (ncell + 1));
    int32_t *fill = (int32_t *)A.get(sizeof(int32_t) * ncell);
    int32_t *cell_of = (int32_t *)A.get(sizeof(int32_t) * n);
    int64_t *rcnt = (int64_t *)A.get(sizeof(int64_t) * (n + 1));
    int *flags = (int *)A.get(sizeof(int) * 4);
    int hflags[4] = {0, 0, 0, 0};
    if (!cell_in || !count || !fill || !cell_of || !rcnt || !flags) {
        snprintf(errmsg, errlen, "device allocation failed during setup");
        status = -2;
        goto done;
    }
    (void)hipMemsetAsync(count, 0, sizeof(int32_t) * (ncell + 1), s);
    (void)hipMemsetAsync(fill, 0, sizeof(int32_t) * ncell, s);
    (void)hipMemsetAsync(flags, 0, sizeof(int) * 4, s);
    (void)hipMemsetAsync(rcnt, 0, sizeof(int64_t) * (n + 1), s);

    hipLaunchKernelGGL(k_bin, dim3(nblk(n)), dim3(256), 0, s, g, X0_in, n, cell_in, count);
    if (!scan_exclusive<int32_t, int32_t>(count, db.cell_start, ncell + 1, A, s)) { status = -2; goto done; }
    hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(256), 0, s, cell_in, n, db.cell_start, fill, perm);
    hipLaunchKernelGGL(k_sort_cells, dim3(nblk(ncell)), dim3(256), 0, s, db.cell_start, ncell, perm);
    hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(256), 0, s, perm, n, D, X0_in, cl_in, db.X, db.clamped);
    hipLaunchKernelGGL(k_cell_of, dim3(nblk(ncell)), dim3(256), 0, s, db.cell_start, ncell, cell_of);
    hipLaunchKernelGGL(k_halo_max, dim3(nblk(ncell)), dim3(256), 0, s, g, db.cell_start, ncell, flags + 2);
    if (D == 2)
        hipLaunchKernelGGL(k_row_count<2>, dim3(nblk(n)), dim3(256), 0, s, g, db.X, n, db.cell_start, cell_of, rcnt,
                           flags + 1);
    else
        hipLaunchKernelGGL(k_row_count<3>, dim3(nblk(n)), dim3(256), 0, s, g, db.X, n, db.cell_start, cell_of, rcnt,
                           flags + 1);
    if (!scan_exclusive<int64_t, int64_t>(rcnt, db.row_ptr, n + 1, A, s)) { status = -2; goto done; }
    if (hipMemcpyAsync(&db.nnz, db.row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hflags, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error during setup: %s", hipGetErrorString(hipGetLastError()));
        status = -7;
        goto done;
    }
    db.row_max = hflags[1];
    db.halo_max = hflags[2];
    if (db.nnz >= ((int64_t)1 << 40)) {
        snprintf(errmsg, errlen, "neighbour list too large (%lld entries)", (long long)db.nnz);
        status = -8;
        goto done;
    }
    db.col = (int32_t *)A.get(sizeof(int32_t) * (db.nnz > 0 ? db.nnz : 1));
    if (!db.col) {
        snprintf(errmsg, errlen, "device allocation of %lld neighbour entries failed", (long long)db.nnz);
        status = -2;
        goto done;
    }
    if (D == 2)
        hipLaunchKernelGGL(k_row_fill<2>, dim3(nblk(n)), dim3(256), 0, s, g, db.X, n, db.cell_start, cell_of,
                           db.row_ptr, db.col);
    else
        hipLaunchKernelGGL(k_row_fill<3>, dim3(nblk(n)), dim3(256), 0, s, g, db.X, n, db.cell_start, cell_of,
                           db.row_ptr, db.col);
    {
        const double aD = (D == 2) ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
        if (D == 2 && precision == 32)
            hipLaunchKernelGGL((k_B0<2, float>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h, aD,
                               vol, (float *)db.B0, (float *)db.gradsum, flags);
        else if (D == 2)
            hipLaunchKernelGGL((k_B0<2, double>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h, aD,
                               vol, (double *)db.B0, (double *)db.gradsum, flags);
        else if (precision == 32)
            hipLaunchKernelGGL((k_B0<3, float>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h, aD,
                               vol, (float *)db.B0, (float *)db.gradsum, flags);
        else
            hipLaunchKernelGGL((k_B0<3, double>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h, aD,
                               vol, (double *)db.B0, (double *)db.gradsum, flags);
    }
    if (hipMemcpyAsync(hflags, flags, sizeof(int) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        snprintf(errmsg, errlen, "HIP error during setup: %s", hipGetErrorString(hipGetLastError()));
        status = -7;
        goto done;
    }
    if (hflags[0]) {
        snprintf(errmsg, errlen, "a particle's correction matrix B0 (Eq. 9) is singular");
        status = -3;
        goto done;
    }
    status = build_slots(db, precision, cell_of, flags, A, s, errmsg, errlen);
    if (status == 0) {
        const double aD = (D == 2) ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
        const size_t rsz = precision == 32 ? 4 : 8;
        db.gdamp = A.get(rsz * (db.nnz > 0 ? db.nnz : 1));
        if (!db.gdamp) {
            snprintf(errmsg, errlen, "device allocation of the damping factors failed");
            status = -2;
            goto done;
        }
        if (D == 2 && precision == 32)
            hipLaunchKernelGGL((k_gdamp<2, float>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h,
                               aD, vol, (float *)db.gdamp);
        else if (D == 2)
            hipLaunchKernelGGL((k_gdamp<2, double>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h,
                               aD, vol, (double *)db.gdamp);
        else if (precision == 32)
            hipLaunchKernelGGL((k_gdamp<3, float>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h,
                               aD, vol, (float *)db.gdamp);
        else
            hipLaunchKernelGGL((k_gdamp<3, double>), dim3(nblk(n)), dim3(256), 0, s, db.X, n, db.row_ptr, db.col, h,
                               aD, vol, (double *)db.gdamp);
        (void)hipMemsetAsync(flags, 0, sizeof(int) * 2, s);
        hipLaunchKernelGGL(k_cell_stats, dim3(nblk(ncell)), dim3(256), 0, s, db.cell_start, db.row_ptr, ncell, flags);
        int cs[2] = {0, 0};
        if (hipMemcpyAsync(cs, flags, sizeof(int) * 2, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            snprintf(errmsg, errlen, "HIP error during setup");
            status = -7;
            goto done;
        }
        db.cell_max = cs[0];
        db.cell_pairs_max = cs[1];
        status = build_damp_order(db, A, s, errmsg, errlen);
        if (status == 0) status = build_damp_compact(db, A, flags, s, errmsg, errlen);
    }
done:
    (void)hipStreamSynchronize(s);
    A.put(cell_in);
    A.put(count);
    A.put(fill);
    A.put(cell_of);
    A.put(rcnt);
    A.put(flags);
    return status;
}

}  // namespace tlsph
