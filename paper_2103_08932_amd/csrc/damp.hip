// damp.hip -- the S_d part of a damped step: pairwise implicit viscous damping (Sec. 3.2) swept
// over the splitting cell-linked list (Sec. 3.4).
//
// S_d(dt) = D_1(dt/2) ... D_N(dt/2) D_N(dt/2) ... D_1(dt/2)   (Eq. 25)
// D_i(tau) visits the pairs of row(i) forward, then backward, each visit integrating tau / 2
// (Eq. 37) with the closed-form two-body implicit solve of Eq. 39 (equal masses m):
//     B = eta_t (dt / 4) 2 V^2 (dW/dr) / r
//     free-free:  v_i += c (v_i - v_j),  v_j -= c (v_i - v_j),  c = B / (m - 2 B)
//     j clamped:  v_i += B (v_i - v_j) / (m - B);   i clamped:  v_j -= B (v_i - v_j) / (m - B)
// The particle order is: colour blocks 0..K-1, all cells of a block (they never touch the same
// particles, so they run in parallel), particles of a cell ascending; then the exact reverse.
//
// One launch per colour block.  A 64-lane wavefront serves four cells of the block, 16 lanes (one
// DPP row) per cell.  The velocities of each cell's 3^dim-cell neighbourhood are staged in LDS;
// the particles of a cell are then processed one after the other.  Along a row the velocity of i
// follows an affine recurrence
//     v_i <- (1 + c_k) v_i - c_k v_j(k)
// (every j appears once in a row, so v_j(k) is its value when the row starts), so the row is a
// composition of affine maps: each lane composes its P consecutive pairs, a DPP scan inside the
// 16-lane row composes the lanes (row_shr for the forward row, row_shl for the backward row), and
// every lane then knows v_i just before its pairs and updates its v_j in registers.  The next
// particle's row (slots, clamp classes, coefficients) is loaded from global memory while the
// current one is processed.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "bricks.hpp"
#include "internal.hpp"

namespace tlsph {
namespace {

constexpr int kWave = 64;
constexpr int kSeg = 16;                 // lanes per cell (one DPP row)
#ifndef TLSPH_DAMP_PREFETCH
#define TLSPH_DAMP_PREFETCH 2
#endif
constexpr int kPrefetch = TLSPH_DAMP_PREFETCH;   // rows in flight ahead of the particle being processed
constexpr int kCellsPerWave = kWave / kSeg;

// DPP lane moves (GFX9 data-parallel primitives).  `old` is returned in lanes without a source.
template <int CTRL>
__device__ __forceinline__ float dpp(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double old, double src)
{
    const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(v & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row shifts inside each 16-lane row: row_shr:k = 0x110 + k (from lane - k), row_shl:k = 0x100 + k.
template <int K> struct ShR { static constexpr int C = 0x110 + K; };
template <int K> struct ShL { static constexpr int C = 0x100 + K; };

// Combine this lane's map (a, b) with the map fetched from another lane of the row (identity where
// there is none); the fetched map is applied first:  x -> a (ap x + bp) + b.
template <int CTRL, typename R, int D>
__device__ __forceinline__ void scan_step(R &a, R (&b)[D])
{
    const R ap = dpp<CTRL>(R(1), a);
    R bp[D];
#pragma unroll
    for (int k = 0; k < D; ++k) bp[k] = dpp<CTRL>(R(0), b[k]);
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = a * bp[k] + b[k];
    a = a * ap;
}

// 1 / x: the hardware reciprocal in FP32 (1 ulp), IEEE division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

struct DampArgs {
    void *v;
    const int64_t *row_ptr;
    const uint16_t *dslot;
    const void *gdamp;  // per CSR entry: 2 V^2 (dW/dr) / r
    const int32_t *cell_start;
    const DevState *st;
    int64_t n;
    int64_t nnz;
    BrickGeom g;        // single-cell bricks
    int hcap;           // LDS capacity in particles per cell
    double mass;
    double eta_t;
};

// Row data of one particle for this lane: P consecutive row entries from position lane * P, as
// loaded (slot with clamp class, damping factor); they are turned into pair coefficients only
// when the row is processed, so the loads of the next row overlap the current one.
template <typename R, int P>
struct RowRaw {
    int L;              // row length (entries at positions >= L are not pairs)
    int raw[P];         // slot | class << 14
    R g[P];             // 2 V^2 (dW/dr) / r
};

// Loads are unconditional (offsets clamped into the cell's entries [0, E), E >= 1) so that no
// select or branch waits on them.  Offsets are relative to the cell's first CSR entry.
template <typename R, int P>
__device__ __forceinline__ void load_row(RowRaw<R, P> &rr, int e0, int L, int sl, int elast,
                                         const uint16_t *__restrict__ dslot, const R *__restrict__ gd)
{
    rr.L = L;
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const int e = min(e0 + sl * P + t, elast);
        rr.raw[t] = dslot[e];
        rr.g[t] = gd[e];
    }
}

template <typename R, int P>
struct RowRegs {
    int slot[P];        // neighbourhood slot of j; entries past the row point at the dummy slot
    R cI[P], dJ[P];     // v_i += cI (v_i - v_j);  v_j -= dJ (v_i - v_j)
};

// Pair coefficient of Eq. 39 with B = eta_t (dt / 4) g_ij and equal masses m: free-free
// c = B / (m - 2 B), one end clamped c = B / (m - B), both clamped 0.  Entries past the row get
// zero coefficients and the dummy slot, so the row code runs without branches.
template <typename R, int P>
__device__ __forceinline__ void decode_row(RowRegs<R, P> &rr, const RowRaw<R, P> &in, int sl, R bscale, R m, int dummy)
{
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const bool ok = sl * P + t < in.L;
        const int raw = in.raw[t];
        const int cls = (raw >> 14) & 3;   // bit 1: i clamped, bit 0: j clamped
        const R B = bscale * in.g[t];
        R c = B * recip(m - (cls == 0 ? R(2) : R(1)) * B);
        c = (ok && cls != 3) ? c : R(0);
        rr.slot[t] = ok ? (raw & 0x3fff) : dummy;
        rr.cI[t] = (cls & 2) ? R(0) : c;
        rr.dJ[t] = (cls & 1) ? R(0) : c;
    }
}

// D_i(dt/2) on the 16-lane row of this cell: the row forward, then the row backward (Eq. 37).
template <typename R, int D, int P>
__device__ __forceinline__ void damp_particle(R (&vi)[D], const RowRegs<R, P> &rr, R *__restrict__ sv, int HC)
{
    R vj[P][D];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
        for (int k = 0; k < D; ++k) vj[t][k] = sv[k * HC + rr.slot[t]];
    // ---- forward: lanes ascending, pairs of a lane ascending ----
    {
        R a = R(1), b[D];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = R(0);
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const R at = R(1) + rr.cI[t];
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = at * b[k] - rr.cI[t] * vj[t][k];
            a = at * a;
        }
        scan_step<ShR<1>::C>(a, b);
        scan_step<ShR<2>::C>(a, b);
        scan_step<ShR<4>::C>(a, b);
        scan_step<ShR<8>::C>(a, b);
        // map of the earlier lanes of the row, applied to v_i
        const R ax = dpp<ShR<1>::C>(R(1), a);
        R x[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = ax * vi[k] + dpp<ShR<1>::C>(R(0), b[k]);
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R w = x[k] - vj[t][k];
                x[k] = x[k] + rr.cI[t] * w;
                vj[t][k] = vj[t][k] - rr.dJ[t] * w;
            }
        // whole-row map sits in lane 15 of the row
        const R aL = __shfl(a, kSeg - 1, kSeg);
#pragma unroll
        for (int k = 0; k < D; ++k) vi[k] = aL * vi[k] + __shfl(b[k], kSeg - 1, kSeg);
    }
    // ---- backward: lanes descending, pairs of a lane descending ----
    {
        R a = R(1), b[D];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = R(0);
#pragma unroll
        for (int t = P - 1; t >= 0; --t) {
            const R at = R(1) + rr.cI[t];
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = at * b[k] - rr.cI[t] * vj[t][k];
            a = at * a;
        }
        scan_step<ShL<1>::C>(a, b);
        scan_step<ShL<2>::C>(a, b);
        scan_step<ShL<4>::C>(a, b);
        scan_step<ShL<8>::C>(a, b);
        const R ax = dpp<ShL<1>::C>(R(1), a);
        R x[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = ax * vi[k] + dpp<ShL<1>::C>(R(0), b[k]);
#pragma unroll
        for (int t = P - 1; t >= 0; --t)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R w = x[k] - vj[t][k];
                x[k] = x[k] + rr.cI[t] * w;
                vj[t][k] = vj[t][k] - rr.dJ[t] * w;
            }
        const R a0 = __shfl(a, 0, kSeg);
#pragma unroll
        for (int k = 0; k < D; ++k) vi[k] = a0 * vi[k] + __shfl(b[k], 0, kSeg);
    }
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
        for (int k = 0; k < D; ++k) sv[k * HC + rr.slot[t]] = vj[t][k];
}

// Workgroup `blk` of one colour launch over one body: cells blk * 4 .. blk * 4 + 3 of the colour
// block (cell index of the block: cz fastest, then cy, then cx).
template <typename R, int D, int P, bool FWD>
__device__ __forceinline__ void damp_cells(const DampArgs &A, int kx, int ky, int kz, int nby, int nbz, int ncells,
                                           int64_t blk)
{
    const int lane = threadIdx.x;
    const int seg = lane / kSeg, sl = lane % kSeg;
    const int64_t n = A.n;
    const int ci = (int)blk * kCellsPerWave + seg;
    BrickRuns<D> BR;
    int p0 = 0, cnt = 0;
    if (ci < ncells) {
        int b = ci, bz = 0;
        if constexpr (D == 3) {
            bz = b % nbz;
            b /= nbz;
        }
        const int by = b % nby, bx = b / nby;
        const int cx = kx + 3 * bx, cy = ky + 3 * by, cz = (D == 3) ? kz + 3 * bz : 0;
        if constexpr (D == 3)
            brick_runs<D>(A.g, A.cell_start, cx, cy, cz, BR);
        else
            brick_runs<D>(A.g, A.cell_start, cx, 0, cy, BR);
        p0 = BR.own0;
        cnt = BR.own1 - BR.own0;
    } else {
#pragma unroll
        for (int r = 0; r < BrickRuns<D>::NR; ++r) BR.start[r] = BR.len[r] = BR.off[r] = 0;
        BR.total = 0;
        BR.own0 = BR.own1 = 0;
    }
    // particles in the busiest cell of the wave
    int maxcnt = cnt;
    maxcnt = max(maxcnt, __shfl_xor(maxcnt, 16));
    maxcnt = max(maxcnt, __shfl_xor(maxcnt, 32));
    if (maxcnt == 0) return;

    // LDS: per segment [D][HC] velocities; slot HC - 1 is a dummy that absorbs the updates of
    // row entries past the end of a row
    extern __shared__ double smem[];
    const int HC = A.hcap + 1;
    const int dummy = HC - 1;
    R *sv = reinterpret_cast<R *>(smem) + seg * D * HC;
    R *vg = reinterpret_cast<R *>(A.v);
    const R *gd = reinterpret_cast<const R *>(A.gdamp);
    // staging: every load of a lane is issued before its LDS stores
    constexpr int U = sizeof(R) == 4 ? 16 : 8;
    for (int base = 0; base < BR.total; base += kSeg * U) {
        // loads are unconditional (padding lanes read particle 0) so none waits at a branch
        R vv[U][D];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kSeg + sl;
            const int64_t j = idx < BR.total ? halo_particle<D>(BR, idx) : 0;
#pragma unroll
            for (int k = 0; k < D; ++k) vv[w][k] = vg[k * n + j];
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kSeg + sl;
            if (idx < BR.total) {
#pragma unroll
                for (int k = 0; k < D; ++k) sv[k * HC + idx] = vv[w][k];
            }
        }
    }
    // row offsets of the cell's particles relative to its first CSR entry: entry q in lane
    // q % 16 of register q / 16
    const int64_t E0 = A.row_ptr[p0];
    const int rlo = sl <= cnt ? (int)(A.row_ptr[p0 + sl] - E0) : 0;
    const int rhi = sl + kSeg <= cnt ? (int)(A.row_ptr[p0 + kSeg + sl] - E0) : 0;
    auto row_at = [&](int q) -> int {
        const int w = q < kSeg ? rlo : rhi;
        return __shfl(w, seg * kSeg + (q % kSeg));
    };
    const int elast = max(__shfl(rlo, seg * kSeg + min(cnt, kSeg - 1)), 1) - 1;
    const int elast_hi = cnt >= kSeg ? __shfl(rhi, seg * kSeg + (cnt - kSeg)) - 1 : -1;
    const int emax = max(elast, elast_hi);
    const uint16_t *__restrict__ cds = A.dslot + E0;
    const R *__restrict__ cgd = gd + E0;
    const R bscale = (R)(A.eta_t * 0.25 * A.st->dt);
    const R m = (R)A.mass;
    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    // the dummy slot holds zeros: entries past a row read it with zero coefficients
    if (sl == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) sv[k * HC + dummy] = R(0);
    }
    // one wavefront per workgroup: its LDS operations complete in issue order, so the loop needs
    // only a compiler-level barrier (a workgroup barrier would also drain the prefetch loads)
    __builtin_amdgcn_wave_barrier();

    // rows are loaded kPrefetch particles ahead (a ring of register buffers, indexed statically by
    // unrolling), so each row's global-memory latency overlaps the processing of the particles
    // before it; particles past the cell's count load a clamped, empty row
    auto fetch = [&](RowRaw<R, P> &rr, int q) {
        const bool act = q < cnt;
        const int qs = act ? (FWD ? q : cnt - 1 - q) : 0;
        const int e0 = row_at(qs), e1 = row_at(qs + 1);
        load_row<R, P>(rr, e0, act ? e1 - e0 : 0, sl, emax, cds, cgd);
    };
    RowRaw<R, P> buf[kPrefetch];
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) fetch(buf[k], k);
    for (int q0 = 0; q0 < maxcnt; q0 += kPrefetch) {
#pragma unroll
        for (int k = 0; k < kPrefetch; ++k) {
            const int q = q0 + k;
            if (q >= maxcnt) break;   // uniform over the wave
            RowRegs<R, P> rr;
            decode_row<R, P>(rr, buf[k], sl, bscale, m, dummy);
            fetch(buf[k], q + kPrefetch);
            const bool active = q < cnt;
            const int qi = FWD ? q : cnt - 1 - q;
            const int islot = active ? p0 + qi + cbase : dummy;
            R vi[D];
#pragma unroll
            for (int d = 0; d < D; ++d) vi[d] = sv[d * HC + islot];
            damp_particle<R, D, P>(vi, rr, sv, HC);
            if (sl == 0) {
#pragma unroll
                for (int d = 0; d < D; ++d) sv[d * HC + islot] = vi[d];
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (int idx = sl; idx < BR.total; idx += kSeg) {
        const int64_t j = halo_particle<D>(BR, idx);
#pragma unroll
        for (int k = 0; k < D; ++k) vg[k * n + j] = sv[k * HC + idx];
    }
}

__host__ __device__ inline int count_mod3(int ncell, int k) { return ncell > k ? (ncell - k + 2) / 3 : 0; }

template <typename R, int D, int P, bool FWD>
__global__ __launch_bounds__(kWave) void k_damp(DampArgs A, int kx, int ky, int kz, int nby, int nbz, int ncells)
{
    if (A.st->done) return;
    // blocks are mapped so that each XCD works on one contiguous slab of cells in every colour launch
    const int64_t blk = xcd_block(blockIdx.x, (ncells + kCellsPerWave - 1) / kCellsPerWave);
    if (blk < 0) return;
    damp_cells<R, D, P, FWD>(A, kx, ky, kz, nby, nbz, ncells, blk);
}

// Colour blocks of one body: cells per axis of colour (kx, ky, kz).
__host__ __device__ inline void colour_cells(const int32_t (&nc)[3], int dim, int kx, int ky, int kz, int &nby,
                                             int &nbz, int &ncells)
{
    const int nbx = count_mod3(nc[0], kx);
    nby = count_mod3(nc[1], ky);
    nbz = dim == 3 ? count_mod3(nc[2], kz) : 1;
    ncells = nbx * nby * nbz;
}

template <typename R, int D, int P, bool FWD>
__global__ __launch_bounds__(kWave) void k_damp_batch(const Inst *__restrict__ I, BatchMap M, int kx, int ky, int kz)
{
    const int64_t w = xcd_block(blockIdx.x, M.start[M.count]);
    if (w < 0) return;
    const int k = batch_find(M, (int)w);
    const Inst *in = I + M.inst[k];
    if (in->st->done) return;
    DampArgs A;
    A.v = in->v;
    A.row_ptr = in->row_ptr;
    A.dslot = in->dslot;
    A.gdamp = in->gdamp;
    A.cell_start = in->cell_start;
    A.st = in->st;
    A.n = in->P.n;
    A.nnz = 1;
    A.g = in->gd;
    A.hcap = in->halo_max;
    A.mass = in->P.mass;
    A.eta_t = in->eta_t;
    int nby, nbz, ncells;
    colour_cells(in->nc, D, kx, ky, kz, nby, nbz, ncells);
    damp_cells<R, D, P, FWD>(A, kx, ky, kz, nby, nbz, ncells, w - M.start[k]);
}

}  // namespace

int damp_pairs_per_lane(int row_max) { return (row_max + kSeg - 1) / kSeg; }

// Colour k -> residues of the cell coordinates: 3D k = 9 (cx mod 3) + 3 (cy mod 3) + cz mod 3,
// 2D k = 3 (cx mod 3) + cy mod 3 (Sec. 3.4).
static void colour_axes(int dim, int colour, int &kx, int &ky, int &kz)
{
    if (dim == 3) {
        kx = colour / 9;
        ky = (colour / 3) % 3;
        kz = colour % 3;
    } else {
        kx = colour / 3;
        ky = colour % 3;
        kz = 0;
    }
}

size_t damp_lds_bytes(int dim, int precision, int hcap, int /*ecap*/)
{
    const size_t rs = precision == 32 ? 4 : 8;
    return (size_t)kCellsPerWave * (hcap + 1) * dim * rs + 16;
}

template <typename R, int D, int P>
static void launch_pb(dim3 g, size_t lds, hipStream_t s, const Inst *I, const BatchMap &M, bool fwd, int kx, int ky,
                      int kz)
{
    if (fwd)
        hipLaunchKernelGGL((k_damp_batch<R, D, P, true>), g, dim3(kWave), lds, s, I, M, kx, ky, kz);
    else
        hipLaunchKernelGGL((k_damp_batch<R, D, P, false>), g, dim3(kWave), lds, s, I, M, kx, ky, kz);
}

template <typename R, int D>
static void launch_rdb(int P, dim3 g, size_t lds, hipStream_t s, const Inst *I, const BatchMap &M, bool fwd, int kx,
                       int ky, int kz)
{
    if (P <= 2) launch_pb<R, D, 2>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 3) launch_pb<R, D, 3>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 4) launch_pb<R, D, 4>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 5) launch_pb<R, D, 5>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 6) launch_pb<R, D, 6>(g, lds, s, I, M, fwd, kx, ky, kz);
    else launch_pb<R, D, 8>(g, lds, s, I, M, fwd, kx, ky, kz);
}

template <typename R, int D, int P>
static void launch_p(dim3 g, size_t lds, hipStream_t s, const DampArgs &A, bool fwd, int kx, int ky, int kz, int nby,
                     int nbz, int ncells)
{
    if (fwd)
        hipLaunchKernelGGL((k_damp<R, D, P, true>), g, dim3(kWave), lds, s, A, kx, ky, kz, nby, nbz, ncells);
    else
        hipLaunchKernelGGL((k_damp<R, D, P, false>), g, dim3(kWave), lds, s, A, kx, ky, kz, nby, nbz, ncells);
}

template <typename R, int D>
static void launch_rd(int P, dim3 g, size_t lds, hipStream_t s, const DampArgs &A, bool fwd, int kx, int ky, int kz,
                      int nby, int nbz, int ncells)
{
    if (P <= 2) launch_p<R, D, 2>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 3) launch_p<R, D, 3>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 4) launch_p<R, D, 4>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 5) launch_p<R, D, 5>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 6) launch_p<R, D, 6>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else launch_p<R, D, 8>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
}

void launch_damp_colour(const DeviceBody &db, const StepParams &p, int precision, int colour, bool forward,
                        double eta_t, hipStream_t s)
{
    DampArgs A;
    A.v = db.v;
    A.row_ptr = db.row_ptr;
    A.dslot = db.dslot;
    A.gdamp = db.gdamp;
    A.cell_start = db.cell_start;
    A.st = db.st;
    A.n = db.n;
    A.nnz = db.nnz > 0 ? db.nnz : 1;
    A.g = db.gd;
    A.hcap = db.halo_max;
    A.mass = p.mass;
    A.eta_t = eta_t;
    int kx, ky, kz;
    colour_axes(db.dim, colour, kx, ky, kz);
    const int nbx = count_mod3(db.nc[0], kx), nby = count_mod3(db.nc[1], ky);
    const int nbz = db.dim == 3 ? count_mod3(db.nc[2], kz) : 1;
    const int64_t ncells = (int64_t)nbx * nby * nbz;
    if (ncells == 0) return;
    const int64_t blocks = xcd_grid((ncells + kCellsPerWave - 1) / kCellsPerWave);
    const size_t lds = damp_lds_bytes(db.dim, precision, db.halo_max, 0);
    const int P = damp_pairs_per_lane(db.row_max);
    const dim3 g((unsigned)blocks);
    if (precision == 32 && db.dim == 2) launch_rd<float, 2>(P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else if (precision == 32) launch_rd<float, 3>(P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else if (db.dim == 2) launch_rd<double, 2>(P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else launch_rd<double, 3>(P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
}

void launch_damp_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision, int colour,
                       bool forward, hipStream_t s)
{
    if (count <= 0) return;
    int kx, ky, kz;
    colour_axes(dim, colour, kx, ky, kz);
    BatchMap M;
    M.count = count;
    int acc = 0, P = 1;
    size_t lds = 0;
    for (int k = 0; k < count; ++k) {
        const Inst &in = h[slots[k]];
        int nby, nbz, ncells;
        colour_cells(in.nc, dim, kx, ky, kz, nby, nbz, ncells);
        M.inst[k] = slots[k];
        M.start[k] = acc;
        acc += (ncells + kCellsPerWave - 1) / kCellsPerWave;
        P = std::max(P, damp_pairs_per_lane(in.row_max));
        lds = std::max(lds, damp_lds_bytes(dim, precision, in.halo_max, 0));
    }
    M.start[count] = acc;
    if (acc == 0) return;
    const dim3 g((unsigned)xcd_grid(acc));
    if (precision == 32 && dim == 2) launch_rdb<float, 2>(P, g, lds, s, I, M, forward, kx, ky, kz);
    else if (precision == 32) launch_rdb<float, 3>(P, g, lds, s, I, M, forward, kx, ky, kz);
    else if (dim == 2) launch_rdb<double, 2>(P, g, lds, s, I, M, forward, kx, ky, kz);
    else launch_rdb<double, 3>(P, g, lds, s, I, M, forward, kx, ky, kz);
}

}  // namespace tlsph
