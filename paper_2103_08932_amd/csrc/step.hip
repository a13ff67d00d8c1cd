// step.hip -- the S_m part of one relaxation step and the end-of-step reductions.
//
//   pass A  u_h = u + dt/2 v                                 (Sec. 2.3, Eq. 15; free particles)
//           F_i = I + H_i,  H_i = V (sum_j (u_h,j - u_h,i) (x) grad0_i W_ij) B0_i   (Eqs. 2, 9, 14)
//           S (Eq. 4 or Eqs. 7-8), P = F S (Eq. 3), T_i = P_i B0_i
//   pass B  a_i = (V / rho0) sum_j (T_i + T_j) grad0_i W_ij + b_i               (Eqs. 12-13)
//           v_i += dt a_i (free particles)                                       (Eq. 16)
//   pass C  u = u_h + dt/2 v (Eq. 17), clamped u = v = 0, FP64 partials of E_k (Neumaier), max |v|
//   finish  E_k, E_peak, window residual, force residual and dt of the next step (Eq. 18)
//
// Passes A and B run one workgroup per brick (bricks.hpp): the brick's neighbourhood is loaded into
// LDS with coalesced reads, and every CSR entry is a 2-byte slot into that tile.  A group of G
// lanes shares one particle's row (lane l takes entries l, l + G, ...), and the G partial sums are
// combined with cross-lane shuffles.
//
// grad0_i W_ij = (dW/dr) (X_i - X_j) / r = kfac (1 - q/2)^3 (X_i - X_j) with the Wendland C2 kernel
// (kfac = -5 a_D / h^2), so no division by r is needed.  In the FP32 path positions and half-step
// displacements are staged relative to one particle of the brick (the differences are taken in
// FP64 and rounded once), so neighbour differences keep their relative precision.  In the FP64
// path the tile holds the FP64 values themselves.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "bricks.hpp"
#include "devmath.hpp"
#include "internal.hpp"

namespace tlsph {
namespace {

#ifndef TLSPH_TILE_THREADS
#define TLSPH_TILE_THREADS 256
#endif
#ifndef TLSPH_LANES_3D
#define TLSPH_LANES_3D 4
#endif
constexpr int kTile = TLSPH_TILE_THREADS;   // threads per brick workgroup (a multiple of 64)
static_assert(kTile % 64 == 0, "brick workgroups are whole wavefronts");

__device__ __forceinline__ int64_t gid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Lanes per particle row (rows hold ~80 entries in 3D, ~20 in 2D) and the number of row entries
// a row's lanes prefetch into registers before the pair loop (longer rows finish in a tail loop);
// rounds(g) = prefetched entries per lane with g lanes per row.
template <int D> struct Lanes {
    static constexpr int G = (D == 3) ? TLSPH_LANES_3D : 4;
    static constexpr int kPre = (D == 3) ? 96 : 24;
    static constexpr int rounds(int g) { return (kPre + g - 1) / g; }
};
static_assert(Lanes<3>::kPre <= kSlotPad && Lanes<2>::kPre <= kSlotPad, "row prologue loads past the slot arrays");

// The own rows of a brick in batches of kTile / G rows with G lanes each, the last batch with twice
// the lanes (half the rounds) when it has at most kTile / (2 G) rows: a brick of 65-96 rows then
// takes 1.5 batch times instead of 2.  rows(lanes, q0, nq) runs rows q0 .. q0 + nq - 1 with
// lanes::value lanes per row.
template <int G> using lanes_t = std::integral_constant<int, G>;
template <int D, typename F>
__device__ __forceinline__ void row_batches(int np, F &&rows)
{
    constexpr int G = Lanes<D>::G;
    constexpr int NB = kTile / G;
    int q0 = 0;
    for (; np - q0 > NB; q0 += NB) rows(lanes_t<G>(), q0, NB);
    if (np - q0 > NB / 2) rows(lanes_t<G>(), q0, np - q0);
    else if (np > q0) rows(lanes_t<2 * G>(), q0, np - q0);
}

// LDS tile records of WU words per neighbourhood particle:
//   pass A: x[D], u_h[D];   pass B: x[D], T[D*D]
// stored as planes of PV-wide vectors, the last plane as narrow as the words left (word w of record
// s is component w % PV of vector s of plane w / PV; plane p starts at word p * PV * hs).  Neighbour
// records are gathered at random slots; narrow planes spread the records of a wavefront's lanes over
// more LDS banks than whole 24- or 48-byte records would.  Register copies of a record are W words
// (WU rounded up to whole planes); the words past WU hold no value.
#ifndef TLSPH_PLANE_A
#define TLSPH_PLANE_A 4
#endif
#ifndef TLSPH_PLANE_B
#define TLSPH_PLANE_B 4
#endif
template <typename R, int PW32> constexpr int plane_width() { return sizeof(R) == 4 ? PW32 : 2; }
template <typename R, int D> struct TileA {
    static constexpr int PV = plane_width<R, TLSPH_PLANE_A>();
    static constexpr int WU = 2 * D;
    static constexpr int W = (WU + PV - 1) / PV * PV;
};
template <typename R, int D> struct TileB {
    static constexpr int PV = plane_width<R, TLSPH_PLANE_B>();
    static constexpr int WU = D + D * D;
    static constexpr int W = (WU + PV - 1) / PV * PV;
};

template <typename R, int N> using vec_t = R __attribute__((ext_vector_type(N)));

// Record `slot` of a planar tile whose planes hold `hs` vectors each, plane by plane.  Only the
// words in use are read: besides the LDS bytes, a padding word loaded and never used is a dead
// register that the compiler hands to the next load, which must then wait for this one.
template <int P0, typename R, int W, int PV, int WU>
__device__ __forceinline__ void tile_load_planes(const R *__restrict__ tile, int hs, int slot, R (&rec)[W])
{
    if constexpr (P0 * PV < WU) {
        constexpr int NW = (WU - P0 * PV < PV) ? WU - P0 * PV : PV;
        const R *a = tile + (size_t)P0 * PV * hs + (size_t)slot * NW;
        if constexpr (NW == 1) {
            rec[P0 * PV] = *a;
        } else {
            const vec_t<R, NW> v = *reinterpret_cast<const vec_t<R, NW> *>(a);
#pragma unroll
            for (int c = 0; c < NW; ++c) rec[P0 * PV + c] = v[c];
        }
        tile_load_planes<P0 + 1, R, W, PV, WU>(tile, hs, slot, rec);
    }
}
template <int P0, typename R, int W, int PV, int WU>
__device__ __forceinline__ void tile_store_planes(R *__restrict__ tile, int hs, int slot, const R (&rec)[W])
{
    if constexpr (P0 * PV < WU) {
        constexpr int NW = (WU - P0 * PV < PV) ? WU - P0 * PV : PV;
        R *a = tile + (size_t)P0 * PV * hs + (size_t)slot * NW;
        if constexpr (NW == 1) {
            *a = rec[P0 * PV];
        } else {
            vec_t<R, NW> v;
#pragma unroll
            for (int c = 0; c < NW; ++c) v[c] = rec[P0 * PV + c];
            *reinterpret_cast<vec_t<R, NW> *>(a) = v;
        }
        tile_store_planes<P0 + 1, R, W, PV, WU>(tile, hs, slot, rec);
    }
}
template <typename R, int W, int PV, int WU>
__device__ __forceinline__ void tile_load(const R *__restrict__ tile, int hs, int slot, R (&rec)[W])
{
    tile_load_planes<0, R, W, PV, WU>(tile, hs, slot, rec);
}
template <typename R, int W, int PV, int WU>
__device__ __forceinline__ void tile_store(R *__restrict__ tile, int hs, int slot, const R (&rec)[W])
{
    tile_store_planes<0, R, W, PV, WU>(tile, hs, slot, rec);
}

// Fixed-order butterflies over the 64 lanes of a wavefront: maximum, and Neumaier-compensated sum
// of (s, c) pairs (the combination is symmetric, so every lane ends with the same value).
__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}
__device__ __forceinline__ int64_t wave_max(int64_t x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = max(x, (int64_t)__shfl_xor((long long)x, off, 64));
    return x;
}
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ __forceinline__ void wave_sum2(double &s, double &c)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double so = __shfl_xor(s, off, 64), co = __shfl_xor(c, off, 64);
        c += co;
        neumaier(s, c, so);
    }
}

// One DPP move of x inside its row (GFX9 data-parallel primitives; every lane has a source).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the G consecutive lanes of a row group (G = 2, 4 or 8, G-aligned), the same value in
// every lane of the group: butterflies with DPP moves -- quad_perm [1,0,3,2] and [2,3,0,1] inside a
// quad, then row_half_mirror (lane l <-> 7 - l) across the two quads of an 8-lane half-row.  Each
// lane adds the same two partial sums (in either order, which rounds the same), so every lane of the
// group ends with the identical total.
template <typename T, int G>
__device__ __forceinline__ T group_sum(T x)
{
    static_assert(G == 2 || G == 4 || G == 8, "row groups of 2, 4 or 8 lanes");
    x += dpp_move<0xB1>(x);                       // quad_perm [1, 0, 3, 2]
    if constexpr (G >= 4) x += dpp_move<0x4E>(x); // quad_perm [2, 3, 0, 1]
    if constexpr (G >= 8) x += dpp_move<0x141>(x); // row_half_mirror
    return x;
}

// |d| for the kernel argument: the hardware square root in FP32 (1 ulp), IEEE in FP64.
__device__ __forceinline__ float kdist(float r2) { return __builtin_amdgcn_sqrtf(r2); }
__device__ __forceinline__ double kdist(double r2) { return sqrt(r2); }

// Gm += (u_j - u_i) (x) grad W_ij / kfac: the constant factor kfac of the kernel gradient is applied
// once per particle after the row sum.  hih = 1 / (2 h), so 1 - q/2 = 1 - r hih.
template <typename R, int D, int W>
__device__ __forceinline__ void accum_F(R (&Gm)[D * D], const R (&rec)[W], const R (&xi)[D], const R (&ui)[D],
                                        R hih)
{
    R dx[D], du[D];
    R r2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        dx[k] = xi[k] - rec[k];
        du[k] = rec[D + k] - ui[k];
        r2 += dx[k] * dx[k];
    }
    const R tq = fma(-kdist(r2), hih, R(1));
    const R w = tq * tq * tq;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const R gb = w * dx[b];
#pragma unroll
        for (int a = 0; a < D; ++a) Gm[a * D + b] += du[a] * gb;
    }
}

// Pass A over brick `blk` of one body.  VM = true is the same gather on u itself (not the half
// step) ending in the von Mises stress of each own particle (written to vm, FP64, internal order)
// instead of T; nothing else is written.
// A brick's compact map in LDS: loaded once per brick (one word per thread, issued together with
// the brick's run lookups), then read with wavefront-uniform addresses by the staging loops.
struct CMapLds {
    unsigned long long mask[32];
    int prefix[32];
};

// Loads the brick's map words into registers (threads below `words`); call before brick_runs.
__device__ __forceinline__ CMapWord cmap_fetch(const BrickGeom &g, int64_t blk, int tid)
{
    CMapWord w{0ull, 0, 0};
    if (g.cmap && tid < g.cmap_words) w = g.cmap[blk * g.cmap_words + tid];
    return w;
}

// Parks the fetched words in LDS (block-uniform: only for compact bricks) and returns the number of
// staged slots and the compact slot of the brick's first own particle.
__device__ __forceinline__ void cmap_park(const BrickGeom &g, CMapLds &L, const CMapWord &w, int tid, int total,
                                          int own_slot, int &hs, int &own_c)
{
    hs = total;
    own_c = own_slot;
    if (!g.cmap) return;
    if (tid < g.cmap_words) {
        L.mask[tid] = w.mask;
        L.prefix[tid] = w.prefix;
    }
    __syncthreads();
    const int last = g.cmap_words - 1;
    hs = L.prefix[last] + (int)__popcll(L.mask[last]);
    const int a = own_slot >> 6;
    own_c = L.prefix[a] + (int)__popcll(L.mask[a] & ((1ull << (own_slot & 63)) - 1ull));
}

// Tile slot of neighbourhood slot idx in the staging loops of passes A and B, or -1 if it is not
// staged (past the neighbourhood, or left out of a compact one).  The 64 threads of a wavefront take
// one aligned 64-slot group, so the compact slot is the group's prefix plus the read slots of the
// lower lanes (mbcnt over the group's mask).
__device__ __forceinline__ int stage_slot(bool compact, const CMapLds &L, int words, int total, int idx)
{
    if (!compact) return idx < total ? idx : -1;
    const int a = idx >> 6;
    const int ac = a < words ? a : words - 1;
    const uint64_t m = a < words ? L.mask[ac] : 0ull;
    if (idx >= total || !((m >> (idx & 63)) & 1ull)) return -1;
    return L.prefix[ac] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename R, int D, bool VM = false>
__device__ __forceinline__ void passA_brick(const StepParams &P, const BrickGeom &g, const double *__restrict__ X,
                                            const double *__restrict__ u, const R *__restrict__ v,
                                            double *__restrict__ uh, const uint8_t *__restrict__ clamped,
                                            const int64_t *__restrict__ row_ptr, const uint16_t *__restrict__ hslot,
                                            const int32_t *__restrict__ brick_lmax, const R *__restrict__ B0,
                                            R *__restrict__ T, int hcap, DevState *__restrict__ st, int64_t blk,
                                            double *__restrict__ vm = nullptr)
{
    constexpr int W = TileA<R, D>::W;
    constexpr int WU = TileA<R, D>::WU;
    constexpr int PV = TileA<R, D>::PV;
    const int64_t n = P.n;
    const int tid = threadIdx.x;
    const CMapWord cw = cmap_fetch(g, blk, tid);
    BrickRuns<D> BR;
    brick_runs_of<D>(g, blk, BR);
    if (BR.own1 == BR.own0) return;
    extern __shared__ double smem[];
    R *tile = reinterpret_cast<R *>(smem);         // W / PV planes of HS vectors
    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    // compact neighbourhood: HS read slots, the brick's own particles from compact slot own_c on
    __shared__ CMapLds cml;
    int HS, own_c;
    cmap_park(g, cml, cw, tid, BR.total, BR.own0 + cbase, HS, own_c);
    const bool compact = g.cmap != nullptr;
    const double hdt = VM ? 0.0 : 0.5 * st->dt;
    const int ref = BR.own0;
    double xref[D], uref[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xref[k] = (sizeof(R) == 4) ? X[k * n + ref] : 0.0;
        uref[k] = (sizeof(R) == 4) ? u[k * n + ref] : 0.0;
    }
    // neighbourhood -> LDS (all loads of a thread in flight before its LDS stores); the brick's own
    // particles also get their half-step displacement written for pass C
    constexpr int U = 4;
    for (int base = 0; base < BR.total; base += kTile * U) {
        // loads are unconditional (padding threads read particle 0) so none waits at a branch
        double xv[U][D], uu[U][D];
        R vv[U][D];
        uint8_t cj[U];
        int jj[U];
        int dst[U];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kTile + tid;
            dst[w] = stage_slot(compact, cml, g.cmap_words, BR.total, idx);
            jj[w] = dst[w] >= 0 ? halo_particle<D>(BR, idx) : 0;
            const int64_t j = jj[w];
            cj[w] = clamped[j];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                xv[w][k] = X[k * n + j];
                uu[w][k] = u[k * n + j];
                vv[w][k] = VM ? R(0) : v[k * n + j];
            }
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            if (dst[w] < 0) continue;
            const bool own = jj[w] >= BR.own0 && jj[w] < BR.own1;
            R rec[W];
#pragma unroll
            for (int k = 0; k < W; ++k) rec[k] = R(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double uhj = cj[w] ? 0.0 : (VM ? uu[w][k] : uu[w][k] + hdt * (double)vv[w][k]);
                rec[k] = (R)(xv[w][k] - xref[k]);
                rec[D + k] = (R)(uhj - uref[k]);
                if (!VM && own) uh[k * n + jj[w]] = uhj;
            }
            tile_store<R, W, PV, WU>(tile, HS, dst[w], rec);
        }
    }
    __syncthreads();
    const R hih = (R)(0.5 * P.inv_h), vol = (R)(P.vol * P.kfac);   // kfac of the row sums applied here
    const int np = BR.own1 - BR.own0;
    const int lmax = brick_lmax[blk];
    R *gsum = tile + hcap * WU;                     // [np][D*D] reduced sums, after the tile
    // phase 1: G lanes per row accumulate sum_j (u_j - u_i) (x) grad W_ij
    row_batches<D>(np, [&](auto lanes, int q0, int nq) {
        constexpr int G = decltype(lanes)::value;
        constexpr int K = Lanes<D>::rounds(G);
        // row rounds of every lane: the brick's longest row (rows past their end add exact zeros)
        const int kmax = (lmax + G - 1) / G;
        const int lane_g = tid % G;
        const int q = q0 + tid / G;
        if (q >= q0 + nq) return;
        const int64_t i = BR.own0 + q;
        const int64_t e0 = row_ptr[i];
        const int L = (int)(row_ptr[i + 1] - e0);
        const uint16_t *__restrict__ hs = hslot + e0;
        // this lane's row entries lane_g, lane_g + G, ... : slots prefetched before any use; past
        // the row the slot of i itself, whose term is exactly zero (X_i - X_i = u_i - u_i = 0)
        const int islot = own_c + q;
        int sl[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = lane_g + k * G;
            const int s0 = hs[e];   // the slot arrays carry kSlotPad entries past the last row
            sl[k] = e < L ? s0 : islot;
        }
        R ri[W];
        tile_load<R, W, PV, WU>(tile, HS, islot, ri);
        R xi[D], ui[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xi[k] = ri[k];
            ui[k] = ri[D + k];
        }
        R Gm[D * D];
#pragma unroll
        for (int k = 0; k < D * D; ++k) Gm[k] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k >= kmax) break;   // uniform over the workgroup
            R rec[W];
            tile_load<R, W, PV, WU>(tile, HS, sl[k], rec);
            accum_F<R, D, W>(Gm, rec, xi, ui, hih);
        }
        for (int e = lane_g + K * G; e < L; e += G) {
            R rec[W];
            tile_load<R, W, PV, WU>(tile, HS, (int)hs[e], rec);
            accum_F<R, D, W>(Gm, rec, xi, ui, hih);
        }
#pragma unroll
        for (int k = 0; k < D * D; ++k) Gm[k] = group_sum<R, G>(Gm[k]);
#pragma unroll
        for (int k = 0; k < D * D; ++k)
            if (k % G == lane_g) gsum[q * D * D + k] = Gm[k];
    });
    __syncthreads();
    // phase 2: one thread per particle: H = V G B0, stress, T = P B0
    for (int q = tid; q < np; q += kTile) {
        const int64_t i = BR.own0 + q;
        R Gm[D * D], Bi[D * D], H[D * D], Ti[D * D];
#pragma unroll
        for (int k = 0; k < D * D; ++k) {
            Gm[k] = gsum[q * D * D + k];
            Bi[k] = B0[k * n + i];
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) {
                R s = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) s += Gm[a * D + k] * Bi[k * D + b];
                H[a * D + b] = vol * s;
            }
        if constexpr (VM) {
            vm[i] = (double)von_mises<R, D>(H, P.model, (R)P.lam, (R)P.mu);
        } else {
            const bool ok = stress_T<R, D>(H, Bi, P.model, (R)P.lam, (R)P.mu, Ti);
#pragma unroll
            for (int k = 0; k < D * D; ++k) T[k * n + i] = Ti[k];
            if (!ok) atomicOr(&st->bad_stress, 1);
        }
    }
}

// Von Mises stress of every particle for the current displacement (pass A's gather on u).
template <typename R, int D>
__global__ __launch_bounds__(kTile) void k_von_mises(StepParams P, BrickGeom g,
                                                     const double *__restrict__ X, const double *__restrict__ u,
                                                     const R *__restrict__ v, const uint8_t *__restrict__ clamped,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const uint16_t *__restrict__ hslot,
                                                     const int32_t *__restrict__ brick_lmax, const R *__restrict__ B0,
                                                     int hcap, DevState *__restrict__ st, double *__restrict__ vm)
{
    const int64_t blk = xcd_block(blockIdx.x, brick_count(g));
    if (blk < 0) return;
    // v is not read in this mode (the pointer is the body's, so any read would stay in bounds); uh and
    // T are not written
    passA_brick<R, D, true>(P, g, X, u, v, nullptr, clamped, row_ptr, hslot, brick_lmax, B0, nullptr, hcap,
                            st, blk, vm);
}

template <typename R, int D>
__global__ __launch_bounds__(kTile) void k_passA(StepParams P, BrickGeom g,
                                                 const double *__restrict__ X, const double *__restrict__ u,
                                                 const R *__restrict__ v, double *__restrict__ uh,
                                                 const uint8_t *__restrict__ clamped,
                                                 const int64_t *__restrict__ row_ptr,
                                                 const uint16_t *__restrict__ hslot,
                                                 const int32_t *__restrict__ brick_lmax, const R *__restrict__ B0,
                                                 R *__restrict__ T, int hcap, DevState *__restrict__ st)
{
    if (st->done) return;
    const int64_t blk = xcd_block(blockIdx.x, brick_count(g));
    if (blk < 0) return;
    passA_brick<R, D>(P, g, X, u, v, uh, clamped, row_ptr, hslot, brick_lmax, B0, T, hcap, st, blk);
}

template <typename R, int D>
__global__ __launch_bounds__(kTile) void k_passA_batch(const Inst *__restrict__ I, BatchMap M)
{
    const int64_t w = xcd_block(blockIdx.x, M.start[M.count]);
    if (w < 0) return;
    const int k = batch_find(M, (int)w);
    const Inst *in = I + M.inst[k];
    if (in->st->done) return;
    passA_brick<R, D>(in->P, in->ga, in->X, in->u, (const R *)in->v, in->uh, in->clamped,
                      in->row_ptr, in->hslot_a, in->brick_lmax_a, (const R *)in->B0, (R *)in->T, in->halo_a, in->st,
                      w - M.start[k]);
}

// Block-wide maximum and sum in a fixed order (deterministic): wavefront butterflies, then the
// per-wave results in wave order.  NT is a multiple of 64; sh holds 2 * NT / 64 doubles.
template <int NT>
__device__ __forceinline__ void block_max_sum(double &mx, double &sm, double *sh)
{
    constexpr int NW = NT / 64;
    const int t = threadIdx.x;
    mx = wave_max(mx);
    sm = wave_sum(sm);
    __syncthreads();
    if ((t & 63) == 0) {
        sh[t >> 6] = mx;
        sh[NW + (t >> 6)] = sm;
    }
    __syncthreads();
    mx = sh[0];
    sm = sh[NW];
    for (int w = 1; w < NW; ++w) {
        mx = fmax(mx, sh[w]);
        sm += sh[NW + w];
    }
}

// acc += T_j grad W_ij / kfac (kfac applied once per particle after the row sum; hih = 1 / (2 h)).
// The T_i part of the pair term, T_i sum_j grad W_ij, uses the row sum fixed at setup.
template <typename R, int D, int W>
__device__ __forceinline__ void accum_a(R (&acc)[D], const R (&rec)[W], const R (&xi)[D], R hih)
{
    R gw[D];
    R r2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        gw[k] = xi[k] - rec[k];
        r2 += gw[k] * gw[k];
    }
    const R tq = fma(-kdist(r2), hih, R(1));
    const R w = tq * tq * tq;
#pragma unroll
    for (int k = 0; k < D; ++k) gw[k] *= w;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) acc[a] = fma(rec[D + a * D + b], gw[b], acc[a]);
}

// Pass B over brick `blk` of one body.
template <typename R, int D>
__device__ __forceinline__ void passB_brick(const StepParams &P, const BrickGeom &g, const double *__restrict__ X,
                                            const int64_t *__restrict__ row_ptr, const uint16_t *__restrict__ hslot,
                                            const int32_t *__restrict__ brick_lmax, const R *__restrict__ T,
                                            const R *__restrict__ gsum, const R *__restrict__ accel,
                                            const uint8_t *__restrict__ clamped, R *__restrict__ v,
                                            double *__restrict__ partB, const DevState *__restrict__ st, int64_t blk)
{
    constexpr int W = TileB<R, D>::W;
    constexpr int WU = TileB<R, D>::WU;
    constexpr int PV = TileB<R, D>::PV;
    const int64_t n = P.n;
    const int tid = threadIdx.x;
    const CMapWord cw = cmap_fetch(g, blk, tid);
    BrickRuns<D> BR;
    brick_runs_of<D>(g, blk, BR);
    if (BR.own1 == BR.own0) {
        if (tid == 0) {
            partB[2 * blk + 0] = 0.0;
            partB[2 * blk + 1] = 0.0;
        }
        return;
    }
    extern __shared__ double smem[];
    R *tile = reinterpret_cast<R *>(smem);         // W / PV planes of HS vectors
    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    __shared__ CMapLds cml;
    int HS, own_c;
    cmap_park(g, cml, cw, tid, BR.total, BR.own0 + cbase, HS, own_c);
    const bool compact = g.cmap != nullptr;
    const int ref = BR.own0;
    double xref[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xref[k] = (sizeof(R) == 4) ? X[k * n + ref] : 0.0;
    constexpr int U = 4;
    for (int base = 0; base < BR.total; base += kTile * U) {
        double xv[U][D];
        R tv[U][D * D];
        int dst[U];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kTile + tid;
            dst[w] = stage_slot(compact, cml, g.cmap_words, BR.total, idx);
            const int64_t j = dst[w] >= 0 ? halo_particle<D>(BR, idx) : 0;
#pragma unroll
            for (int k = 0; k < D; ++k) xv[w][k] = X[k * n + j];
#pragma unroll
            for (int k = 0; k < D * D; ++k) tv[w][k] = T[k * n + j];
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            if (dst[w] < 0) continue;
            R rec[W];
#pragma unroll
            for (int k = 0; k < W; ++k) rec[k] = R(0);
#pragma unroll
            for (int k = 0; k < D; ++k) rec[k] = (R)(xv[w][k] - xref[k]);
#pragma unroll
            for (int k = 0; k < D * D; ++k) rec[D + k] = tv[w][k];
            tile_store<R, W, PV, WU>(tile, HS, dst[w], rec);
        }
    }
    __syncthreads();
    const R hih = (R)(0.5 * P.inv_h);
    const R cvr = (R)(P.vol / P.rho0 * P.kfac);   // kfac of the row sums applied here
    const double dt = st->dt;
    const int np = BR.own1 - BR.own0;
    const int lmax = brick_lmax[blk];
    double amax = 0.0, asq = 0.0;
    row_batches<D>(np, [&](auto lanes, int q0, int nq) {
        constexpr int G = decltype(lanes)::value;
        constexpr int K = Lanes<D>::rounds(G);
        // row rounds of every lane: the brick's longest row (rows past their end add exact zeros)
        const int kmax = (lmax + G - 1) / G;
        const int lane_g = tid % G;
        const int q = q0 + tid / G;
        if (q >= q0 + nq) return;
        const int64_t i = BR.own0 + q;
        if (clamped[i]) return;   // uniform within the group
        const int64_t e0 = row_ptr[i];
        const int L = (int)(row_ptr[i + 1] - e0);
        const uint16_t *__restrict__ hs = hslot + e0;
        // past the row the slot of i itself, whose term is exactly zero (X_i - X_i = 0)
        const int islot = own_c + q;
        int sl[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = lane_g + k * G;
            const int s0 = hs[e];   // the slot arrays carry kSlotPad entries past the last row
            sl[k] = e < L ? s0 : islot;
        }
        R ri[W];
        tile_load<R, W, PV, WU>(tile, HS, islot, ri);
        R xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = ri[k];
        R acc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k >= kmax) break;   // uniform over the workgroup
            R rec[W];
            tile_load<R, W, PV, WU>(tile, HS, sl[k], rec);
            accum_a<R, D, W>(acc, rec, xi, hih);
        }
        for (int e = lane_g + K * G; e < L; e += G) {
            R rec[W];
            tile_load<R, W, PV, WU>(tile, HS, (int)hs[e], rec);
            accum_a<R, D, W>(acc, rec, xi, hih);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = group_sum<R, G>(acc[k]);
        if (lane_g == 0) {
            R sg[D];
#pragma unroll
            for (int k = 0; k < D; ++k) sg[k] = gsum[k * n + i];
            double a2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                R s2 = acc[a];
#pragma unroll
                for (int b = 0; b < D; ++b) s2 += ri[D + a * D + b] * sg[b];
                R aa = cvr * s2 + (R)P.g[a];
                if (P.has_accel) aa += accel[a * n + i];
                v[a * n + i] = (R)((double)v[a * n + i] + dt * (double)aa);
                a2 += (double)aa * (double)aa;
            }
            amax = fmax(amax, sqrt(a2));
            asq += a2;
        }
    });
    __shared__ double sh[2 * (kTile / 64)];   // block_max_sum: 2 doubles per wavefront
    block_max_sum<kTile>(amax, asq, sh);
    if (tid == 0) {
        partB[2 * blk + 0] = amax;
        partB[2 * blk + 1] = asq;
    }
}

// MW: wavefronts per SIMD the compiler must allow.  Bodies with compact pass-B neighbourhoods take
// MW = 5 in FP32 3D (at most 96 VGPRs, 4 of them spilled), so that five bricks fit on a CU where
// their LDS allows: the 40M-particle column's launch takes 7.4 instead of 8.6 ms (MW = 6 spills far
// more: 10.3 ms).  Other bodies, whose LDS holds four bricks per CU anyway, keep MW = 1 (the spills
// cost them 1.5 %).
template <typename R, int D, int MW>
__global__ __launch_bounds__(kTile, MW) void k_passB(StepParams P, BrickGeom g,
                                                 const double *__restrict__ X, const int64_t *__restrict__ row_ptr,
                                                 const uint16_t *__restrict__ hslot,
                                                 const int32_t *__restrict__ brick_lmax, const R *__restrict__ T,
                                                 const R *__restrict__ gsum, const R *__restrict__ accel,
                                                 const uint8_t *__restrict__ clamped, R *__restrict__ v,
                                                 double *__restrict__ partB, const DevState *__restrict__ st)
{
    if (st->done) return;
    const int64_t blk = xcd_block(blockIdx.x, brick_count(g));
    if (blk < 0) return;
    passB_brick<R, D>(P, g, X, row_ptr, hslot, brick_lmax, T, gsum, accel, clamped, v, partB, st, blk);
}

template <typename R, int D>
__global__ __launch_bounds__(kTile) void k_passB_batch(const Inst *__restrict__ I, BatchMap M)
{
    const int64_t w = xcd_block(blockIdx.x, M.start[M.count]);
    if (w < 0) return;
    const int k = batch_find(M, (int)w);
    const Inst *in = I + M.inst[k];
    if (in->st->done) return;
    passB_brick<R, D>(in->P, in->gb, in->X, in->row_ptr, in->hslot_b, in->brick_lmax_b, (const R *)in->T,
                      (const R *)in->gradsum, (const R *)in->accel, in->clamped, (R *)in->v, in->partB, in->st,
                      w - M.start[k]);
}

constexpr int kBlockC = kBlock;

// Pass C over block `lb` (particles lb * kBlockC ...) of one body.
template <typename R, int D>
__device__ __forceinline__ void passC_block(const StepParams &P, double *__restrict__ u, const double *__restrict__ uh,
                                            R *__restrict__ v, const uint8_t *__restrict__ clamped,
                                            double *__restrict__ partC, const DevState *__restrict__ st, int64_t lb)
{
    __shared__ double sh[4 * kBlockC];
    const int64_t n = P.n;
    const int64_t p = lb * kBlockC + threadIdx.x;
    double ek = 0.0, vmax = 0.0, bad = 0.0;
    if (p < n) {
        if (clamped[p]) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                u[k * n + p] = 0.0;
                v[k * n + p] = R(0);
            }
        } else {
            const double hdt = 0.5 * st->dt;
            double vn2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double vk = (double)v[k * n + p];
                const double uk = uh[k * n + p] + hdt * vk;
                u[k * n + p] = uk;
                vn2 += vk * vk;
                if (!isfinite(uk) || !isfinite(vk)) bad = 1.0;
            }
            ek = 0.5 * P.mass * vn2;
            vmax = sqrt(vn2);
        }
    }
    // fixed-order tree: Neumaier-combined sum of ek, max of vmax and the bad flag
    const int t = threadIdx.x;
    sh[t] = ek;
    sh[kBlockC + t] = 0.0;
    sh[2 * kBlockC + t] = vmax;
    sh[3 * kBlockC + t] = bad;
    __syncthreads();
    for (int off = kBlockC / 2; off > 0; off >>= 1) {
        if (t < off) {
            double s = sh[t], c = sh[kBlockC + t] + sh[kBlockC + t + off];
            neumaier(s, c, sh[t + off]);
            sh[t] = s;
            sh[kBlockC + t] = c;
            sh[2 * kBlockC + t] = fmax(sh[2 * kBlockC + t], sh[2 * kBlockC + t + off]);
            sh[3 * kBlockC + t] = fmax(sh[3 * kBlockC + t], sh[3 * kBlockC + t + off]);
        }
        __syncthreads();
    }
    if (t == 0) {
        partC[4 * lb + 0] = sh[0];
        partC[4 * lb + 1] = sh[kBlockC];
        partC[4 * lb + 2] = sh[2 * kBlockC];
        partC[4 * lb + 3] = sh[3 * kBlockC];
    }
}

template <typename R, int D>
__global__ __launch_bounds__(kBlockC) void k_passC(StepParams P, double *__restrict__ u,
                                                   const double *__restrict__ uh, R *__restrict__ v,
                                                   const uint8_t *__restrict__ clamped, double *__restrict__ partC,
                                                   const DevState *__restrict__ st)
{
    if (st->done) return;
    passC_block<R, D>(P, u, uh, v, clamped, partC, st, blockIdx.x);
}

template <typename R, int D>
__global__ __launch_bounds__(kBlockC) void k_passC_batch(const Inst *__restrict__ I, BatchMap M)
{
    const int w = (int)blockIdx.x;
    const int k = batch_find(M, w);
    const Inst *in = I + M.inst[k];
    if (in->st->done) return;
    passC_block<R, D>(in->P, in->u, in->uh, (R *)in->v, in->clamped, in->partC, in->st, w - M.start[k]);
}

constexpr int kFinishThreads = 1024;
constexpr int kPartialThreads = 256;
constexpr int kResidThreads = 256;

// Eq. 18, capped by the viscous limit of Eq. 35 where the particle-by-particle damping applies
// (dt_visc = infinity otherwise).
__device__ __forceinline__ double time_step(const StepParams &P, double vmax, double amax)
{
    const double t1 = (P.c + vmax > 0.0) ? P.h / (P.c + vmax) : INFINITY;
    const double t2 = (amax > 0.0) ? sqrt(P.h / amax) : INFINITY;
    return fmin(0.6 * fmin(t1, t2), P.dt_visc);
}

// End-of-step reductions of one body by one workgroup of kFinishThreads threads: E_k (Neumaier),
// max |a|, sum |a|^2, max |v| and the non-finite flag from the pass B / pass C partials; E_peak, the
// window ring, the next dt (Eq. 18) and the stop rule.
//
// Stop rule.  The window residual r_n = max over the last W steps (since the last reset) of
// E_k(m) / E_peak(n) is below tol exactly when no step m of the window is "high", i.e. has
// E_k(m) / E_peak(m) >= tol (or E_peak(m) = 0): E_peak never decreases and grows only at a step
// that is itself high, so the latest high step m* has E_peak(m*) = E_peak(n) and decides.  The
// finish kernel therefore keeps the index of the latest high step instead of scanning the window;
// the residual's value is computed only when the host reads the state (k_resid).
__device__ __forceinline__ void finish_body(const StepParams &P, int nbB, int nbC, const double *__restrict__ partB,
                                            const double *__restrict__ partC, double *__restrict__ win_buf,
                                            DevState *__restrict__ st, const double *__restrict__ partF = nullptr,
                                            int nbF = 0)
{
    constexpr int NW = kFinishThreads / 64;
    __shared__ double sw[7][NW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double amax = 0.0, asq = 0.0, asq_c = 0.0, ek = 0.0, ek_c = 0.0, vmax = 0.0, bad = 0.0;
    // two-stage bodies: the nbF slice results of k_partials (amax, sum |a|^2 and its compensation,
    // E_k and its compensation, vmax, non-finite flag) stand for the block partials
    for (int f = t; f < nbF; f += kFinishThreads) {
        const double *pf = partF + 8 * f;
        amax = fmax(amax, pf[0]);
        neumaier(asq, asq_c, pf[1]);
        asq_c += pf[2];
        neumaier(ek, ek_c, pf[3]);
        ek_c += pf[4];
        vmax = fmax(vmax, pf[5]);
        bad = fmax(bad, pf[6]);
    }
    if (nbF > 0) nbB = nbC = 0;
    // each thread takes partials t, t + kFinishThreads, ... in order; U of them are loaded before
    // any is accumulated (a missing partial adds exact zeros)
    constexpr int U = 8;
    for (int b0 = t; b0 < nbB; b0 += kFinishThreads * U) {
        double pa[U], ps[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int b = b0 + k * kFinishThreads;
            pa[k] = b < nbB ? partB[2 * b] : 0.0;
            ps[k] = b < nbB ? partB[2 * b + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            amax = fmax(amax, pa[k]);
            neumaier(asq, asq_c, ps[k]);
        }
    }
    for (int b0 = t; b0 < nbC; b0 += kFinishThreads * U) {
        double pc[U][4];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int b = b0 + k * kFinishThreads;
#pragma unroll
            for (int c = 0; c < 4; ++c) pc[k][c] = b < nbC ? partC[4 * b + c] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            neumaier(ek, ek_c, pc[k][0]);
            ek_c += pc[k][1];
            vmax = fmax(vmax, pc[k][2]);
            bad = fmax(bad, pc[k][3]);
        }
    }
    amax = wave_max(amax);
    vmax = wave_max(vmax);
    bad = wave_max(bad);
    wave_sum2(asq, asq_c);
    wave_sum2(ek, ek_c);
    if (lane == 0) {
        sw[0][wv] = amax;
        sw[1][wv] = asq;
        sw[2][wv] = asq_c;
        sw[3][wv] = ek;
        sw[4][wv] = ek_c;
        sw[5][wv] = vmax;
        sw[6][wv] = bad;
    }
    __syncthreads();
    if (t != 0) return;
    double a_max = sw[0][0], a_s = sw[1][0], a_c = sw[2][0], e_s = sw[3][0], e_c = sw[4][0], v_max = sw[5][0];
    double bd = sw[6][0];
    for (int w = 1; w < NW; ++w) {
        a_max = fmax(a_max, sw[0][w]);
        a_c += sw[2][w];
        neumaier(a_s, a_c, sw[1][w]);
        e_c += sw[4][w];
        neumaier(e_s, e_c, sw[3][w]);
        v_max = fmax(v_max, sw[5][w]);
        bd = fmax(bd, sw[6][w]);
    }
    const double a_sq = a_s + a_c;
    const double e_k = e_s + e_c;
    st->amax = a_max;
    st->vmax = v_max;
    st->ek = e_k;
    st->fres = (P.bsq > 0.0) ? sqrt(a_sq) / sqrt(P.bsq) : sqrt(a_sq);
    if (e_k > st->ek_peak) st->ek_peak = e_k;
    if (st->ek_turn == 0.0 && e_k < st->ek_peak) st->ek_turn = st->ek_peak;
    win_buf[st->win_pos] = e_k;
    st->win_pos = (st->win_pos + 1) % st->win;
    if (st->win_fill < st->win) st->win_fill += 1;
    st->dt = time_step(P, v_max, a_max);
    const int64_t n = st->step + 1;
    st->step = n;
    const double peak = st->ek_peak;
    if (!(peak > 0.0) || e_k / peak >= st->tol) st->last_high = n;
    if (bd > 0.0 || st->bad_stress != 0 || !isfinite(e_k)) {
        st->error = -5;
        st->done = 1;
    } else if (st->ek_turn > 0.0 && e_k > P.div_factor * st->ek_turn) {
        // blow-up: the kinetic energy has grown far beyond the peak it turned over from
        st->error = -6;
        st->done = 1;
    }
    const bool conv = st->last_high <= max(n - st->win, st->win_start) && n >= st->win;
    if (st->stop_on_converge && conv) st->done = 1;
    if (n >= st->max_step) st->done = 1;
}

__global__ __launch_bounds__(kFinishThreads) void k_finish(StepParams P, int nbB, int nbC,
                                                           const double *__restrict__ partB,
                                                           const double *__restrict__ partC,
                                                           double *__restrict__ win_buf, DevState *__restrict__ st,
                                                           const double *__restrict__ partF, int nbF)
{
    if (st->done) return;
    finish_body(P, nbB, nbC, partB, partC, win_buf, st, partF, nbF);
}

// First stage of the two-stage finish: workgroup g combines a contiguous slice of the pass-B and
// pass-C block partials (the finish's own max / Neumaier combination) into partF[8 g .. 8 g + 6].
// A single workgroup reading the 14 MB of partials of a 40M-particle body took 280 us per step.
__global__ __launch_bounds__(kPartialThreads) void k_partials(int nbB, int nbC, const double *__restrict__ partB,
                                                              const double *__restrict__ partC,
                                                              double *__restrict__ partF,
                                                              const DevState *__restrict__ st)
{
    if (st->done) return;
    constexpr int NW = kPartialThreads / 64;
    __shared__ double sw[7][NW];
    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int cb = (nbB + kFinishGroups - 1) / kFinishGroups, cc = (nbC + kFinishGroups - 1) / kFinishGroups;
    const int b0 = g * cb, b1 = min(nbB, b0 + cb), c0 = g * cc, c1 = min(nbC, c0 + cc);
    double amax = 0.0, asq = 0.0, asq_c = 0.0, ek = 0.0, ek_c = 0.0, vmax = 0.0, bad = 0.0;
    for (int b = b0 + t; b < b1; b += kPartialThreads) {
        amax = fmax(amax, partB[2 * b]);
        neumaier(asq, asq_c, partB[2 * b + 1]);
    }
    for (int b = c0 + t; b < c1; b += kPartialThreads) {
        neumaier(ek, ek_c, partC[4 * b]);
        ek_c += partC[4 * b + 1];
        vmax = fmax(vmax, partC[4 * b + 2]);
        bad = fmax(bad, partC[4 * b + 3]);
    }
    amax = wave_max(amax);
    vmax = wave_max(vmax);
    bad = wave_max(bad);
    wave_sum2(asq, asq_c);
    wave_sum2(ek, ek_c);
    if (lane == 0) {
        sw[0][wv] = amax;
        sw[1][wv] = asq;
        sw[2][wv] = asq_c;
        sw[3][wv] = ek;
        sw[4][wv] = ek_c;
        sw[5][wv] = vmax;
        sw[6][wv] = bad;
    }
    __syncthreads();
    if (t != 0) return;
    double a_max = sw[0][0], a_s = sw[1][0], a_c = sw[2][0], e_s = sw[3][0], e_c = sw[4][0], v_max = sw[5][0];
    double bd = sw[6][0];
    for (int w = 1; w < NW; ++w) {
        a_max = fmax(a_max, sw[0][w]);
        a_c += sw[2][w];
        neumaier(a_s, a_c, sw[1][w]);
        e_c += sw[4][w];
        neumaier(e_s, e_c, sw[3][w]);
        v_max = fmax(v_max, sw[5][w]);
        bd = fmax(bd, sw[6][w]);
    }
    double *out = partF + 8 * g;
    out[0] = a_max;
    out[1] = a_s;
    out[2] = a_c;
    out[3] = e_s;
    out[4] = e_c;
    out[5] = v_max;
    out[6] = bd;
}

// One workgroup per body of the table rows `M.inst[0 .. count)`.
__global__ __launch_bounds__(kFinishThreads) void k_finish_batch(const Inst *__restrict__ I, BatchMap M)
{
    const Inst *in = I + M.inst[blockIdx.x];
    if (in->st->done) return;
    finish_body(in->P, in->nbB, in->nbC, in->partB, in->partC, in->win_buf, in->st);
}

// Window residual r = max of the stored E_k / E_peak (1 while E_peak = 0), by a workgroup of
// kResidThreads threads; thread 0 returns it.
__device__ __forceinline__ double resid_body(const double *__restrict__ win_buf, const DevState *__restrict__ st)
{
    constexpr int NW = kResidThreads / 64;
    __shared__ double sw[NW];
    const int t = threadIdx.x;
    const int64_t fill = st->win_fill;
    double m = 0.0;
    for (int64_t q = t; q < fill; q += kResidThreads) m = fmax(m, win_buf[q]);
    m = wave_max(m);
    if ((t & 63) == 0) sw[t >> 6] = m;
    __syncthreads();
    double mx = sw[0];
    for (int w = 1; w < NW; ++w) mx = fmax(mx, sw[w]);
    const double peak = st->ek_peak;
    return peak > 0.0 ? mx / peak : 1.0;
}

__global__ __launch_bounds__(kResidThreads) void k_resid(const double *__restrict__ win_buf, DevState *__restrict__ st)
{
    const double r = resid_body(win_buf, st);
    if (threadIdx.x == 0) st->resid = r;
}

// The state of every body of the table rows `M.inst[0 .. count)`, with its window residual.
__global__ __launch_bounds__(kResidThreads) void k_gather_state(const Inst *__restrict__ I, BatchMap M,
                                                                DevState *__restrict__ out)
{
    const Inst *in = I + M.inst[blockIdx.x];
    const double r = resid_body(in->win_buf, in->st);
    if (threadIdx.x == 0) {
        in->st->resid = r;
        DevState s = *in->st;
        s.resid = r;
        out[blockIdx.x] = s;
    }
}

// max |v| over free particles and the dt that Eq. 18 gives with max |b| for the acceleration.
template <typename R, int D>
__global__ __launch_bounds__(kFinishThreads) void k_init_dt(StepParams P, const R *__restrict__ v,
                                                            const uint8_t *__restrict__ clamped, double bmax,
                                                            double dt_given, DevState *__restrict__ st)
{
    constexpr int NW = kFinishThreads / 64;
    __shared__ double sw[NW];
    const int t = threadIdx.x;
    const int64_t n = P.n;
    double m = 0.0;
    for (int64_t p = t; p < n; p += kFinishThreads) {
        if (clamped[p]) continue;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += (double)v[k * n + p] * (double)v[k * n + p];
        m = fmax(m, sqrt(s));
    }
    m = wave_max(m);
    if ((t & 63) == 0) sw[t >> 6] = m;
    __syncthreads();
    if (t == 0) {
        double mx = sw[0];
        for (int w = 1; w < NW; ++w) mx = fmax(mx, sw[w]);
        st->vmax = mx;
        st->dt = dt_given > 0.0 ? dt_given : time_step(P, mx, bmax);
    }
}

// Arms a run: clears the stop flags, sets the stop rule and re-derives the latest high step of the
// stored window for this tol (the stored E_k / current E_peak; see finish_body).
__global__ __launch_bounds__(kResidThreads) void k_control(DevState *st, const double *__restrict__ win_buf,
                                                           int stop_on_converge, double tol, int64_t max_step)
{
    constexpr int NW = kResidThreads / 64;
    __shared__ int64_t sw[NW];
    const int t = threadIdx.x;
    const int64_t fill = st->win_fill, W = st->win, pos = st->win_pos, n = st->step, start = st->win_start;
    const double peak = st->ek_peak;
    int64_t hi = start;
    for (int64_t q = t; q < fill; q += kResidThreads) {
        const double e = win_buf[q];
        const int64_t age = ((pos - 1 - q) % W + W) % W;
        if (!(peak > 0.0) || e / peak >= tol) hi = max(hi, n - age);
    }
    hi = wave_max(hi);
    if ((t & 63) == 0) sw[t >> 6] = hi;
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < NW; ++w) hi = max(hi, sw[w]);
        st->last_high = hi;
        st->done = 0;
        st->error = 0;
        st->bad_stress = 0;
        st->stop_on_converge = stop_on_converge;
        st->tol = tol;
        st->max_step = max_step;
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// pass A: the neighbourhood tile plus the reduced sums of the brick's own particles (at most
// zb * kMaxCell of them)
size_t passA_lds_bytes(int dim, int precision, int hcap, int zb)
{
    const size_t w = precision == 32 ? (dim == 3 ? TileA<float, 3>::WU : TileA<float, 2>::WU)
                                     : (dim == 3 ? TileA<double, 3>::WU : TileA<double, 2>::WU);
    const size_t rs = precision == 32 ? 4 : 8;
    return ((size_t)hcap * w + (size_t)zb * kMaxCell * dim * dim) * rs;
}
size_t passB_lds_bytes(int dim, int precision, int hcap)
{
    const size_t w = precision == 32 ? (dim == 3 ? TileB<float, 3>::WU : TileB<float, 2>::WU)
                                     : (dim == 3 ? TileB<double, 3>::WU : TileB<double, 2>::WU);
    return (size_t)hcap * w * (precision == 32 ? 4 : 8);
}

void launch_control(DevState *st, const double *win_buf, int stop_on_converge, double tol, int64_t max_step,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kResidThreads), 0, s, st, win_buf, stop_on_converge, tol, max_step);
}

void launch_resid(const DeviceBody &db, hipStream_t s)
{
    hipLaunchKernelGGL(k_resid, dim3(1), dim3(kResidThreads), 0, s, db.win_buf, db.st);
}

#define TLSPH_DISPATCH(prec, dim, KERNEL_CALL)                         \
    do {                                                               \
        if ((prec) == 32 && (dim) == 2) { using R = float; constexpr int D = 2; KERNEL_CALL; }        \
        else if ((prec) == 32) { using R = float; constexpr int D = 3; KERNEL_CALL; }                 \
        else if ((dim) == 2) { using R = double; constexpr int D = 2; KERNEL_CALL; }                  \
        else { using R = double; constexpr int D = 3; KERNEL_CALL; }                                  \
    } while (0)

int passB_blocks(const DeviceBody &db) { return (int)brick_count(db.gb); }

void launch_passA(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s)
{
    const unsigned nb = (unsigned)xcd_grid(brick_count(db.ga));
    const size_t lds = passA_lds_bytes(db.dim, precision, db.halo_a, db.ga.zb);
    TLSPH_DISPATCH(precision, db.dim,
                   hipLaunchKernelGGL((k_passA<R, D>), dim3(nb), dim3(kTile), lds, s, p, db.ga, db.X,
                                      db.u, (const R *)db.v, db.uh, db.clamped, db.row_ptr, db.hslot_a,
                                      db.brick_lmax_a, (const R *)db.B0, (R *)db.T, db.halo_a, db.st));
}

void launch_von_mises(const DeviceBody &db, const StepParams &p, int precision, double *vm, hipStream_t s)
{
    const unsigned nb = (unsigned)xcd_grid(brick_count(db.ga));
    const size_t lds = passA_lds_bytes(db.dim, precision, db.halo_a, db.ga.zb);
    TLSPH_DISPATCH(precision, db.dim,
                   hipLaunchKernelGGL((k_von_mises<R, D>), dim3(nb), dim3(kTile), lds, s, p, db.ga,
                                      db.X, db.u, (const R *)db.v, db.clamped, db.row_ptr, db.hslot_a,
                                      db.brick_lmax_a, (const R *)db.B0, db.halo_a, db.st, vm));
}

void launch_passB(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s)
{
    const unsigned nb = (unsigned)xcd_grid(brick_count(db.gb));
    const size_t lds = passB_lds_bytes(db.dim, precision, db.halo_b);
    if (precision == 32 && db.dim == 3 && db.gb.cmap) {
        hipLaunchKernelGGL((k_passB<float, 3, 5>), dim3(nb), dim3(kTile), lds, s, p, db.gb, db.X,
                           db.row_ptr, db.hslot_b, db.brick_lmax_b, (const float *)db.T, (const float *)db.gradsum,
                           (const float *)db.accel, db.clamped, (float *)db.v, db.partB, db.st);
        return;
    }
    TLSPH_DISPATCH(precision, db.dim,
                   hipLaunchKernelGGL((k_passB<R, D, 1>), dim3(nb), dim3(kTile), lds, s, p, db.gb,
                                      db.X, db.row_ptr, db.hslot_b, db.brick_lmax_b, (const R *)db.T,
                                      (const R *)db.gradsum, (const R *)db.accel, db.clamped, (R *)db.v, db.partB,
                                      db.st));
}

void launch_passC(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s)
{
    TLSPH_DISPATCH(precision, db.dim,
                   hipLaunchKernelGGL((k_passC<R, D>), dim3(blocks_for(db.n)), dim3(kBlockC), 0, s, p, db.u, db.uh,
                                      (R *)db.v, db.clamped, db.partC, db.st));
}

void launch_finish(const DeviceBody &db, const StepParams &p, hipStream_t s)
{
    const int nbB = (int)brick_count(db.gb);
    if (db.partF) {
        hipLaunchKernelGGL(k_partials, dim3(kFinishGroups), dim3(kPartialThreads), 0, s, nbB, db.nblocks, db.partB,
                           db.partC, db.partF, db.st);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s, p, nbB, db.nblocks, db.partB, db.partC,
                           db.win_buf, db.st, (const double *)db.partF, kFinishGroups);
    } else {
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s, p, nbB, db.nblocks, db.partB, db.partC,
                           db.win_buf, db.st, (const double *)nullptr, 0);
    }
}

void launch_init_dt(const DeviceBody &db, const StepParams &p, int precision, double bmax, double dt_given,
                    hipStream_t s)
{
    TLSPH_DISPATCH(precision, db.dim,
                   hipLaunchKernelGGL((k_init_dt<R, D>), dim3(1), dim3(kFinishThreads), 0, s, p, (const R *)db.v,
                                      db.clamped, bmax, dt_given, db.st));
}

// ---- batched launches ----
template <typename F>
static BatchMap batch_map(const Inst *h, const int *slots, int count, F blocks)
{
    BatchMap M;
    M.count = count;
    int acc = 0;
    for (int k = 0; k < count; ++k) {
        M.inst[k] = slots[k];
        M.start[k] = acc;
        acc += blocks(h[slots[k]]);
    }
    M.start[count] = acc;
    return M;
}

// one workgroup per body
static BatchMap unit_map(const int *slots, int count)
{
    BatchMap M;
    M.count = count;
    for (int k = 0; k < count; ++k) {
        M.inst[k] = slots[k];
        M.start[k] = k;
    }
    M.start[count] = count;
    return M;
}

void launch_passA_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s)
{
    if (count <= 0) return;
    size_t lds = 0;
    const BatchMap M = batch_map(h, slots, count, [&](const Inst &in) {
        lds = std::max(lds, passA_lds_bytes(dim, precision, in.halo_a, in.ga.zb));
        return in.nbA;
    });
    if (M.start[count] == 0) return;
    const unsigned nb = (unsigned)xcd_grid(M.start[count]);
    TLSPH_DISPATCH(precision, dim,
                   hipLaunchKernelGGL((k_passA_batch<R, D>), dim3(nb), dim3(kTile), lds, s, I, M));
}

void launch_passB_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s)
{
    if (count <= 0) return;
    size_t lds = 0;
    const BatchMap M = batch_map(h, slots, count, [&](const Inst &in) {
        lds = std::max(lds, passB_lds_bytes(dim, precision, in.halo_b));
        return in.nbB;
    });
    if (M.start[count] == 0) return;
    const unsigned nb = (unsigned)xcd_grid(M.start[count]);
    TLSPH_DISPATCH(precision, dim,
                   hipLaunchKernelGGL((k_passB_batch<R, D>), dim3(nb), dim3(kTile), lds, s, I, M));
}

void launch_passC_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s)
{
    if (count <= 0) return;
    const BatchMap M = batch_map(h, slots, count, [](const Inst &in) { return in.nbC; });
    if (M.start[count] == 0) return;
    TLSPH_DISPATCH(precision, dim,
                   hipLaunchKernelGGL((k_passC_batch<R, D>), dim3((unsigned)M.start[count]), dim3(kBlockC), 0, s, I,
                                      M));
}

void launch_finish_batch(const Inst *I, const int *slots, int count, hipStream_t s)
{
    if (count <= 0) return;
    const BatchMap M = unit_map(slots, count);
    hipLaunchKernelGGL(k_finish_batch, dim3((unsigned)count), dim3(kFinishThreads), 0, s, I, M);
}

void launch_gather_state(const Inst *I, const int *slots, int count, DevState *out, hipStream_t s)
{
    if (count <= 0) return;
    const BatchMap M = unit_map(slots, count);
    hipLaunchKernelGGL(k_gather_state, dim3((unsigned)count), dim3(kResidThreads), 0, s, I, M, out);
}

}  // namespace tlsph
