// damp.hip -- the S_d part of a damped step: pairwise (Sec. 3.2) or particle-by-particle (Sec. 3.1)
// implicit viscous damping swept over the splitting cell-linked list (Sec. 3.4).
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
// DPP row) per cell.  The velocities of each cell's 3^dim-cell neighbourhood (in bodies above 2M
// particles only the slots the cell's visits read, numbered compactly) are staged in LDS;
// the particles of a cell are then processed one after the other.  Along a row the velocity of i
// follows an affine recurrence
//     v_i <- (1 + c_k) v_i - c_k v_j(k)
// (every j appears once in a row, so v_j(k) is its value when the row starts), so the row is a
// composition of affine maps: each lane composes its P consecutive pairs, a DPP scan inside the
// 16-lane row composes the lanes (row_shr for the forward row, row_shl for the backward row), and
// every lane then knows v_i just before its pairs and updates its v_j in registers.  Rows are
// loaded from global memory two particles ahead of the one being processed; row totals are
// broadcast with DPP row_newbcast, so no cross-lane LDS permute sits on the particle chain.
// Wavefronts whose rows hold no clamped particle use one coefficient per pair.
//
// The particle-by-particle scheme (Sec. 3.1, Eqs. 26-34) is the second instantiation of the same
// sweep: D_i(dt/2) takes B_j = eta_t (dt / 2) 2 V^2 (dW/dr) / r, row reductions give sum B_j,
// sum B_j^2 over free neighbours and E_i = -sum B_j (v_i - v_j), k = E_i / ((sum B_j - m)^2 +
// sum B_j^2), v_i += (sum B_j - m) k and every free neighbour v_j -= (B_j / m)(v_i' - v_j + B_j k);
// a clamped i damps each free neighbour by v_j <- m v_j / (m - B_j).
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

// DPP lane moves (GFX9 data-parallel primitives) that write 0 in lanes without a source lane.
template <int CTRL>
__device__ __forceinline__ float dpp0(float src)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp0(double src)
{
    const long long v = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane L of each 16-lane row broadcast to the whole row (DPP row_newbcast:L = 0x150 + L, a VALU
// move in place of a cross-lane LDS permute).
template <int L>
__device__ __forceinline__ int bcast(int src)
{
    return __builtin_amdgcn_update_dpp(0, src, 0x150 + L, 0xf, 0xf, false);
}
template <int L>
__device__ __forceinline__ float bcast(float src)
{
    return __int_as_float(bcast<L>(__float_as_int(src)));
}
template <int L>
__device__ __forceinline__ double bcast(double src)
{
    const long long v = __double_as_longlong(src);
    const int lo = bcast<L>((int)(v & 0xffffffffll));
    const int hi = bcast<L>((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row shifts inside each 16-lane row: row_shr:k = 0x110 + k (from lane - k), row_shl:k = 0x100 + k.
template <int K> struct ShR { static constexpr int C = 0x110 + K; };
template <int K> struct ShL { static constexpr int C = 0x100 + K; };

// Affine maps x -> (1 + d) x + b, kept as (d, b) so that the identity is all zeros (the value the
// DPP moves write where there is no source lane).  Combine this lane's map with the map fetched from
// another lane of the row, the fetched map applied first:
//     x -> (1 + d) ((1 + dp) x + bp) + b = (1 + d + dp + d dp) x + (1 + d) bp + b
template <int CTRL, typename R, int D>
__device__ __forceinline__ void scan_step(R &d, R (&b)[D])
{
    const R dp = dpp0<CTRL>(d);
    R bp[D];
#pragma unroll
    for (int k = 0; k < D; ++k) bp[k] = dpp0<CTRL>(b[k]);
    const R ad = R(1) + d;
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = ad * bp[k] + b[k];
    d = d * dp + (d + dp);
}

// The row scan of a lane's affine map (four scan_steps, row_shr for the forward row, row_shl for the
// backward row), then: x = map of the lanes before this one applied to v_i (the lane one step back
// in row order), and v_i <- the whole row's map applied to v_i (the map in the row's last lane).
template <bool FWD, typename R, int D>
__device__ __forceinline__ void row_maps_generic(R &d, R (&b)[D], R (&vi)[D], R (&x)[D])
{
    constexpr int S1 = FWD ? ShR<1>::C : ShL<1>::C;
    scan_step<FWD ? ShR<1>::C : ShL<1>::C>(d, b);
    scan_step<FWD ? ShR<2>::C : ShL<2>::C>(d, b);
    scan_step<FWD ? ShR<4>::C : ShL<4>::C>(d, b);
    scan_step<FWD ? ShR<8>::C : ShL<8>::C>(d, b);
    const R dx = dpp0<S1>(d);
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = dx * vi[k] + (vi[k] + dpp0<S1>(b[k]));
    constexpr int LAST = FWD ? kSeg - 1 : 0;
    const R aL = R(1) + bcast<LAST>(d);
#pragma unroll
    for (int k = 0; k < D; ++k) vi[k] = aL * vi[k] + bcast<LAST>(b[k]);
}

// FP32 form of row_maps_generic with every DPP move folded into the instruction that consumes it
// (v_fmac_f32 / v_add_f32 with a DPP source operand): per scan step
//     ad = 1 + d;  b_k += ad * b_k[src];  d' = d[src] + d + d[src] * d
// the same operations in the same order as scan_step, without the separate moves.  The block starts
// with s_nop 4: five wait states cover a DPP read of a VGPR (or EXEC) written just before the block;
// inside it every DPP source was written at least two instructions earlier.  d alternates between
// two registers so that each step reads its input while writing its output.
#define TLSPH_DPP(ctl) " " ctl " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define TLSPH_BC(ctl) " " ctl " row_mask:0xf bank_mask:0xf\n\t"
#define TLSPH_STEP2(ctl, DI, DO)                                         \
    "v_add_f32 %[ad], 1.0, " DI "\n\t"                                   \
    "v_fmac_f32_dpp %[b0], %[b0], %[ad]" TLSPH_DPP(ctl)                  \
    "v_fmac_f32_dpp %[b1], %[b1], %[ad]" TLSPH_DPP(ctl)                  \
    "v_add_f32_dpp " DO ", " DI ", " DI TLSPH_DPP(ctl)                   \
    "v_fmac_f32_dpp " DO ", " DI ", " DI TLSPH_DPP(ctl)
#define TLSPH_STEP3(ctl, DI, DO)                                         \
    "v_add_f32 %[ad], 1.0, " DI "\n\t"                                   \
    "v_fmac_f32_dpp %[b0], %[b0], %[ad]" TLSPH_DPP(ctl)                  \
    "v_fmac_f32_dpp %[b1], %[b1], %[ad]" TLSPH_DPP(ctl)                  \
    "v_fmac_f32_dpp %[b2], %[b2], %[ad]" TLSPH_DPP(ctl)                  \
    "v_add_f32_dpp " DO ", " DI ", " DI TLSPH_DPP(ctl)                   \
    "v_fmac_f32_dpp " DO ", " DI ", " DI TLSPH_DPP(ctl)
#define TLSPH_SCAN(STEP, s1, s2, s4, s8)                                 \
    "s_nop 4\n\t"                                                        \
    STEP(s1, "%[d]", "%[t]") STEP(s2, "%[t]", "%[d]")                    \
    STEP(s4, "%[d]", "%[t]") STEP(s8, "%[t]", "%[d]")
#define TLSPH_TAIL2(s1, bc)                                              \
    "v_add_f32_dpp %[x0], %[b0], %[v0]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[x1], %[b1], %[v1]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[n0], %[b0], %[v0]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[x0], %[d], %[v0]" TLSPH_DPP(s1)                    \
    "v_fmac_f32_dpp %[x1], %[d], %[v1]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[n1], %[b1], %[v1]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[n0], %[d], %[v0]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[n1], %[d], %[v1]" TLSPH_BC(bc)
#define TLSPH_TAIL3(s1, bc)                                              \
    "v_add_f32_dpp %[x0], %[b0], %[v0]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[x1], %[b1], %[v1]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[x2], %[b2], %[v2]" TLSPH_DPP(s1)                    \
    "v_fmac_f32_dpp %[x0], %[d], %[v0]" TLSPH_DPP(s1)                    \
    "v_fmac_f32_dpp %[x1], %[d], %[v1]" TLSPH_DPP(s1)                    \
    "v_fmac_f32_dpp %[x2], %[d], %[v2]" TLSPH_DPP(s1)                    \
    "v_add_f32_dpp %[n0], %[b0], %[v0]" TLSPH_BC(bc)                     \
    "v_add_f32_dpp %[n1], %[b1], %[v1]" TLSPH_BC(bc)                     \
    "v_add_f32_dpp %[n2], %[b2], %[v2]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[n0], %[d], %[v0]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[n1], %[d], %[v1]" TLSPH_BC(bc)                     \
    "v_fmac_f32_dpp %[n2], %[d], %[v2]" TLSPH_BC(bc)

template <bool FWD, typename R, int D>
__device__ __forceinline__ void row_maps(R &d, R (&b)[D], R (&vi)[D], R (&x)[D])
{
    if constexpr (sizeof(R) == 4 && D == 3) {
        float ad, t, n0, n1, n2;
        if constexpr (FWD)
            asm volatile(TLSPH_SCAN(TLSPH_STEP3, "row_shr:1", "row_shr:2", "row_shr:4", "row_shr:8")
                         TLSPH_TAIL3("row_shr:1", "row_newbcast:15")
                         : [d] "+v"(d), [b0] "+v"(b[0]), [b1] "+v"(b[1]), [b2] "+v"(b[2]), [ad] "=&v"(ad),
                           [t] "=&v"(t), [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [n0] "=&v"(n0),
                           [n1] "=&v"(n1), [n2] "=&v"(n2)
                         : [v0] "v"(vi[0]), [v1] "v"(vi[1]), [v2] "v"(vi[2]));
        else
            asm volatile(TLSPH_SCAN(TLSPH_STEP3, "row_shl:1", "row_shl:2", "row_shl:4", "row_shl:8")
                         TLSPH_TAIL3("row_shl:1", "row_newbcast:0")
                         : [d] "+v"(d), [b0] "+v"(b[0]), [b1] "+v"(b[1]), [b2] "+v"(b[2]), [ad] "=&v"(ad),
                           [t] "=&v"(t), [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [n0] "=&v"(n0),
                           [n1] "=&v"(n1), [n2] "=&v"(n2)
                         : [v0] "v"(vi[0]), [v1] "v"(vi[1]), [v2] "v"(vi[2]));
        vi[0] = n0;
        vi[1] = n1;
        vi[2] = n2;
    } else if constexpr (sizeof(R) == 4 && D == 2) {
        float ad, t, n0, n1;
        if constexpr (FWD)
            asm volatile(TLSPH_SCAN(TLSPH_STEP2, "row_shr:1", "row_shr:2", "row_shr:4", "row_shr:8")
                         TLSPH_TAIL2("row_shr:1", "row_newbcast:15")
                         : [d] "+v"(d), [b0] "+v"(b[0]), [b1] "+v"(b[1]), [ad] "=&v"(ad), [t] "=&v"(t),
                           [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [n0] "=&v"(n0), [n1] "=&v"(n1)
                         : [v0] "v"(vi[0]), [v1] "v"(vi[1]));
        else
            asm volatile(TLSPH_SCAN(TLSPH_STEP2, "row_shl:1", "row_shl:2", "row_shl:4", "row_shl:8")
                         TLSPH_TAIL2("row_shl:1", "row_newbcast:0")
                         : [d] "+v"(d), [b0] "+v"(b[0]), [b1] "+v"(b[1]), [ad] "=&v"(ad), [t] "=&v"(t),
                           [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [n0] "=&v"(n0), [n1] "=&v"(n1)
                         : [v0] "v"(vi[0]), [v1] "v"(vi[1]));
        vi[0] = n0;
        vi[1] = n1;
    } else {
        row_maps_generic<FWD, R, D>(d, b, vi, x);
    }
}
#undef TLSPH_DPP
#undef TLSPH_BC
#undef TLSPH_STEP2
#undef TLSPH_STEP3
#undef TLSPH_SCAN
#undef TLSPH_TAIL2
#undef TLSPH_TAIL3

// Halo velocities of a cell in LDS.  Slot s holds v of neighbourhood particle s.  FP32 3D: a plane of
// (x, y) pairs and a plane of z, 12 bytes per slot, so a neighbour is two LDS reads (a padded 16-byte
// vector is one, but the LDS per wavefront then limits a large body's damping launch to one
// wavefront per SIMD; with 12 bytes a CU holds half as many again, and the 40M-particle column's
// colour launch runs 23 % faster; TLSPH_DAMP_HALO12=0 restores the vector).  FP32 and FP64 2D: one
// vector per slot.  FP64 3D: D planes of HC words.
#ifndef TLSPH_DAMP_HALO12
#define TLSPH_DAMP_HALO12 1
#endif
template <typename R, int D> struct HaloV {
    static constexpr bool kPair = TLSPH_DAMP_HALO12 && D == 3 && sizeof(R) == 4;
    static constexpr bool kVec = !kPair && ((D == 2) || (sizeof(R) == 4));
    static constexpr int VW = (D == 3) ? 4 : 2;
    static constexpr int words = kVec ? VW : D;
};
template <typename R, int N> using vec_t = R __attribute__((ext_vector_type(N)));

template <typename R, int D>
__device__ __forceinline__ void hv_load(const R *__restrict__ sv, int HC, int slot, R (&x)[D])
{
    if constexpr (HaloV<R, D>::kPair) {
        const vec_t<R, 2> v = *reinterpret_cast<const vec_t<R, 2> *>(sv + slot * 2);
        x[0] = v[0];
        x[1] = v[1];
        x[2] = sv[2 * HC + slot];
    } else if constexpr (HaloV<R, D>::kVec) {
        constexpr int VW = HaloV<R, D>::VW;
        const vec_t<R, VW> v = *reinterpret_cast<const vec_t<R, VW> *>(sv + slot * VW);
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = v[k];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = sv[k * HC + slot];
    }
}
template <typename R, int D>
__device__ __forceinline__ void hv_store(R *__restrict__ sv, int HC, int slot, const R (&x)[D])
{
    if constexpr (HaloV<R, D>::kPair) {
        vec_t<R, 2> v;
        v[0] = x[0];
        v[1] = x[1];
        *reinterpret_cast<vec_t<R, 2> *>(sv + slot * 2) = v;
        sv[2 * HC + slot] = x[2];
    } else if constexpr (HaloV<R, D>::kVec) {
        constexpr int VW = HaloV<R, D>::VW;
        vec_t<R, VW> v;
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = k < D ? x[k] : R(0);
        *reinterpret_cast<vec_t<R, VW> *>(sv + slot * VW) = v;
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) sv[k * HC + slot] = x[k];
    }
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
    const int32_t *order;   // this colour's cells (linear cell ids) in launch order
    const uint64_t *touch;  // compact neighbourhoods: per cell and lane, the slots staged (or null)
    const int32_t *own_rank;  // compact neighbourhoods: per cell, the compact slot of its first particle
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
    R ci[P], dj[P];     // v_i += cI (v_i - v_j);  v_j -= dJ (v_i - v_j)
    __device__ R cI(int t) const { return ci[t]; }
    __device__ R dJ(int t) const { return dj[t]; }
};

// The same for a row whose particle and neighbours are all free: one coefficient per pair.
template <typename R, int P>
struct RowFree {
    int slot[P];
    R c[P];
    __device__ R cI(int t) const { return c[t]; }
    __device__ R dJ(int t) const { return c[t]; }
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
        rr.ci[t] = (cls & 2) ? R(0) : c;
        rr.dj[t] = (cls & 1) ? R(0) : c;
    }
}

// decode_row for rows without clamped particles (every class 0): c = B / (m - 2 B).
template <typename R, int P>
__device__ __forceinline__ void decode_row_free(RowFree<R, P> &rr, const RowRaw<R, P> &in, int sl, R bscale, R m,
                                                int dummy)
{
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const bool ok = sl * P + t < in.L;
        const R B = bscale * in.g[t];
        const R c = B * recip(m - R(2) * B);
        rr.slot[t] = ok ? in.raw[t] : dummy;
        rr.c[t] = ok ? c : R(0);
    }
}

// D_i(dt/2) on the 16-lane row of this cell: the row forward, then the row backward (Eq. 37).
template <typename R, int D, int P, typename Row>
__device__ __forceinline__ void damp_particle(R (&vi)[D], const Row &rr, R *__restrict__ sv, int HC)
{
    R vj[P][D];
#pragma unroll
    for (int t = 0; t < P; ++t) hv_load<R, D>(sv, HC, rr.slot[t], vj[t]);
    // ---- forward: lanes ascending, pairs of a lane ascending ----
    {
        // this lane's pairs composed: pair t maps x -> (1 + c) x - c v_j (the first one from the
        // identity: d = c, b = -c v_j)
        R d = rr.cI(0), b[D];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = -(rr.cI(0) * vj[0][k]);
#pragma unroll
        for (int t = 1; t < P; ++t) {
            const R c = rr.cI(t);
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = b[k] + c * (b[k] - vj[t][k]);
            d = c * d + (c + d);
        }
        // x: v_i as this lane's pairs start; v_i: after the whole row (its map sits in lane 15)
        R x[D];
        row_maps<true, R, D>(d, b, vi, x);
#pragma unroll
        for (int t = 0; t < P; ++t)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R w = x[k] - vj[t][k];
                x[k] = x[k] + rr.cI(t) * w;
                vj[t][k] = vj[t][k] - rr.dJ(t) * w;
            }
    }
    // ---- backward: lanes descending, pairs of a lane descending ----
    {
        R d = rr.cI(P - 1), b[D];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = -(rr.cI(P - 1) * vj[P - 1][k]);
#pragma unroll
        for (int t = P - 2; t >= 0; --t) {
            const R c = rr.cI(t);
#pragma unroll
            for (int k = 0; k < D; ++k) b[k] = b[k] + c * (b[k] - vj[t][k]);
            d = c * d + (c + d);
        }
        // the whole backward row's map sits in lane 0
        R x[D];
        row_maps<false, R, D>(d, b, vi, x);
#pragma unroll
        for (int t = P - 1; t >= 0; --t)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R w = x[k] - vj[t][k];
                x[k] = x[k] + rr.cI(t) * w;
                vj[t][k] = vj[t][k] - rr.dJ(t) * w;
            }
    }
#pragma unroll
    for (int t = 0; t < P; ++t) hv_store<R, D>(sv, HC, rr.slot[t], vj[t]);
}

// ---- particle-by-particle scheme (Sec. 3.1) ----

// Row data of one particle for this lane: B_j of Eq. 27 (B = eta_t (dt / 2) g_ij, zero past the
// row), whether j is free, and j's slot (the dummy slot past the row).
template <typename R, int P>
struct PbpRegs {
    int slot[P];
    R B[P];
    R jfree[P];
};

template <typename R, int P>
__device__ __forceinline__ void decode_row_pbp(PbpRegs<R, P> &pr, const RowRaw<R, P> &in, int sl, R bscale, int dummy)
{
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const bool ok = sl * P + t < in.L;
        const int raw = in.raw[t];
        pr.slot[t] = ok ? (raw & 0x3fff) : dummy;
        pr.B[t] = ok ? bscale * in.g[t] : R(0);
        pr.jfree[t] = (ok && !(raw & (1 << 14))) ? R(1) : R(0);
    }
}

// Sum over the 16 lanes of the row, the same value in every lane (inclusive DPP scan, lane 15's
// total broadcast).
template <typename R>
__device__ __forceinline__ R row_sum(R x)
{
    x += dpp0<ShR<1>::C>(x);
    x += dpp0<ShR<2>::C>(x);
    x += dpp0<ShR<4>::C>(x);
    x += dpp0<ShR<8>::C>(x);
    return bcast<kSeg - 1>(x);
}

// D_i(dt/2) of the particle-by-particle scheme on the 16-lane row of this cell: one gradient step on
// the implicit local system (Eqs. 29-32) for v_i, the neighbours' predictions (Eq. 33) and their
// momentum-conserving update (Eq. 34); clamped neighbours are not variables.  A clamped i (wall)
// damps each free neighbour by the exact one-neighbour solution v_j m / (m - B_j).
template <typename R, int D, int P>
__device__ __forceinline__ void damp_particle_pbp(R (&vi)[D], const PbpRegs<R, P> &pr, bool iclamped, R *__restrict__ sv,
                                                  int HC, R m)
{
    R vj[P][D];
#pragma unroll
    for (int t = 0; t < P; ++t) hv_load<R, D>(sv, HC, pr.slot[t], vj[t]);
    R sB = R(0), sB2 = R(0), E[D];
#pragma unroll
    for (int k = 0; k < D; ++k) E[k] = R(0);
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const R b = pr.B[t];
        sB += b;
        sB2 += pr.jfree[t] * b * b;
#pragma unroll
        for (int k = 0; k < D; ++k) E[k] -= b * (vi[k] - vj[t][k]);
    }
    sB = row_sum(sB);
    sB2 = row_sum(sB2);
#pragma unroll
    for (int k = 0; k < D; ++k) E[k] = row_sum(E[k]);
    const R smm = sB - m;
    const R rden = recip(smm * smm + sB2);
    const R rm = recip(m);
    R kk[D], vin[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        kk[k] = E[k] * rden;
        vin[k] = vi[k] + smm * kk[k];
    }
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const R b = pr.B[t];
        const R wall = m * recip(m - b);
        const R c = b * rm;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R gen = vj[t][k] - c * (vin[k] - vj[t][k] + b * kk[k]);
            const R upd = iclamped ? wall * vj[t][k] : gen;
            vj[t][k] = pr.jfree[t] > R(0) ? upd : vj[t][k];
        }
    }
    if (!iclamped) {
#pragma unroll
        for (int k = 0; k < D; ++k) vi[k] = vin[k];
    }
#pragma unroll
    for (int t = 0; t < P; ++t) hv_store<R, D>(sv, HC, pr.slot[t], vj[t]);
}

// Workgroup `blk` of one colour launch over one body: cells blk * 4 .. blk * 4 + 3 of the colour
// block's launch order (A.order: within windows of consecutive cells the cells with most particles
// first, so the four chains of a wavefront have similar lengths; cells of one colour are independent,
// so their order does not change the result).
//
// COMPACT (bodies with compact neighbourhoods, A.touch set): the cell stages only the slots its
// visits read, numbered consecutively in slot order (their rank), and its rows' slots are those
// numbers.  Staging and write-back take the neighbourhood in slot order, 16 slots a round, and a
// lane's compact slot is the number of read slots before it: the count of earlier rounds plus the
// read slots of lower lanes in its own round (one ballot per round).  A.touch null in a COMPACT
// instantiation (a batched launch mixing both kinds of body) stages every slot at its own index.
template <typename R, int D, int P, bool FWD, int SCHEME, bool COMPACT>
__device__ __forceinline__ void damp_cells(const DampArgs &A, int kx, int ky, int kz, int nby, int nbz, int ncells,
                                           int64_t blk)
{
    const int lane = threadIdx.x;
    const int seg = lane / kSeg, sl = lane % kSeg;
    const int64_t n = A.n;
    const int ci = (int)blk * kCellsPerWave + seg;
    BrickRuns<D> BR;
    int p0 = 0, cnt = 0;
    uint64_t tm = ~0ull;   // COMPACT: bit k set if slot 16 k + sl is staged
    int own_r = -1;        // COMPACT: compact slot of the cell's first particle (-1: full layout)
    if (ci < ncells) {
        const int lin = A.order[ci];
        if constexpr (COMPACT) {
            if (A.touch) {
                tm = A.touch[(int64_t)lin * kSeg + sl];
                own_r = A.own_rank[lin];
            }
        }
        int cx, cy, cz = 0;
        if constexpr (D == 3) {
            cz = lin % A.g.nc[2];
            cy = (lin / A.g.nc[2]) % A.g.nc[1];
            cx = lin / A.g.nc[2] / A.g.nc[1];
        } else {
            cy = lin % A.g.nc[1];
            cx = lin / A.g.nc[1];
        }
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

    // LDS: per segment HC slots of halo velocities (HaloV); slot HC - 1 is a dummy that absorbs the updates of
    // row entries past the end of a row
    extern __shared__ double smem[];
    const int HC = (A.hcap + 2) & ~1;   // even, so the 8-byte pairs of the 12-byte layout stay aligned
    const int dummy = HC - 1;
    R *sv = reinterpret_cast<R *>(smem) + seg * HaloV<R, D>::words * HC;
    R *vg = reinterpret_cast<R *>(A.v);
    const R *gd = reinterpret_cast<const R *>(A.gdamp);
    // COMPACT: whether slot idx (taken by lane idx % 16) is staged, and the ranking of a round
    auto staged = [&](int idx) { return ((tm >> ((idx >> 4) & 63)) & 1ull) != 0; };
    auto compact_slot = [&](bool t, int idx, int &run) {
        const uint32_t segbits = (uint32_t)(__ballot(t) >> (seg * kSeg)) & 0xffffu;
        const int r = run + __popc(segbits & ((1u << sl) - 1u));
        run += __popc(segbits);
        return own_r >= 0 ? r : idx;
    };
    // staging: every load of a lane is issued before its LDS stores
    constexpr int U = sizeof(R) == 4 ? 16 : 8;
    int run = 0;
    for (int base = 0; base < BR.total; base += kSeg * U) {
        // loads are unconditional (padding lanes, and slots a compact neighbourhood leaves out,
        // read particle 0) so none waits at a branch
        R vv[U][D];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kSeg + sl;
            bool t = idx < BR.total;
            if constexpr (COMPACT) t = t && staged(idx);
            const int64_t j = t ? halo_particle<D>(BR, idx) : 0;
#pragma unroll
            for (int k = 0; k < D; ++k) vv[w][k] = vg[k * n + j];
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kSeg + sl;
            if constexpr (COMPACT) {
                const bool t = idx < BR.total && staged(idx);
                const int dst = compact_slot(t, idx, run);
                if (t) hv_store<R, D>(sv, HC, dst, vv[w]);
            } else if (idx < BR.total) {
                hv_store<R, D>(sv, HC, idx, vv[w]);
            }
        }
    }
    // the cell's CSR entries relative to its first one: [0, emax] (p0 + cnt <= n)
    const int64_t E0 = A.row_ptr[p0];
    const int emax = max((int)(A.row_ptr[p0 + cnt] - E0), 1) - 1;
    const uint16_t *__restrict__ cds = A.dslot + E0;
    const R *__restrict__ cgd = gd + E0;
    // pairwise: each pair visit integrates dt / 4 (Eq. 37 inside Eq. 25); particle-by-particle:
    // each D_i integrates dt / 2 (Eq. 25)
    const R bscale = (R)(A.eta_t * (SCHEME == kPairwise ? 0.25 : 0.5) * A.st->dt);
    const R m = (R)A.mass;
    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    // the dummy slot holds zeros: entries past a row read it with zero coefficients
    if (sl == 0) {
        {
            const R z[D] = {};
            hv_store<R, D>(sv, HC, dummy, z);
        }
    }
    // one wavefront per workgroup: its LDS operations complete in issue order, so the loop needs
    // only a compiler-level barrier (a workgroup barrier would also drain the prefetch loads)
    __builtin_amdgcn_wave_barrier();

    // rows are loaded kPrefetch particles ahead (a ring of register buffers, indexed statically by
    // unrolling), so each row's global-memory latency overlaps the processing of the particles
    // before it; particles past the cell's count load a clamped, empty row
    // The rows in visiting order as a 32-entry shift register per cell: lane l of (sA, lA) holds
    // the first entry and the length of the row at position l, (sB, lB) positions 16 + l (length 0
    // past the cell's count).  Each fetch takes lane 0 and shifts the register down by one with
    // DPP moves, so no cross-lane LDS permute sits in the particle loop.
    int sA, lA, sB, lB;
    {
        auto row_pos = [&](int j, int &st, int &len) {
            const bool act = j < cnt;
            const int qs = act ? (FWD ? j : cnt - 1 - j) : 0;
            // reads stay within row_ptr[p0 .. p0 + cnt]
            const int64_t r0 = A.row_ptr[p0 + qs];
            const int64_t r1 = A.row_ptr[p0 + (act ? qs + 1 : qs)];
            st = act ? (int)(r0 - E0) : 0;
            len = (int)(r1 - r0);
        };
        row_pos(sl, sA, lA);
        row_pos(sl + kSeg, sB, lB);
    }
    // The shift is one DPP move per register with every lane active: row_shl:1 has no source for
    // lane 15, which then keeps the move's "old" operand (bound_ctrl off) -- B's lane 0 for the A
    // registers, 0 for the B registers.  (A select around the move would let the compiler run the
    // move with lane 15 masked off, and a masked-off source lane reads as 0 in lane 14.)
    auto next_row = [&](int &e0, int &len) {
        e0 = bcast<0>(sA);
        len = bcast<0>(lA);
        const int s0 = bcast<0>(sB), l0 = bcast<0>(lB);
        sA = __builtin_amdgcn_update_dpp(s0, sA, ShL<1>::C, 0xf, 0xf, false);
        lA = __builtin_amdgcn_update_dpp(l0, lA, ShL<1>::C, 0xf, 0xf, false);
        sB = __builtin_amdgcn_update_dpp(0, sB, ShL<1>::C, 0xf, 0xf, false);
        lB = __builtin_amdgcn_update_dpp(0, lB, ShL<1>::C, 0xf, 0xf, false);
    };
    RowRaw<R, P> buf[kPrefetch];
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
        int e0, len;
        next_row(e0, len);
        load_row<R, P>(buf[k], e0, len, sl, emax, cds, cgd);
    }
    for (int q0 = 0; q0 < maxcnt; q0 += kPrefetch) {
#pragma unroll
        for (int k = 0; k < kPrefetch; ++k) {
            const int q = q0 + k;
            if (q >= maxcnt) break;   // uniform over the wave
            // offsets of the row to prefetch, read first so that their latency overlaps this
            // particle's work; the row itself is loaded once this particle's registers are free
            int e0n, lenn;
            next_row(e0n, lenn);
            const bool active = q < cnt;
            const int qi = FWD ? q : cnt - 1 - q;
            const int islot = active ? (own_r >= 0 ? own_r + qi : p0 + qi + cbase) : dummy;
            R vi[D];
            hv_load<R, D>(sv, HC, islot, vi);
            if constexpr (SCHEME == kPairwise) {
                // rows with a clamped particle anywhere in the wavefront take the general
                // coefficients; the rest (nearly all) one coefficient per pair
                int cls = 0;
#pragma unroll
                for (int t = 0; t < P; ++t) cls |= buf[k].raw[t];
                if (__any(cls & 0xc000)) {
                    RowRegs<R, P> rr;
                    decode_row<R, P>(rr, buf[k], sl, bscale, m, dummy);
                    load_row<R, P>(buf[k], e0n, lenn, sl, emax, cds, cgd);
                    damp_particle<R, D, P>(vi, rr, sv, HC);
                } else {
                    RowFree<R, P> rr;
                    decode_row_free<R, P>(rr, buf[k], sl, bscale, m, dummy);
                    load_row<R, P>(buf[k], e0n, lenn, sl, emax, cds, cgd);
                    damp_particle<R, D, P>(vi, rr, sv, HC);
                }
            } else {
                PbpRegs<R, P> pr;
                decode_row_pbp<R, P>(pr, buf[k], sl, bscale, dummy);
                // the clamp class of i sits in every entry of its row; lane 0 holds entry 0
                const bool iclamped = (bcast<0>(buf[k].raw[0]) >> 15) & 1;
                load_row<R, P>(buf[k], e0n, lenn, sl, emax, cds, cgd);
                damp_particle_pbp<R, D, P>(vi, pr, iclamped, sv, HC, m);
            }
            if (sl == 0) {
                hv_store<R, D>(sv, HC, islot, vi);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    run = 0;
    for (int idx = sl; idx < BR.total; idx += kSeg) {
        int src = idx;
        if constexpr (COMPACT) {
            const bool t = staged(idx);
            src = compact_slot(t, idx, run);
            if (!t) continue;   // not staged, not changed
        }
        const int64_t j = halo_particle<D>(BR, idx);
        {
            R x[D];
            hv_load<R, D>(sv, HC, src, x);
#pragma unroll
            for (int k = 0; k < D; ++k) vg[k * n + j] = x[k];
        }
    }
}


template <typename R, int D, int P, bool FWD, int SCHEME, bool COMPACT>
__global__ __launch_bounds__(kWave) void k_damp(DampArgs A, int kx, int ky, int kz, int nby, int nbz, int ncells)
{
    if (A.st->done) return;
    // blocks are mapped so that each XCD works on one contiguous slab of cells in every colour launch
    const int64_t blk = xcd_block(blockIdx.x, (ncells + kCellsPerWave - 1) / kCellsPerWave);
    if (blk < 0) return;
    damp_cells<R, D, P, FWD, SCHEME, COMPACT>(A, kx, ky, kz, nby, nbz, ncells, blk);
}

template <typename R, int D, int P, bool FWD, int SCHEME, bool COMPACT>
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
    A.order = in->dorder + colour_offset(in->nc, D, D == 3 ? 9 * kx + 3 * ky + kz : 3 * kx + ky);
    A.touch = in->dtouch;
    A.own_rank = in->downr;
    A.st = in->st;
    A.n = in->P.n;
    A.nnz = 1;
    A.g = in->gd;
    A.hcap = in->halo_damp;
    A.mass = in->P.mass;
    A.eta_t = in->eta_t;
    int nby, nbz, ncells;
    colour_cells(in->nc, D, kx, ky, kz, nby, nbz, ncells);
    damp_cells<R, D, P, FWD, SCHEME, COMPACT>(A, kx, ky, kz, nby, nbz, ncells, w - M.start[k]);
}

}  // namespace

int damp_pairs_per_lane(int row_max) { return (row_max + kSeg - 1) / kSeg; }

size_t damp_lds_bytes(int dim, int precision, int hcap, int /*ecap*/)
{
    const size_t rs = precision == 32 ? 4 : 8;
    const size_t words = precision == 32 ? (dim == 3 ? HaloV<float, 3>::words : HaloV<float, 2>::words)
                                         : (dim == 3 ? HaloV<double, 3>::words : HaloV<double, 2>::words);
    return (size_t)kCellsPerWave * ((hcap + 2) & ~1) * words * rs + 16;
}

template <typename R, int D, int P, int SCHEME, bool COMPACT>
static void launch_pb(dim3 g, size_t lds, hipStream_t s, const Inst *I, const BatchMap &M, bool fwd, int kx, int ky,
                      int kz)
{
    if (fwd)
        hipLaunchKernelGGL((k_damp_batch<R, D, P, true, SCHEME, COMPACT>), g, dim3(kWave), lds, s, I, M, kx, ky, kz);
    else
        hipLaunchKernelGGL((k_damp_batch<R, D, P, false, SCHEME, COMPACT>), g, dim3(kWave), lds, s, I, M, kx, ky, kz);
}

template <typename R, int D, int SCHEME, bool COMPACT>
static void launch_rdb_s(int P, dim3 g, size_t lds, hipStream_t s, const Inst *I, const BatchMap &M, bool fwd, int kx,
                         int ky, int kz)
{
    if (P <= 2) launch_pb<R, D, 2, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 3) launch_pb<R, D, 3, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 4) launch_pb<R, D, 4, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 5) launch_pb<R, D, 5, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
    else if (P <= 6) launch_pb<R, D, 6, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
    else launch_pb<R, D, 8, SCHEME, COMPACT>(g, lds, s, I, M, fwd, kx, ky, kz);
}

template <typename R, int D>
static void launch_rdb(int scheme, bool compact, int P, dim3 g, size_t lds, hipStream_t s, const Inst *I,
                       const BatchMap &M, bool fwd, int kx, int ky, int kz)
{
    if (compact) {
        if (scheme == kParticle) launch_rdb_s<R, D, kParticle, true>(P, g, lds, s, I, M, fwd, kx, ky, kz);
        else launch_rdb_s<R, D, kPairwise, true>(P, g, lds, s, I, M, fwd, kx, ky, kz);
    } else {
        if (scheme == kParticle) launch_rdb_s<R, D, kParticle, false>(P, g, lds, s, I, M, fwd, kx, ky, kz);
        else launch_rdb_s<R, D, kPairwise, false>(P, g, lds, s, I, M, fwd, kx, ky, kz);
    }
}

template <typename R, int D, int P, int SCHEME, bool COMPACT>
static void launch_p(dim3 g, size_t lds, hipStream_t s, const DampArgs &A, bool fwd, int kx, int ky, int kz, int nby,
                     int nbz, int ncells)
{
    if (fwd)
        hipLaunchKernelGGL((k_damp<R, D, P, true, SCHEME, COMPACT>), g, dim3(kWave), lds, s, A, kx, ky, kz, nby, nbz,
                           ncells);
    else
        hipLaunchKernelGGL((k_damp<R, D, P, false, SCHEME, COMPACT>), g, dim3(kWave), lds, s, A, kx, ky, kz, nby, nbz,
                           ncells);
}

template <typename R, int D, int SCHEME, bool COMPACT>
static void launch_rd_s(int P, dim3 g, size_t lds, hipStream_t s, const DampArgs &A, bool fwd, int kx, int ky, int kz,
                        int nby, int nbz, int ncells)
{
    if (P <= 2) launch_p<R, D, 2, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 3) launch_p<R, D, 3, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 4) launch_p<R, D, 4, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 5) launch_p<R, D, 5, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else if (P <= 6) launch_p<R, D, 6, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    else launch_p<R, D, 8, SCHEME, COMPACT>(g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
}

template <typename R, int D>
static void launch_rd(int scheme, bool compact, int P, dim3 g, size_t lds, hipStream_t s, const DampArgs &A, bool fwd,
                      int kx, int ky, int kz, int nby, int nbz, int ncells)
{
    if (compact) {
        if (scheme == kParticle) launch_rd_s<R, D, kParticle, true>(P, g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
        else launch_rd_s<R, D, kPairwise, true>(P, g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    } else {
        if (scheme == kParticle) launch_rd_s<R, D, kParticle, false>(P, g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
        else launch_rd_s<R, D, kPairwise, false>(P, g, lds, s, A, fwd, kx, ky, kz, nby, nbz, ncells);
    }
}

void launch_damp_colour(const DeviceBody &db, const StepParams &p, int precision, int scheme, int colour, bool forward,
                        double eta_t, hipStream_t s)
{
    DampArgs A;
    A.v = db.v;
    A.row_ptr = db.row_ptr;
    A.dslot = db.dslot;
    A.gdamp = db.gdamp;
    A.cell_start = db.cell_start;
    A.order = db.dorder + colour_offset(db.nc, db.dim, colour);
    A.touch = db.dtouch;
    A.own_rank = db.downr;
    A.st = db.st;
    A.n = db.n;
    A.nnz = db.nnz > 0 ? db.nnz : 1;
    A.g = db.gd;
    A.hcap = db.halo_damp;
    A.mass = p.mass;
    A.eta_t = eta_t;
    int kx, ky, kz;
    colour_axes(db.dim, colour, kx, ky, kz);
    const int nbx = count_mod3(db.nc[0], kx), nby = count_mod3(db.nc[1], ky);
    const int nbz = db.dim == 3 ? count_mod3(db.nc[2], kz) : 1;
    const int64_t ncells = (int64_t)nbx * nby * nbz;
    if (ncells == 0) return;
    const int64_t blocks = xcd_grid((ncells + kCellsPerWave - 1) / kCellsPerWave);
    const size_t lds = damp_lds_bytes(db.dim, precision, db.halo_damp, 0);
    const int P = damp_pairs_per_lane(db.row_max);
    const bool compact = db.dtouch != nullptr;
    const dim3 g((unsigned)blocks);
    if (precision == 32 && db.dim == 2)
        launch_rd<float, 2>(scheme, compact, P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else if (precision == 32)
        launch_rd<float, 3>(scheme, compact, P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else if (db.dim == 2)
        launch_rd<double, 2>(scheme, compact, P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
    else
        launch_rd<double, 3>(scheme, compact, P, g, lds, s, A, forward, kx, ky, kz, nby, nbz, (int)ncells);
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
    bool compact = false;
    for (int k = 0; k < count; ++k) {
        const Inst &in = h[slots[k]];
        int nby, nbz, ncells;
        colour_cells(in.nc, dim, kx, ky, kz, nby, nbz, ncells);
        M.inst[k] = slots[k];
        M.start[k] = acc;
        acc += (ncells + kCellsPerWave - 1) / kCellsPerWave;
        P = std::max(P, damp_pairs_per_lane(in.row_max));
        lds = std::max(lds, damp_lds_bytes(dim, precision, in.halo_damp, 0));
        compact = compact || in.dtouch != nullptr;
    }
    M.start[count] = acc;
    if (acc == 0) return;
    const dim3 g((unsigned)xcd_grid(acc));
    const int scheme = h[slots[0]].scheme;   // the caller groups bodies by scheme
    if (precision == 32 && dim == 2) launch_rdb<float, 2>(scheme, compact, P, g, lds, s, I, M, forward, kx, ky, kz);
    else if (precision == 32) launch_rdb<float, 3>(scheme, compact, P, g, lds, s, I, M, forward, kx, ky, kz);
    else if (dim == 2) launch_rdb<double, 2>(scheme, compact, P, g, lds, s, I, M, forward, kx, ky, kz);
    else launch_rdb<double, 3>(scheme, compact, P, g, lds, s, I, M, forward, kx, ky, kz);
}

}  // namespace tlsph
