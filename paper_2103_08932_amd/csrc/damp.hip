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
// One launch per colour block, one 64-wide wavefront per cell.  Before the sequential part the
// wave stages in LDS the velocities and clamp flags of the cell's 3^dim-cell neighbourhood and,
// for every CSR entry of the cell's particles, its neighbourhood slot and damping factor B; row
// offsets sit one per lane.  The particles of the cell are then processed one after the other
// without touching global memory.  Along a row the velocity of i follows an affine recurrence
//     v_i <- (1 + c_k) v_i - c_k v_j(k)
// (every j appears once in a row, so v_j(k) is its value when the row starts), so the row is a
// composition of affine maps: each lane composes its share of the row, a DPP wavefront scan
// composes the lanes, and every lane then knows v_i just before its pairs and updates its v_j.
// The backward row uses the same scan with the lane -> pair assignment mirrored.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bricks.hpp"
#include "internal.hpp"

namespace tlsph {
namespace {

constexpr int kWave = 64;

// DPP lane moves (GFX9 data-parallel primitives).  `old` is returned in lanes without a source.
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ float dpp(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, ROWM, BANKM,
                                                      false));
}
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ double dpp(double old, double src)
{
    const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(v & 0xffffffffll), CTRL, ROWM, BANKM,
                                               false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROWM, BANKM, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double readlane(double x, int l)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One step of the composition scan: combine this lane's map (a, b) with the map (ap, bp) fetched
// from an earlier lane (identity where there is none): x -> a (ap x + bp) + b.
template <int CTRL, int ROWM, typename R, int D>
__device__ __forceinline__ void scan_step(R &a, R (&b)[D])
{
    const R ap = dpp<CTRL, ROWM, 0xf>(R(1), a);
    R bp[D];
#pragma unroll
    for (int k = 0; k < D; ++k) bp[k] = dpp<CTRL, ROWM, 0xf>(R(0), b[k]);
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = a * bp[k] + b[k];
    a = a * ap;
}

// Inclusive wavefront scan of affine maps in lane order (lane 0 applied first): Hillis-Steele
// inside each row of 16 lanes, then row 0 -> 1 and 2 -> 3 through lane 15, then rows 0-1 -> 2-3
// through lane 31.
template <typename R, int D>
__device__ __forceinline__ void wave_affine_scan(R &a, R (&b)[D])
{
    scan_step<0x111, 0xf>(a, b);   // row_shr:1
    scan_step<0x112, 0xf>(a, b);   // row_shr:2
    scan_step<0x114, 0xf>(a, b);   // row_shr:4
    scan_step<0x118, 0xf>(a, b);   // row_shr:8
    scan_step<0x142, 0xa>(a, b);   // row_bcast:15 into rows 1 and 3
    scan_step<0x143, 0xc>(a, b);   // row_bcast:31 into rows 2 and 3
}

struct DampArgs {
    void *v;
    const uint8_t *clamped;
    const int64_t *row_ptr;
    const uint16_t *dslot;
    const void *gdamp;  // per CSR entry: 2 V^2 (dW/dr) / r
    const int32_t *cell_start;
    const DevState *st;
    int64_t n;
    BrickGeom g;        // single-cell bricks
    int hcap;           // LDS capacity in particles
    int ecap;           // LDS capacity in CSR entries of one cell
    double mass;
    double eta_t;
};

// Applies the pair operators of one row of particle i to v_i (registers) and the v_j in LDS, in
// row order (MIRROR: reversed row order), lanes in order, P consecutive pairs per lane.  Every
// entry of the row holds its neighbourhood slot with the clamp class in the top two bits (bit 15:
// i clamped, bit 14: j clamped) and the pair coefficient c of Eq. 39 for this step.
template <typename R, int D, int P, bool MIRROR>
__device__ __forceinline__ void damp_row(R (&vi)[D], int L, int lane, const uint16_t *__restrict__ ps,
                                         const R *__restrict__ pc, R *__restrict__ sv, int HC)
{
    R cI[P], dJ[P], vj[P][D];
    int sj[P];
    bool ok[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const int idx = lane * P + t;
        ok[t] = idx < L;
        const int pos = ok[t] ? (MIRROR ? L - 1 - idx : idx) : 0;
        const int raw = ps[pos];
        const R c = ok[t] ? pc[pos] : R(0);
        sj[t] = raw & 0x3fff;
        cI[t] = (raw & 0x8000) ? R(0) : c;    // i clamped: v_i does not move
        dJ[t] = (raw & 0x4000) ? R(0) : c;    // j clamped: v_j does not move
#pragma unroll
        for (int k = 0; k < D; ++k) vj[t][k] = sv[k * HC + sj[t]];
    }
    // this lane's composite map x -> a x + b over its pairs in order
    R a = R(1), b[D];
#pragma unroll
    for (int k = 0; k < D; ++k) b[k] = R(0);
#pragma unroll
    for (int t = 0; t < P; ++t) {
        const R at = R(1) + cI[t];
#pragma unroll
        for (int k = 0; k < D; ++k) b[k] = at * b[k] - cI[t] * vj[t][k];
        a = at * a;
    }
    wave_affine_scan<R, D>(a, b);
    // map of all earlier lanes (wave_shr:1), applied to v_i: v_i before this lane's first pair
    const R ax = dpp<0x138, 0xf, 0xf>(R(1), a);
    R x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = ax * vi[k] + dpp<0x138, 0xf, 0xf>(R(0), b[k]);
#pragma unroll
    for (int t = 0; t < P; ++t) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const R w = x[k] - vj[t][k];
            x[k] = x[k] + cI[t] * w;
            vj[t][k] = vj[t][k] - dJ[t] * w;
        }
    }
#pragma unroll
    for (int t = 0; t < P; ++t)
        if (ok[t]) {
#pragma unroll
            for (int k = 0; k < D; ++k) sv[k * HC + sj[t]] = vj[t][k];
        }
    const R aL = readlane(a, kWave - 1);
#pragma unroll
    for (int k = 0; k < D; ++k) vi[k] = aL * vi[k] + readlane(b[k], kWave - 1);
}

// D_i(dt/2): the row forward, then the row backward (Eq. 37).
template <typename R, int D, int P>
__device__ __forceinline__ void damp_particle(R (&vi)[D], int L, int lane, const uint16_t *__restrict__ ps,
                                              const R *__restrict__ pc, R *__restrict__ sv, int HC)
{
    damp_row<R, D, P, false>(vi, L, lane, ps, pc, sv, HC);
    __syncthreads();
    damp_row<R, D, P, true>(vi, L, lane, ps, pc, sv, HC);
}

template <typename R, int D, bool FWD>
__global__ __launch_bounds__(kWave) void k_damp(DampArgs A, int kx, int ky, int kz, int nby, int nbz)
{
    if (A.st->done) return;
    const int lane = threadIdx.x;
    const int64_t n = A.n;
    int b = blockIdx.x;
    int bz = 0;
    if constexpr (D == 3) {
        bz = b % nbz;
        b /= nbz;
    }
    const int by = b % nby, bx = b / nby;
    const int cx = kx + 3 * bx, cy = ky + 3 * by, cz = (D == 3) ? kz + 3 * bz : 0;
    BrickRuns<D> BR;
    if constexpr (D == 3)
        brick_runs<D>(A.g, A.cell_start, cx, cy, cz, BR);
    else
        brick_runs<D>(A.g, A.cell_start, cx, 0, cy, BR);
    const int p0 = BR.own0, p1 = BR.own1;
    if (p0 == p1) return;
    constexpr int NR = BrickRuns<D>::NR;
    const int64_t E0 = A.row_ptr[p0];
    const int E = (int)(A.row_ptr[p1] - E0);

    // LDS: velocities of the 3^dim-cell neighbourhood, and for every CSR entry of the cell's
    // particles its slot (with the clamp class) and its pair coefficient c of Eq. 39 at this step
    extern __shared__ double smem[];
    const int HC = A.hcap;
    R *sv = reinterpret_cast<R *>(smem);                       // [D][HC]
    R *pc = sv + D * HC;                                       // [ecap]
    uint16_t *ps = reinterpret_cast<uint16_t *>(pc + A.ecap);  // [ecap]
    R *vg = reinterpret_cast<R *>(A.v);
    const R *gd = reinterpret_cast<const R *>(A.gdamp);
    // staging: every load of a lane is issued before its LDS stores
    constexpr int U = 8;
    for (int base = 0; base < BR.total; base += kWave * U) {
        R vv[U][D];
        int jj[U];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int idx = base + w * kWave + lane;
            jj[w] = idx < BR.total ? halo_particle<D>(BR, idx) : -1;
            if (jj[w] >= 0) {
#pragma unroll
                for (int k = 0; k < D; ++k) vv[w][k] = vg[k * n + jj[w]];
            }
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            if (jj[w] < 0) continue;
            const int idx = base + w * kWave + lane;
#pragma unroll
            for (int k = 0; k < D; ++k) sv[k * HC + idx] = vv[w][k];
        }
    }
    // pair coefficient of Eq. 39 with B = eta_t (dt / 4) g_ij and equal masses m:
    // free-free c = B / (m - 2 B), one end clamped c = B / (m - B), both clamped 0
    const R bscale = (R)(A.eta_t * 0.25 * A.st->dt);
    const R m = (R)A.mass;
    for (int base = 0; base < E; base += kWave * U) {
        uint16_t sl[U];
        R gv[U];
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int e = base + w * kWave + lane;
            if (e < E) {
                sl[w] = A.dslot[E0 + e];
                gv[w] = gd[E0 + e];
            }
        }
#pragma unroll
        for (int w = 0; w < U; ++w) {
            const int e = base + w * kWave + lane;
            if (e < E) {
                const int cls = sl[w] >> 14;
                const R B = bscale * gv[w];
                ps[e] = sl[w];
                pc[e] = cls == 3 ? R(0) : B / (m - (cls == 0 ? R(2) : R(1)) * B);
            }
        }
    }
    const int cnt = p1 - p0;
    // row offsets of the cell's particles, one per lane (cells hold at most 63 particles)
    const int rofs = lane <= cnt ? (int)(A.row_ptr[p0 + lane] - E0) : 0;
    __syncthreads();

    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    for (int q = 0; q < cnt; ++q) {
        const int qi = FWD ? q : cnt - 1 - q;
        const int islot = p0 + qi + cbase;
        const int rb = __builtin_amdgcn_readlane(rofs, qi);
        const int L = __builtin_amdgcn_readlane(rofs, qi + 1) - rb;
        R vi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) vi[k] = sv[k * HC + islot];
        if (L <= kWave)
            damp_particle<R, D, 1>(vi, L, lane, ps + rb, pc + rb, sv, HC);
        else if (L <= 2 * kWave)
            damp_particle<R, D, 2>(vi, L, lane, ps + rb, pc + rb, sv, HC);
        else
            damp_particle<R, D, kMaxRowChunks>(vi, L, lane, ps + rb, pc + rb, sv, HC);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) sv[k * HC + islot] = vi[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        for (int t = lane; t < BR.len[r]; t += kWave) {
            const int64_t j = BR.start[r] + t;
            const int s = BR.off[r] + t;
#pragma unroll
            for (int k = 0; k < D; ++k) vg[k * n + j] = sv[k * HC + s];
        }
}

inline int count_mod3(int ncell, int k) { return ncell > k ? (ncell - k + 2) / 3 : 0; }

}  // namespace

size_t damp_lds_bytes(int dim, int precision, int hcap, int ecap)
{
    const size_t rs = precision == 32 ? 4 : 8;
    return (size_t)hcap * dim * rs + (size_t)ecap * (rs + 2) + 16;
}

void launch_damp_colour(const DeviceBody &db, const StepParams &p, int precision, int colour, bool forward,
                        double eta_t, hipStream_t s)
{
    DampArgs A;
    A.v = db.v;
    A.clamped = db.clamped;
    A.row_ptr = db.row_ptr;
    A.dslot = db.dslot;
    A.cell_start = db.cell_start;
    A.st = db.st;
    A.n = db.n;
    A.g = db.gd;
    A.hcap = db.halo_max;
    A.ecap = db.cell_pairs_max;
    A.gdamp = db.gdamp;
    A.mass = p.mass;
    A.eta_t = eta_t;
    int kx, ky, kz;
    if (db.dim == 3) {
        kx = colour / 9;
        ky = (colour / 3) % 3;
        kz = colour % 3;
    } else {
        kx = colour / 3;
        ky = colour % 3;
        kz = 0;
    }
    const int nbx = count_mod3(db.nc[0], kx), nby = count_mod3(db.nc[1], ky);
    const int nbz = db.dim == 3 ? count_mod3(db.nc[2], kz) : 1;
    const int64_t blocks = (int64_t)nbx * nby * nbz;
    if (blocks == 0) return;
    const size_t lds = damp_lds_bytes(db.dim, precision, db.halo_max, db.cell_pairs_max);
    const dim3 g((unsigned)blocks), t(kWave);
    if (precision == 32 && db.dim == 2) {
        if (forward) hipLaunchKernelGGL((k_damp<float, 2, true>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
        else hipLaunchKernelGGL((k_damp<float, 2, false>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
    } else if (precision == 32) {
        if (forward) hipLaunchKernelGGL((k_damp<float, 3, true>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
        else hipLaunchKernelGGL((k_damp<float, 3, false>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
    } else if (db.dim == 2) {
        if (forward) hipLaunchKernelGGL((k_damp<double, 2, true>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
        else hipLaunchKernelGGL((k_damp<double, 2, false>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
    } else {
        if (forward) hipLaunchKernelGGL((k_damp<double, 3, true>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
        else hipLaunchKernelGGL((k_damp<double, 3, false>), g, t, lds, s, A, kx, ky, kz, nby, nbz);
    }
}

}  // namespace tlsph
