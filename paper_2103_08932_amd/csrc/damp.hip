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
// One launch per colour block, one 64-wide wavefront per cell.  The velocities of the cell's
// 3^dim-cell neighbourhood are staged in LDS.  Particles of the cell are processed one after the
// other.  Along a row the velocity of i follows an affine recurrence
//     v_i <- (1 + c_k) v_i - c_k v_j(k)
// (every j appears once in a row, so v_j(k) is its value when the row starts), so the row is a
// composition of affine maps: each lane composes its share of the row, a wavefront scan composes
// the lanes, and every lane then knows v_i just before its pairs and updates its v_j in place.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bricks.hpp"
#include "internal.hpp"

namespace tlsph {
namespace {

constexpr int kWave = 64;

template <typename R>
__device__ __forceinline__ R shfl_up(R x, int d) { return __shfl_up(x, d, kWave); }
template <typename R>
__device__ __forceinline__ R shfl_down(R x, int d) { return __shfl_down(x, d, kWave); }
template <typename R>
__device__ __forceinline__ R shfl_idx(R x, int l) { return __shfl(x, l, kWave); }

struct DampArgs {
    const double *X;
    void *v;
    const uint8_t *clamped;
    const int64_t *row_ptr;
    const uint16_t *dslot;
    const int32_t *cell_start;
    const DevState *st;
    int64_t n;
    BrickGeom g;        // single-cell bricks
    int hcap;           // LDS capacity in particles
    double h_inv;
    double kfac;        // -5 a_D / h^2
    double vol, mass;
    double eta_t;
};

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

    // LDS tile: positions relative to the cell's first particle (FP64 path: absolute), velocities,
    // clamp flags of the 3^dim-cell neighbourhood
    extern __shared__ double smem[];
    const int HC = A.hcap;
    R *sx = reinterpret_cast<R *>(smem);                     // [D][HC]
    R *sv = sx + D * HC;                                     // [D][HC]
    uint8_t *sc = reinterpret_cast<uint8_t *>(sv + D * HC);  // [HC]
    R *vg = reinterpret_cast<R *>(A.v);
    double xref[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xref[k] = sizeof(R) == 4 ? A.X[k * n + p0] : 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        for (int t = lane; t < BR.len[r]; t += kWave) {
            const int64_t j = BR.start[r] + t;
            const int s = BR.off[r] + t;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                sx[k * HC + s] = (R)(A.X[k * n + j] - xref[k]);
                sv[k * HC + s] = vg[k * n + j];
            }
            sc[s] = A.clamped[j];
        }
    __syncthreads();

    const int cbase = BR.off[BrickRuns<D>::CR] - BR.start[BrickRuns<D>::CR];
    const R m = (R)A.mass;
    const R cB = (R)(A.eta_t * 0.25 * A.st->dt * 2.0 * A.vol * A.vol * A.kfac);
    const R h_inv = (R)A.h_inv;

    const int cnt = p1 - p0;
    for (int q = 0; q < cnt; ++q) {
        const int i = FWD ? p0 + q : p1 - 1 - q;
        const int islot = i + cbase;
        const int64_t e0 = A.row_ptr[i];
        const int L = (int)(A.row_ptr[i + 1] - e0);
        const int P = (L + kWave - 1) / kWave;
        const bool ci = sc[islot] != 0;
        R xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = sx[k * HC + islot];
        R cI[kMaxRowChunks], dJ[kMaxRowChunks], vj[kMaxRowChunks][D];
        int sj[kMaxRowChunks];
#pragma unroll
        for (int t = 0; t < kMaxRowChunks; ++t) {
            cI[t] = R(0);
            dJ[t] = R(0);
            sj[t] = -1;
#pragma unroll
            for (int k = 0; k < D; ++k) vj[t][k] = R(0);
            const int idx = lane * P + t;
            if (t < P && idx < L) {
                const int s = A.dslot[e0 + idx];
                sj[t] = s;
                R r2 = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const R d = xi[k] - sx[k * HC + s];
                    r2 += d * d;
                }
                const R tq = R(1) - R(0.5) * sqrt(r2) * h_inv;
                const R B = cB * tq * tq * tq;
                const bool cj = sc[s] != 0;
                if (ci && cj) {
                } else if (cj) {
                    cI[t] = B / (m - B);
                } else if (ci) {
                    dJ[t] = B / (m - B);
                } else {
                    cI[t] = dJ[t] = B / (m - R(2) * B);
                }
#pragma unroll
                for (int k = 0; k < D; ++k) vj[t][k] = sv[k * HC + s];
            }
        }
        R vi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) vi[k] = sv[k * HC + islot];

        // ---- forward row: pairs in ascending order (lane-major) ----
        {
            R a = R(1), bv[D];
#pragma unroll
            for (int k = 0; k < D; ++k) bv[k] = R(0);
#pragma unroll
            for (int t = 0; t < kMaxRowChunks; ++t) {
                const R at = R(1) + cI[t];
#pragma unroll
                for (int k = 0; k < D; ++k) bv[k] = at * bv[k] - cI[t] * vj[t][k];
                a = at * a;
            }
            // inclusive scan: map of lanes 0..lane, later lanes applied after earlier ones
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const R ap = shfl_up(a, off);
                R bp[D];
#pragma unroll
                for (int k = 0; k < D; ++k) bp[k] = shfl_up(bv[k], off);
                if (lane >= off) {
#pragma unroll
                    for (int k = 0; k < D; ++k) bv[k] = a * bp[k] + bv[k];
                    a = a * ap;
                }
            }
            R ax = shfl_up(a, 1);
            R x[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R bx_ = shfl_up(bv[k], 1);
                x[k] = lane == 0 ? vi[k] : ax * vi[k] + bx_;
            }
#pragma unroll
            for (int t = 0; t < kMaxRowChunks; ++t) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const R w = x[k] - vj[t][k];
                    x[k] = x[k] + cI[t] * w;
                    vj[t][k] = vj[t][k] - dJ[t] * w;
                }
            }
            const R aL = shfl_idx(a, kWave - 1);
#pragma unroll
            for (int k = 0; k < D; ++k) vi[k] = aL * vi[k] + shfl_idx(bv[k], kWave - 1);
        }
        // ---- backward row: pairs in descending order ----
        {
            R a = R(1), bv[D];
#pragma unroll
            for (int k = 0; k < D; ++k) bv[k] = R(0);
#pragma unroll
            for (int t = kMaxRowChunks - 1; t >= 0; --t) {
                const R at = R(1) + cI[t];
#pragma unroll
                for (int k = 0; k < D; ++k) bv[k] = at * bv[k] - cI[t] * vj[t][k];
                a = at * a;
            }
            // inclusive suffix scan: map of lanes 63..lane, lower lanes applied after higher ones
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const R an = shfl_down(a, off);
                R bn[D];
#pragma unroll
                for (int k = 0; k < D; ++k) bn[k] = shfl_down(bv[k], off);
                if (lane + off < kWave) {
#pragma unroll
                    for (int k = 0; k < D; ++k) bv[k] = a * bn[k] + bv[k];
                    a = a * an;
                }
            }
            const R ax = shfl_down(a, 1);
            R x[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const R bx_ = shfl_down(bv[k], 1);
                x[k] = lane == kWave - 1 ? vi[k] : ax * vi[k] + bx_;
            }
#pragma unroll
            for (int t = kMaxRowChunks - 1; t >= 0; --t) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const R w = x[k] - vj[t][k];
                    x[k] = x[k] + cI[t] * w;
                    vj[t][k] = vj[t][k] - dJ[t] * w;
                }
            }
            const R a0 = shfl_idx(a, 0);
#pragma unroll
            for (int k = 0; k < D; ++k) vi[k] = a0 * vi[k] + shfl_idx(bv[k], 0);
        }
#pragma unroll
        for (int t = 0; t < kMaxRowChunks; ++t)
            if (sj[t] >= 0) {
#pragma unroll
                for (int k = 0; k < D; ++k) sv[k * HC + sj[t]] = vj[t][k];
            }
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

size_t damp_lds_bytes(int dim, int precision, int hcap)
{
    return (size_t)hcap * (size_t)(2 * dim * (precision == 32 ? 4 : 8) + 1) + 16;
}

void launch_damp_colour(const DeviceBody &db, const StepParams &p, int precision, int colour, bool forward,
                        double eta_t, hipStream_t s)
{
    DampArgs A;
    A.X = db.X;
    A.v = db.v;
    A.clamped = db.clamped;
    A.row_ptr = db.row_ptr;
    A.dslot = db.dslot;
    A.cell_start = db.cell_start;
    A.st = db.st;
    A.n = db.n;
    A.g = db.gd;
    A.hcap = db.halo_max;
    A.h_inv = p.inv_h;
    A.kfac = p.kfac;
    A.vol = p.vol;
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
    const size_t lds = damp_lds_bytes(db.dim, precision, db.halo_max);
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
