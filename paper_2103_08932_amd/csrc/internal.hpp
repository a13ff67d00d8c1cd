// internal.hpp -- device layout of a body and the kernel launchers shared by the library's
// translation units (setup.hip, step.hip, damp.hip, api.hip).  Not part of the C ABI.
//
// Layout in HBM (internal order = particles sorted by cell id, stable in the input index):
//   X        double [dim][n]        reference positions (SoA)
//   u        double [dim][n]        displacement u = x - X0, FP64 in both precisions
//   v        Real   [dim][n]        velocity
//   B0       Real   [dim*dim][n]    correction matrix of Eq. 9 (row-major entries as planes)
//   T        Real   [dim*dim][n]    T = P B0 of the current step
//   accel    Real   [dim][n]        per-particle load added to g (optional)
//   clamped  uint8  [n]
//   row_ptr  int64  [n+1], col int32 [nnz]   CSR neighbour rows, ascending
//   hslot_a, hslot_b, dslot uint16 [nnz]      halo slots of the CSR entries (bricks.hpp)
//   uh       double [dim][n]        displacement at the half step
//   cell_start int32 [ncell+1]               particles of cell c: [cell_start[c], cell_start[c+1])
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bricks.hpp"

namespace tlsph {

constexpr int kMaxRow = 128;            // damping pass: a row is split over 16 lanes x up to 8 pairs
// Bodies with more than kTwoStageMin pass-B and pass-C block partials reduce them in two stages,
// kFinishGroups workgroups and then the finish (no body the server batches has that many).
constexpr int kFinishGroups = 256;
constexpr int64_t kTwoStageMin = 65536;
constexpr int kMaxCell = 31;            // damping pass: particles of one cell
constexpr int kMaxHalo = 2048;          // particles in the 3^dim cells around one cell
constexpr int kSlotPad = 128;           // padding entries after the pass A / B slot arrays
constexpr int kBlock = 256;             // threads per block of the per-particle passes
constexpr int kPairwise = 0;            // damping schemes: pairwise splitting (Sec. 3.2)
constexpr int kParticle = 1;            // particle-by-particle splitting (Sec. 3.1)

// Scalars of one body that live on the device and are updated by the step kernels.
struct DevState {
    double dt;          // time step of the step being executed (set by the previous finish)
    double ek;          // kinetic energy after the last step
    double ek_peak;     // max E_k so far
    double resid;       // window residual after the last step
    double fres;        // force residual diagnostic of the last step
    double amax;        // max |a| over free particles (last S_m)
    double vmax;        // max |v| over free particles (end of last step)
    double tol;         // stop threshold (relax mode)
    int64_t step;       // body step index (steps completed)
    int64_t win;        // residual window W
    int64_t win_fill;
    int64_t win_pos;
    int32_t done;       // nonzero: skip the remaining enqueued steps
    int32_t error;      // nonzero: tlsph_status of a device-detected failure
    int32_t stop_on_converge;
    int32_t bad_stress; // pass A saw J <= 0 or a non-finite stress
    int64_t max_step;   // finish marks the body done once step reaches this
    int64_t win_start;  // step index at the last reset of the residual tracking
    int64_t last_high;  // latest step whose E_k / E_peak was >= tol (win_start if none since)
    double ek_turn;     // E_peak when E_k first fell below it since the last reset (0 before)
};

// Per-body constants of the step.
struct StepParams {
    int64_t n;
    double h;           // smoothing length
    double inv_h;
    double kfac;        // -5 a_D / h^2 : grad W = kfac (1 - q/2)^3 (X_i - X_j)
    double vol;         // V0 = dp^dim
    double mass;        // m = rho0 V0
    double rho0;
    double lam, mu;     // Lame constants
    double c;           // sound speed sqrt(K / rho0)
    double bsq;         // sum over free particles of |b|^2 (force-residual denominator)
    double g[3];        // uniform body force
    double dt_visc;     // viscous time-step limit of Eq. 35 (particle-by-particle damping), else infinity
    double div_factor;  // blow-up: a step with E_k > div_factor * DevState::ek_turn fails (TLSPH_E_DIVERGED)
    int model;          // 0 SVK, 1 neo-Hookean
    int has_accel;
};

struct DeviceBody {
    int dim;
    int64_t n, nnz;
    int32_t nc[3];
    int64_t ncell;
    double *X, *u;
    void *v, *B0, *T, *accel;
    uint8_t *clamped;
    int64_t *row_ptr;
    int32_t *col;
    int32_t *cell_start;
    double *partB;      // per block: amax, sum |a|^2
    double *partC;      // per block: ek sum, ek compensation, vmax, nonfinite flag
    double *partF;      // [kFinishGroups][8] or null: first-stage results of the two-stage finish
    double *win_buf;    // residual window ring
    DevState *st;
    int nblocks;
    int halo_max;       // largest 3^dim-cell neighbourhood (particles)
    int row_max;        // longest CSR row
    double *uh;         // displacement at the half step (written by pass A, read by pass C)
    uint16_t *hslot_a;  // per CSR entry: halo slot in the neighbourhood of i's brick of pass A
    uint16_t *hslot_b;  // the same for the bricks of pass B (hslot_a when both passes use one geometry)
    int32_t *brick_lmax_a;  // per brick of ga: the longest row of its own particles
    int32_t *brick_lmax_b;  // per brick of gb (brick_lmax_a when both passes use one geometry)
    int32_t *runs_a;    // run descriptors of the bricks of ga (ga.runs)
    int32_t *runs_b;    // the same for gb (runs_a when both passes use one geometry)
    uint16_t *dslot;    // per CSR entry: halo slot in the neighbourhood of i's cell (damping)
    int32_t *dorder;    // [ncell]: the cells of each colour (colours ascending) in the order the damping
                        // launches take them: within windows of consecutive cells, most particles first
    uint64_t *dtouch;   // [ncell][16] or null: compact damping neighbourhoods (bit k of lane l's word:
                        // slot 16 k + l is read by the cell's visits and staged); dslot then holds
                        // compact slots
    int32_t *downr;     // [ncell] with dtouch: compact slot of the cell's first own particle
    int halo_damp;      // damping LDS capacity per cell: the largest (compact) neighbourhood
    CMapWord *cmap;     // compact brick neighbourhoods of pass B (or null; gb.cmap), its slots in hslot_b
    BrickGeom ga, gb;   // bricks of pass A (and of the von Mises output) and of pass B
    BrickGeom gd;       // single-cell bricks of the damping pass
    int halo_a, halo_b; // largest brick neighbourhood of pass A and of pass B
    void *gdamp;        // Real [nnz]: 2 V^2 (dW/dr) / r of every CSR entry (damping)
    void *gradsum;      // Real [dim][n]: sum over the row of grad0 W_ij / kfac (pass B)
    int cell_max;       // most particles in one cell
    int cell_pairs_max; // most CSR entries of the particles of one cell
};

// Colour blocks of the splitting cell-linked list (Sec. 3.4).  Colour k -> residues of the cell
// coordinates: 3D k = 9 (cx mod 3) + 3 (cy mod 3) + cz mod 3, 2D k = 3 (cx mod 3) + cy mod 3.
__host__ __device__ inline void colour_axes(int dim, int colour, int &kx, int &ky, int &kz)
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
__host__ __device__ inline int count_mod3(int ncell, int k) { return ncell > k ? (ncell - k + 2) / 3 : 0; }
// Cells per axis of colour (kx, ky, kz) and their number.
__host__ __device__ inline void colour_cells(const int32_t (&nc)[3], int dim, int kx, int ky, int kz, int &nby,
                                             int &nbz, int &ncells)
{
    const int nbx = count_mod3(nc[0], kx);
    nby = count_mod3(nc[1], ky);
    nbz = dim == 3 ? count_mod3(nc[2], kz) : 1;
    ncells = nbx * nby * nbz;
}
// Position of colour `colour`'s first cell in the damping cell order (colours ascending).
__host__ __device__ inline int colour_offset(const int32_t (&nc)[3], int dim, int colour)
{
    int off = 0;
    for (int c = 0; c < colour; ++c) {
        int kx, ky, kz, nby, nbz, ncells;
        colour_axes(dim, c, kx, ky, kz);
        colour_cells(nc, dim, kx, ky, kz, nby, nbz, ncells);
        off += ncells;
    }
    return off;
}

// One body of a batched launch: everything the step kernels read from a DeviceBody and its
// StepParams, gathered so that a kernel can serve several bodies of different sizes.
struct Inst {
    StepParams P;
    BrickGeom ga, gb, gd;
    int32_t nc[3];
    int halo_a, halo_b, halo_max;
    int row_max;
    int nbA, nbB;       // bricks of pass A and of pass B
    int nbC;            // blocks of pass C
    double eta_t;       // eta / alpha of the damping pass
    int scheme;         // kPairwise or kParticle
    const int32_t *cell_start;
    const double *X;
    double *u, *uh;
    void *v;
    const void *B0;
    void *T;
    const void *accel;
    const uint8_t *clamped;
    const int64_t *row_ptr;
    const uint16_t *hslot_a, *hslot_b, *dslot;
    const int32_t *dorder;
    const uint64_t *dtouch;
    const int32_t *downr;
    int halo_damp;
    const int32_t *brick_lmax_a, *brick_lmax_b;
    const void *gdamp;
    const void *gradsum;
    double *partB, *partC, *win_buf;
    DevState *st;
};

// Launch table of a batched launch (passed by value): workgroup w of the launch (after the XCD
// remap) serves body inst[k] for start[k] <= w < start[k + 1], as its local block w - start[k].
constexpr int kMaxBatch = 64;
struct BatchMap {
    int count;
    int inst[kMaxBatch];
    int start[kMaxBatch + 1];
};

__host__ __device__ inline int batch_find(const BatchMap &M, int w)
{
    int lo = 0, hi = M.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (w >= M.start[mid]) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---- setup (setup.hip) ----
struct SetupScratch;
// Builds perm/order, X, clamped, cell_start, row_ptr, col, B0 of `db` from input-order host
// data already copied to the device (X0_in, clamped_in).  Returns 0 or a tlsph_status.
int setup_topology(DeviceBody &db, int precision, const double *X0_in_dev, const uint8_t *clamped_in_dev,
                   const double xmin[3], double rc, double rc2, double h, double vol,
                   int32_t *perm_out_dev, void *(*alloc)(size_t, void *), void (*dfree)(void *, void *),
                   void *actx, hipStream_t s, char *errmsg, size_t errlen);

// ---- step passes (step.hip) ----
void launch_passA(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s);
// Von Mises stress of every particle for the current u into vm (device, n doubles, internal order).
void launch_von_mises(const DeviceBody &db, const StepParams &p, int precision, double *vm, hipStream_t s);
void launch_passB(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s);
void launch_passC(const DeviceBody &db, const StepParams &p, int precision, hipStream_t s);
void launch_finish(const DeviceBody &db, const StepParams &p, hipStream_t s);
// Computes dt of the next step from the current v (max |v|) and max |b| (Eq. 18 at n = 0).
void launch_init_dt(const DeviceBody &db, const StepParams &p, int precision, double bmax, double dt_given,
                    hipStream_t s);

// ---- damping pass (damp.hip) ----
// One colour launch of the damping sweep (scheme kPairwise or kParticle); forward = true for the
// forward global sweep.
void launch_damp_colour(const DeviceBody &db, const StepParams &p, int precision, int scheme, int colour, bool forward,
                        double eta_t, hipStream_t s);

// ---- batched launches over a table of bodies of one dimension and precision ----
// `I` is the device copy of the table; `h` its host copy (grid sizes and LDS are taken from it);
// `slots` are the table rows served by the launch.
void launch_passA_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s);
void launch_passB_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s);
void launch_passC_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision,
                        hipStream_t s);
void launch_finish_batch(const Inst *I, const int *slots, int count, hipStream_t s);
void launch_damp_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int precision, int colour,
                       bool forward, hipStream_t s);
// Copies the DevState of every table row in `slots` to out[0 .. count).
void launch_gather_state(const Inst *I, const int *slots, int count, DevState *out, hipStream_t s);
// Arms a run (stop flags, stop rule, latest high step of the stored window for this tol).
void launch_control(DevState *st, const double *win_buf, int stop_on_converge, double tol, int64_t max_step,
                    hipStream_t s);
// Window residual of the stored steps -> DevState::resid.
void launch_resid(const DeviceBody &db, hipStream_t s);
int damp_pairs_per_lane(int row_max);

}  // namespace tlsph
