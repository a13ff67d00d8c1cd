/*
 * tlsph_oracle.c -- plain, slow FP64 CPU oracle for the splitting random-choice dynamic
 * relaxation of total Lagrangian SPH (Zhu, Zhang & Hu, arXiv:2103.08932).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or constant with the
 * HIP library; the two are fed from the same seeded input generators and nothing else.
 *
 * Everything is double precision and the file is compiled with -ffp-contract=off so that every
 * multiply and add is rounded on its own.  The step follows the paper's algorithm in its own
 * order and notation:
 *
 *   Sec. 2.2  Eqs. 9-10   kernel-correction matrix B0 and reference gradient grad0 W
 *   Sec. 2.1  Eqs. 2-8    F = I + grad0 u, P = F S, S from St Venant-Kirchhoff or neo-Hookean
 *   Sec. 2.2  Eqs. 12-13  pairwise force with the averaged P B0
 *   Sec. 2.3  Eqs. 15-18  position-based Verlet and the acoustic / body-force time step
 *   Sec. 3    Eqs. 24-25  Lie-Trotter split S_d o S_m; particle-by-particle Strang sweep
 *   Sec. 3.1  Eqs. 26-35  particle-by-particle D_i: one gradient step on the implicit local system,
 *                         then the momentum-conserving neighbour update; viscous time-step limit
 *   Sec. 3.2  Eqs. 37-39  pairwise Strang split of D_i and the closed-form two-body implicit solve
 *   Sec. 3.3  Eq. 40      random choice: damp with eta/alpha on a fraction alpha of the steps
 *   Sec. 3.4              splitting cell-linked list: cells of size r_c, 3^D colour blocks swept
 *                         one after another (forward), then in reverse (backward)
 *   Sec. 4.2  Eq. 41      von Mises stress of the Cauchy stress J^-1 F S F^T (the output of the
 *                         twisting example; plane strain in 2D)
 *
 * Readings where the paper is silent or garbled (each is also listed in the design notes):
 *   - Wendland C2 kernel with support 2h, normalisation 7/(4 pi h^2) (2D), 21/(16 pi h^3) (3D).
 *   - Damp iff phi < alpha (Eq. 40 as printed says alpha < phi, which contradicts alpha = 1
 *     meaning "damp every step" and the ~20 % cost at alpha = 0.2).  phi comes from
 *     Philox4x64-10, key (seed, 0), counter (step, 0, 0, 0), word 0: damped iff
 *     (w0 >> 40) < ceil(alpha * 2^24).
 *   - Nested Strang: each D_i(dt/2) visits its row forward then backward, each pair visit
 *     integrating dt/4 (Eq. 37 inside Eq. 25).  Rows are full (i sees j and j sees i).
 *   - Clamped particles keep u = v = 0, have rows, F, P and T (they feed T_j), and act as
 *     infinite masses in the pair solve; clamped-clamped pairs are skipped.
 *   - E = 2 mu (1 + nu) (Eq. 6 as printed has 1 + 2 nu).  2D is plane strain.
 *   - The damping operator is applied after the kick and before the second half drift.
 *   - Particle-by-particle scheme: a clamped neighbour's velocity is not a variable of the local
 *     system; a clamped particle's visit damps each free neighbour against the wall by the exact
 *     one-neighbour solution m v_j / (m - B_j).  Eq. 35 uses the kinematic viscosity eta / rho0 with
 *     eta (not eta / alpha) and D = dimension; it limits every step's dt, not the window length.
 *     The scheme as printed is only conditionally stable (the pairwise scheme is the
 *     unconditionally stable one): at this limit with alpha = 1 a nearest neighbour's |B_j| / m is
 *     about 10 in 2D and 4 in 3D (1 / alpha times more on a random-choice damped step), where the
 *     predicted-velocity correction can amplify; no further limit is added.
 *   - Convergence residual: max over the last W steps of E_k / E_peak, W = ceil(T_w / dt0),
 *     T_w = L_max^2 / (L_min c); stop when it is below tol and at least W steps were taken.
 *
 * Shared-memory mode (the paper's own parallelisation, Sec. 3.4): with OpenMP the per-particle
 * loops (neighbour rows, B0, F / stress / T, the pair-force sum) run over particles in parallel, and
 * the damping sweep runs the cells of one colour block in parallel (their neighbourhoods are
 * disjoint, so the writes are).  Every particle's arithmetic is the same sequence as in the serial
 * order and the order-dependent sums (E_k and the force residual) stay serial, so the results are
 * bit-identical for any thread count (orc_set_threads; 1 = the plain serial oracle).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_E_INVALID (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_SINGULAR (-3)
#define ORC_E_NONFINITE (-5)
#define ORC_E_DIVERGED (-6)

#define ORC_SVK 0
#define ORC_NH 1

#define ORC_PAIRWISE 0
#define ORC_PARTICLE 1

typedef struct orc_body {
    int dim;
    int64_t n;
    double dp, h, rc, rc2, vol, mass, rho0;
    double xmin[3];
    int64_t nc[3];
    int64_t ncell;
    /* internal (cell-sorted) order */
    int64_t *perm;       /* internal -> input index */
    int64_t *iperm;      /* input -> internal index */
    int64_t *cell;       /* linear cell id of each internal particle */
    int64_t *cell_start; /* ncell + 1 */
    int64_t ncolour;
    int64_t *colour_start; /* ncolour + 1, offsets into colour_cells */
    int64_t *colour_cells; /* cells of each colour, ascending */
    int64_t *row_ptr;    /* n + 1 */
    int64_t *col;        /* row_ptr[n] */
    double *X;           /* n * dim */
    double *B0;          /* n * dim * dim, row-major */
    unsigned char *clamped;
    double *u, *v, *T, *acc, *bf;
    /* material */
    int model;
    double E, nu, lam, mu, K, c;
    int material_set;
    /* damping */
    double eta, alpha;
    uint64_t seed;
    int scheme;          /* ORC_PAIRWISE (Sec. 3.2) or ORC_PARTICLE (Sec. 3.1) */
    /* loads */
    double bmax;
    /* step state */
    int64_t step;
    double dt;           /* dt of the next step; <= 0 means "derive from max|v|, max|b|" */
    double amax_prev;
    double ek_peak, ek_last, resid_last, fres_last;
    double ek_turn;      /* E_peak when E_k first fell below it since the reset (0 before) */
    double div_factor;   /* blow-up: E_k > div_factor * ek_turn */
    double *ek_win;
    int64_t win, win_fill, win_pos;
    double extent_min, extent_max;
} orc_body;

/* ------------------------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4x64 Philox S-box with   */
/* the published multipliers and Weyl key increments.                                          */
/* ------------------------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Eq. 40 (reading above): is step n of the body keyed by seed a damped step? */
int orc_damped_decision(uint64_t seed, int64_t n, double alpha)
{
    if (alpha >= 1.0) return 1;
    if (alpha <= 0.0) return 0;
    uint64_t ctr[4] = {(uint64_t)n, 0, 0, 0}, key[2] = {seed, 0}, out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t u24 = out[0] >> 40;
    uint64_t thr = (uint64_t)ceil(alpha * 16777216.0);
    return u24 < thr;
}

/* Threads of the shared-memory mode (n >= 1); returns the count in effect. */
int orc_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* Eq. 36: eta = (beta / 4) sqrt(rho0 E) L */
double orc_eta(double beta, double rho0, double E, double L)
{
    return beta / 4.0 * sqrt(rho0 * E) * L;
}

/* ------------------------------------------------------------------------------------------ */
/* Wendland C2 kernel (Sec. 4: "5th-order C2 Wendland", h = 1.3 dp; support 2h).               */
/*   W(q) = a_D (1 - q/2)^4 (1 + 2q),  dW/dr = (a_D / h) (-5 q) (1 - q/2)^3,  q = r / h         */
/* ------------------------------------------------------------------------------------------ */
static double wendland_alpha(int dim, double h)
{
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    return 21.0 / (16.0 * M_PI * h * h * h);
}

void orc_wendland(int dim, double h, double r, double *W, double *dW)
{
    double q = r / h;
    double a = wendland_alpha(dim, h);
    if (q >= 2.0) { *W = 0.0; *dW = 0.0; return; }
    double t = 1.0 - 0.5 * q;
    *W = a * t * t * t * t * (1.0 + 2.0 * q);
    *dW = a / h * (-5.0 * q) * t * t * t;
}

/* grad0_i W_ij (Eq. 10) for the pair (i, j): (dW/dr) e_ij, e_ij = (X_i - X_j) / r_ij */
static void grad_w(const orc_body *b, int64_t i, int64_t j, double g[3], double *r_out, double *dW_out)
{
    int D = b->dim;
    double d[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) d[k] = b->X[i * D + k] - b->X[j * D + k];
    double r2 = d[0] * d[0] + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    double r = sqrt(r2);
    double W, dW;
    orc_wendland(D, b->h, r, &W, &dW);
    for (int k = 0; k < 3; ++k) g[k] = 0.0;
    for (int k = 0; k < D; ++k) g[k] = dW * d[k] / r;
    if (r_out) *r_out = r;
    if (dW_out) *dW_out = dW;
}

/* ------------------------------------------------------------------------------------------ */
/* small dense helpers                                                                         */
/* ------------------------------------------------------------------------------------------ */
static double det_n(int D, const double *A)
{
    if (D == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse through the adjugate; returns the determinant */
static double inv_n(int D, const double *A, double *Ai)
{
    double det = det_n(D, A);
    if (D == 2) {
        Ai[0] = A[3] / det; Ai[1] = -A[1] / det;
        Ai[2] = -A[2] / det; Ai[3] = A[0] / det;
        return det;
    }
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return det;
}

static void matmul_n(int D, const double *A, const double *B, double *C)
{
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += A[r * D + k] * B[k * D + c];
            C[r * D + c] = s;
        }
}

/* ------------------------------------------------------------------------------------------ */
/* Constitutive laws (Sec. 2.1)                                                                */
/*   SVK  (Eqs. 4-5):  E = (F^T F - I) / 2,  S = lambda tr(E) I + 2 mu E                       */
/*   NH   (Eqs. 7-8):  S = dW/dE = mu (I - C^-1) + lambda ln J C^-1,  C = F^T F, J = det F      */
/*   P = F S (Eq. 3).  Returns 0, or ORC_E_NONFINITE when J <= 0 for the neo-Hookean law.      */
/* ------------------------------------------------------------------------------------------ */
int orc_stress(int dim, int model, double lam, double mu, const double *F, double *S, double *P)
{
    int D = dim;
    double C[9] = {0}, Ci[9] = {0};
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += F[k * D + r] * F[k * D + c];
            C[r * D + c] = s;
        }
    if (model == ORC_SVK) {
        double Eg[9], tr = 0.0;
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) Eg[r * D + c] = 0.5 * (C[r * D + c] - (r == c ? 1.0 : 0.0));
        for (int k = 0; k < D; ++k) tr += Eg[k * D + k];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) S[r * D + c] = 2.0 * mu * Eg[r * D + c] + (r == c ? lam * tr : 0.0);
    } else {
        double J = det_n(D, F);
        if (!(J > 0.0)) return ORC_E_NONFINITE;
        inv_n(D, C, Ci);
        double lnJ = log(J);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c)
                S[r * D + c] = mu * ((r == c ? 1.0 : 0.0) - Ci[r * D + c]) + lam * lnJ * Ci[r * D + c];
    }
    matmul_n(D, F, S, P);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Pair operator of the pairwise splitting scheme (Sec. 3.2, Eqs. 38-39).                      */
/*   B = eta_t * s * g_ij with g_ij = 2 V_i V_j (dW/dr) / r_ij (Eq. 27 without eta and dt)     */
/*   free-free:  dv_i =  m_j B v_ij / (m_i m_j - (m_i + m_j) B),  dv_j = -m_i B v_ij / (same)   */
/*   j clamped (m_j -> inf):  dv_i = B v_ij / (m_i - B);   i clamped:  dv_j = -B v_ij / (m_j - B)*/
/* ------------------------------------------------------------------------------------------ */
void orc_pair_op(int dim, double mi, double mj, double B, int clamped_i, int clamped_j,
                 double *vi, double *vj)
{
    if (clamped_i && clamped_j) return;
    double w[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) w[k] = vi[k] - vj[k];
    if (!clamped_i && !clamped_j) {
        double den = mi * mj - (mi + mj) * B;
        for (int k = 0; k < dim; ++k) {
            vi[k] += mj * B * w[k] / den;
            vj[k] -= mi * B * w[k] / den;
        }
    } else if (clamped_j) {
        for (int k = 0; k < dim; ++k) vi[k] += B * w[k] / (mi - B);
    } else {
        for (int k = 0; k < dim; ++k) vj[k] -= B * w[k] / (mj - B);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Body construction: cells, splitting-CLL colours, neighbour rows, B0                         */
/* ------------------------------------------------------------------------------------------ */
static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

void orc_body_destroy(orc_body *b)
{
    if (!b) return;
    free(b->perm); free(b->iperm); free(b->cell); free(b->cell_start);
    free(b->colour_start); free(b->colour_cells); free(b->row_ptr); free(b->col);
    free(b->X); free(b->B0); free(b->clamped); free(b->u); free(b->v); free(b->T);
    free(b->acc); free(b->bf); free(b->ek_win);
    free(b);
}

/* cell coordinates of a position: floor((X - Xmin) / r_c) per axis (Sec. 3.4, cell = cut-off) */
static void cell_coords(const orc_body *b, const double *x, int64_t c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (int k = 0; k < b->dim; ++k) c[k] = (int64_t)floor((x[k] - b->xmin[k]) / b->rc);
}

static int64_t cell_linear(const orc_body *b, const int64_t c[3])
{
    if (b->dim == 2) return c[0] * b->nc[1] + c[1];
    return (c[0] * b->nc[1] + c[1]) * b->nc[2] + c[2];
}

/* colour block of a cell: 3 (cx mod 3) + (cy mod 3) in 2D, 9 (cx mod 3) + 3 (cy mod 3) + (cz mod 3) in 3D */
static int64_t cell_colour(const orc_body *b, int64_t lin)
{
    if (b->dim == 2) {
        int64_t cx = lin / b->nc[1], cy = lin % b->nc[1];
        return 3 * (cx % 3) + (cy % 3);
    }
    int64_t cz = lin % b->nc[2];
    int64_t t = lin / b->nc[2];
    int64_t cy = t % b->nc[1], cx = t / b->nc[1];
    return 9 * (cx % 3) + 3 * (cy % 3) + (cz % 3);
}

static void cell_unlinear(const orc_body *b, int64_t lin, int64_t c[3])
{
    if (b->dim == 2) { c[0] = lin / b->nc[1]; c[1] = lin % b->nc[1]; c[2] = 0; return; }
    c[2] = lin % b->nc[2];
    int64_t t = lin / b->nc[2];
    c[1] = t % b->nc[1];
    c[0] = t / b->nc[1];
}

/* Visit the neighbour rows of particle i: candidates in the 3^D adjacent cells, visited in
 * ascending cell id and ascending particle index, kept when j != i and d^2 < r_c^2. */
static int64_t scan_row(const orc_body *b, int64_t i, int64_t *out)
{
    int D = b->dim;
    int64_t ci[3];
    cell_unlinear(b, b->cell[i], ci);
    int64_t cnt = 0;
    int dz_lo = (D == 3) ? -1 : 0, dz_hi = (D == 3) ? 1 : 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = dz_lo; dz <= dz_hi; ++dz) {
                int64_t cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                if (cc[0] < 0 || cc[0] >= b->nc[0] || cc[1] < 0 || cc[1] >= b->nc[1]) continue;
                if (D == 3 && (cc[2] < 0 || cc[2] >= b->nc[2])) continue;
                int64_t lin = cell_linear(b, cc);
                for (int64_t j = b->cell_start[lin]; j < b->cell_start[lin + 1]; ++j) {
                    if (j == i) continue;
                    double d0 = b->X[j * D + 0] - b->X[i * D + 0];
                    double d1 = b->X[j * D + 1] - b->X[i * D + 1];
                    double d2 = (D == 3) ? b->X[j * D + 2] - b->X[i * D + 2] : 0.0;
                    double r2 = d0 * d0 + d1 * d1;
                    r2 = r2 + d2 * d2;
                    if (r2 < b->rc2) {
                        if (out) out[cnt] = j;
                        ++cnt;
                    }
                }
            }
    return cnt;
}

static void recompute_limits(orc_body *b);

/* Create a body from the reference configuration X0 (input order, n x dim) and clamp flags.
 * h = h_over_dp * dp, r_c = 2 h.  Returns NULL and sets *status on failure. */
orc_body *orc_body_create(int dim, int64_t n, const double *X0, const unsigned char *clamped, double dp,
                          double h_over_dp, double rho0, int *status)
{
    *status = ORC_E_INVALID;
    if ((dim != 2 && dim != 3) || n < 1 || !X0 || !(dp > 0.0) || !(h_over_dp > 0.0) || !(rho0 > 0.0))
        return NULL;
    orc_body *b = (orc_body *)calloc(1, sizeof(orc_body));
    if (!b) { *status = ORC_E_NOMEM; return NULL; }
    int D = dim;
    b->dim = dim; b->n = n; b->dp = dp; b->rho0 = rho0;
    b->h = h_over_dp * dp;
    b->rc = 2.0 * b->h;
    b->rc2 = b->rc * b->rc;
    b->vol = (D == 2) ? dp * dp : dp * dp * dp;
    b->mass = rho0 * b->vol;
    b->alpha = 1.0;
    b->model = ORC_NH;
    b->div_factor = 1e6;

    /* bounding box and cell grid */
    double xmax[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) { b->xmin[k] = X0[k]; xmax[k] = X0[k]; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < D; ++k) {
            double x = X0[i * D + k];
            if (!isfinite(x)) { free(b); return NULL; }
            if (x < b->xmin[k]) b->xmin[k] = x;
            if (x > xmax[k]) xmax[k] = x;
        }
    b->nc[0] = b->nc[1] = b->nc[2] = 1;
    for (int k = 0; k < D; ++k) b->nc[k] = (int64_t)floor((xmax[k] - b->xmin[k]) / b->rc) + 1;
    b->ncell = b->nc[0] * b->nc[1] * b->nc[2];
    b->extent_min = 1e300; b->extent_max = 0.0;
    for (int k = 0; k < D; ++k) {
        double e = (xmax[k] - b->xmin[k]) + dp;
        if (e < b->extent_min) b->extent_min = e;
        if (e > b->extent_max) b->extent_max = e;
    }

    /* stable counting sort of particles by cell id (ties keep input order) */
    int64_t *cell_in = (int64_t *)xcalloc(n, sizeof(int64_t));
    b->cell_start = (int64_t *)xcalloc(b->ncell + 1, sizeof(int64_t));
    b->perm = (int64_t *)xcalloc(n, sizeof(int64_t));
    b->iperm = (int64_t *)xcalloc(n, sizeof(int64_t));
    b->cell = (int64_t *)xcalloc(n, sizeof(int64_t));
    if (!cell_in || !b->cell_start || !b->perm || !b->iperm || !b->cell) {
        free(cell_in); orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        cell_coords(b, &X0[i * D], c);
        cell_in[i] = cell_linear(b, c);
        b->cell_start[cell_in[i] + 1] += 1;
    }
    for (int64_t c = 0; c < b->ncell; ++c) b->cell_start[c + 1] += b->cell_start[c];
    {
        int64_t *fill = (int64_t *)xcalloc(b->ncell, sizeof(int64_t));
        if (!fill) { free(cell_in); orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = cell_in[i];
            int64_t pos = b->cell_start[c] + fill[c]++;
            b->perm[pos] = i;
        }
        free(fill);
    }
    free(cell_in);

    b->X = (double *)xcalloc((size_t)n * D, sizeof(double));
    b->clamped = (unsigned char *)xcalloc(n, 1);
    if (!b->X || !b->clamped) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
    for (int64_t p = 0; p < n; ++p) {
        int64_t i = b->perm[p];
        b->iperm[i] = p;
        for (int k = 0; k < D; ++k) b->X[p * D + k] = X0[i * D + k];
        b->clamped[p] = clamped ? (clamped[i] != 0) : 0;
        int64_t c[3];
        cell_coords(b, &b->X[p * D], c);
        b->cell[p] = cell_linear(b, c);
    }

    /* colour blocks: cells of each colour in ascending id */
    b->ncolour = (D == 2) ? 9 : 27;
    b->colour_start = (int64_t *)xcalloc(b->ncolour + 1, sizeof(int64_t));
    b->colour_cells = (int64_t *)xcalloc(b->ncell, sizeof(int64_t));
    if (!b->colour_start || !b->colour_cells) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
    for (int64_t c = 0; c < b->ncell; ++c) b->colour_start[cell_colour(b, c) + 1] += 1;
    for (int64_t k = 0; k < b->ncolour; ++k) b->colour_start[k + 1] += b->colour_start[k];
    {
        int64_t *fill = (int64_t *)xcalloc(b->ncolour, sizeof(int64_t));
        for (int64_t c = 0; c < b->ncell; ++c) {
            int64_t k = cell_colour(b, c);
            b->colour_cells[b->colour_start[k] + fill[k]++] = c;
        }
        free(fill);
    }

    /* neighbour rows: count, then fill */
    b->row_ptr = (int64_t *)xcalloc(n + 1, sizeof(int64_t));
    if (!b->row_ptr) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) b->row_ptr[i + 1] = scan_row(b, i, NULL);
    for (int64_t i = 0; i < n; ++i) b->row_ptr[i + 1] += b->row_ptr[i];
    b->col = (int64_t *)xcalloc(b->row_ptr[n], sizeof(int64_t));
    if (!b->col) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) scan_row(b, i, &b->col[b->row_ptr[i]]);

    /* kernel-correction matrix, Eq. 9:  B0_i = ( - sum_j V_j (X_i - X_j) (x) grad0_i W_ij )^-1 */
    b->B0 = (double *)xcalloc((size_t)n * D * D, sizeof(double));
    if (!b->B0) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
    int singular = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        double nrm = 0.0;
        for (int64_t e = b->row_ptr[i]; e < b->row_ptr[i + 1]; ++e) {
            int64_t j = b->col[e];
            double g[3];
            grad_w(b, i, j, g, NULL, NULL);
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c)
                    M[r * D + c] -= b->vol * (b->X[i * D + r] - b->X[j * D + r]) * g[c];
        }
        for (int k = 0; k < D * D; ++k) nrm = fmax(nrm, fabs(M[k]));
        double det = det_n(D, M);
        if (!(fabs(det) > 1e-12 * pow(nrm, D)) || nrm == 0.0) {
#pragma omp atomic write
            singular = 1;
            continue;
        }
        inv_n(D, M, &b->B0[i * D * D]);
    }
    if (singular) { orc_body_destroy(b); *status = ORC_E_SINGULAR; return NULL; }

    b->u = (double *)xcalloc((size_t)n * D, sizeof(double));
    b->v = (double *)xcalloc((size_t)n * D, sizeof(double));
    b->T = (double *)xcalloc((size_t)n * D * D, sizeof(double));
    b->acc = (double *)xcalloc((size_t)n * D, sizeof(double));
    b->bf = (double *)xcalloc((size_t)n * D, sizeof(double));
    if (!b->u || !b->v || !b->T || !b->acc || !b->bf) { orc_body_destroy(b); *status = ORC_E_NOMEM; return NULL; }
    b->dt = 0.0;
    *status = ORC_OK;
    return b;
}

/* ------------------------------------------------------------------------------------------ */
/* Parameters                                                                                  */
/* ------------------------------------------------------------------------------------------ */
static void reset_tracking(orc_body *b)
{
    b->ek_peak = 0.0; b->ek_last = 0.0; b->resid_last = 1.0; b->ek_turn = 0.0;
    b->win_fill = 0; b->win_pos = 0;
}

/* Lame constants from E and nu (E = 2 mu (1 + nu)), bulk modulus K = lambda + 2 mu / 3 (Eq. 6)
 * and the sound speed c = sqrt(K / rho0) of Eq. 18. */
int orc_body_set_material(orc_body *b, int model, double E, double nu)
{
    if (!b || (model != ORC_SVK && model != ORC_NH) || !(E >= 0.0) || !(nu > -1.0 && nu < 0.5))
        return ORC_E_INVALID;
    b->model = model; b->E = E; b->nu = nu;
    b->lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    b->mu = E / (2.0 * (1.0 + nu));
    b->K = b->lam + 2.0 * b->mu / 3.0;
    b->c = sqrt(b->K / b->rho0);
    b->material_set = 1;
    b->dt = 0.0;
    recompute_limits(b);
    reset_tracking(b);
    return ORC_OK;
}

/* Body force per particle: g (every particle) plus an optional per-particle acceleration
 * (input order, n x dim). */
int orc_body_set_loads(orc_body *b, const double *g, const double *accel)
{
    if (!b || !g) return ORC_E_INVALID;
    int D = b->dim;
    for (int64_t p = 0; p < b->n; ++p) {
        int64_t i = b->perm[p];
        for (int k = 0; k < D; ++k) b->bf[p * D + k] = g[k] + (accel ? accel[i * D + k] : 0.0);
    }
    b->dt = 0.0;
    recompute_limits(b);
    reset_tracking(b);
    return ORC_OK;
}

/* eta <= 0 selects the Eq. 36 value from (beta, Lc). */
int orc_body_set_damping(orc_body *b, double eta, double beta, double Lc, double alpha, uint64_t seed)
{
    if (!b || !(alpha > 0.0 && alpha <= 1.0)) return ORC_E_INVALID;
    if (eta <= 0.0) {
        if (!b->material_set || !(beta >= 0.0) || !(Lc >= 0.0)) return ORC_E_INVALID;
        eta = orc_eta(beta, b->rho0, b->E, Lc);
    }
    b->eta = eta; b->alpha = alpha; b->seed = seed;
    return ORC_OK;
}

double orc_body_eta(const orc_body *b) { return b->eta; }

/* Damping scheme: ORC_PAIRWISE (Sec. 3.2, Eqs. 37-39) or ORC_PARTICLE (Sec. 3.1, Eqs. 26-34). */
int orc_body_set_damping_scheme(orc_body *b, int scheme)
{
    if (!b || (scheme != ORC_PAIRWISE && scheme != ORC_PARTICLE)) return ORC_E_INVALID;
    b->scheme = scheme;
    return ORC_OK;
}

/* Divergence detection (not in the paper, which relaxes to fixed end times): a step whose kinetic
 * energy exceeds `factor` times the peak E_k had reached when it first fell again (since the last
 * reset of the tracking) fails with ORC_E_DIVERGED.  factor > 0; the default is 1e6. */
int orc_body_set_divergence(orc_body *b, double factor)
{
    if (!b || !(factor > 0.0)) return ORC_E_INVALID;
    b->div_factor = factor;
    return ORC_OK;
}

static double vnorm(int D, const double *x)
{
    double s = x[0] * x[0] + x[1] * x[1];
    if (D == 3) s = s + x[2] * x[2];
    return sqrt(s);
}

/* Window length of the residual and max|b| over free particles. */
static void recompute_limits(orc_body *b)
{
    int D = b->dim;
    double bmax = 0.0;
    for (int64_t p = 0; p < b->n; ++p)
        if (!b->clamped[p]) bmax = fmax(bmax, vnorm(D, &b->bf[p * D]));
    b->bmax = bmax;
    if (!b->material_set) return;
    double dt0 = HUGE_VAL;
    if (b->c > 0.0) dt0 = b->h / b->c;
    if (bmax > 0.0) dt0 = fmin(dt0, sqrt(b->h / bmax));
    dt0 *= 0.6;
    int64_t W = 1;
    if (b->c > 0.0 && isfinite(dt0)) {
        double Tw = b->extent_max * b->extent_max / (b->extent_min * b->c);
        W = (int64_t)ceil(Tw / dt0);
        if (W < 1) W = 1;
    }
    if (W != b->win) {
        free(b->ek_win);
        b->ek_win = (double *)xcalloc(W, sizeof(double));
        b->win = W;
    }
    b->win_fill = 0; b->win_pos = 0;
}

int64_t orc_body_window(const orc_body *b) { return b->win; }

/* Eq. 18: dt = 0.6 min(h / (c + |v|max), sqrt(h / |dv/dt|max)) over free particles; with the
 * particle-by-particle scheme also the viscous limit of Eq. 35, dt <= 50 h^2 / (nu D) with the
 * kinematic viscosity nu = eta / rho0 of Eq. 19 (eta, not eta / alpha). */
static double time_step(const orc_body *b, double vmax, double amax)
{
    double t1 = (b->c + vmax > 0.0) ? b->h / (b->c + vmax) : HUGE_VAL;
    double t2 = (amax > 0.0) ? sqrt(b->h / amax) : HUGE_VAL;
    double dt = 0.6 * fmin(t1, t2);
    if (b->scheme == ORC_PARTICLE && b->eta > 0.0) {
        double nu_k = b->eta / b->rho0;
        dt = fmin(dt, 50.0 * b->h * b->h / (nu_k * b->dim));
    }
    return dt;
}

static double max_free_speed(const orc_body *b)
{
    double m = 0.0;
    for (int64_t p = 0; p < b->n; ++p)
        if (!b->clamped[p]) m = fmax(m, vnorm(b->dim, &b->v[p * b->dim]));
    return m;
}

/* ------------------------------------------------------------------------------------------ */
/* S_m: deformation gradient, stress, T = P B0, pairwise force (Eqs. 2-13)                     */
/* ------------------------------------------------------------------------------------------ */
/* F_i = I + ( sum_j V (u_j - u_i) (x) grad0_i W_ij ) B0_i   (total form of Eq. 14 for fixed X0) */
static void deformation_gradient(const orc_body *b, int64_t i, double *F)
{
    int D = b->dim;
    double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = b->row_ptr[i]; e < b->row_ptr[i + 1]; ++e) {
        int64_t j = b->col[e];
        double g[3];
        grad_w(b, i, j, g, NULL, NULL);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) G[r * D + c] += b->vol * (b->u[j * D + r] - b->u[i * D + r]) * g[c];
    }
    matmul_n(D, G, &b->B0[i * D * D], F);
    for (int k = 0; k < D; ++k) F[k * D + k] += 1.0;
}

static int compute_T(orc_body *b)
{
    int D = b->dim;
    int status = ORC_OK;   /* orc_stress fails only with ORC_E_NONFINITE */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < b->n; ++i) {
        double F[9], S[9], P[9];
        deformation_gradient(b, i, F);
        int st = orc_stress(D, b->model, b->lam, b->mu, F, S, P);
        if (st != ORC_OK) {
#pragma omp atomic write
            status = st;
            continue;
        }
        matmul_n(D, P, &b->B0[i * D * D], &b->T[i * D * D]);
    }
    return status;
}

/* Eq. 12:  dv_i/dt = (1/rho0) sum_j V (T_i + T_j) grad0_i W_ij + b_i   (T = P B0, Eq. 13) */
static void compute_accel(orc_body *b)
{
    int D = b->dim;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < b->n; ++i) {
        double a[3] = {0, 0, 0};
        for (int64_t e = b->row_ptr[i]; e < b->row_ptr[i + 1]; ++e) {
            int64_t j = b->col[e];
            double g[3];
            grad_w(b, i, j, g, NULL, NULL);
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c)
                    a[r] += b->vol * (b->T[i * D * D + r * D + c] + b->T[j * D * D + r * D + c]) * g[c];
        }
        for (int r = 0; r < D; ++r) b->acc[i * D + r] = a[r] / b->rho0 + b->bf[i * D + r];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* S_d: pairwise implicit damping swept over the splitting cell-linked list (Secs. 3.2-3.4)     */
/* ------------------------------------------------------------------------------------------ */
/* D_i(tau): row forward then row backward, each pair visit integrating tau / 2 (Eq. 37). */
static void damp_particle(orc_body *b, int64_t i, double eta_t, double tau)
{
    int D = b->dim;
    double s = 0.5 * tau;
    int64_t lo = b->row_ptr[i], hi = b->row_ptr[i + 1];
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t q = 0; q < hi - lo; ++q) {
            int64_t e = (pass == 0) ? lo + q : hi - 1 - q;
            int64_t j = b->col[e];
            double g[3], r, dW;
            grad_w(b, i, j, g, &r, &dW);
            double gij = 2.0 * b->vol * b->vol * dW / r;
            double B = eta_t * s * gij;
            orc_pair_op(D, b->mass, b->mass, B, b->clamped[i], b->clamped[j], &b->v[i * D], &b->v[j * D]);
        }
    }
}

/* D_i(tau) of the particle-by-particle scheme (Sec. 3.1): the implicit local system of Eq. 29
 *     E_i = (sum_j B_j - m_i) dv_i - sum_j B_j dv_j,   B_j = 2 eta V_i V_j (dW/dr) / r tau  (Eq. 27),
 *     E_i = -sum_j B_j (v_i - v_j)                                                   (Eq. 28)
 * is met by one gradient step dv = k grad E_i (Eqs. 30-32), k = E_i / ((sum B - m_i)^2 + sum B_j^2)
 * (Eq. 32); v_i takes its increment, the neighbours their predictions v_j^p = v_j - B_j k (Eq. 33),
 * and each neighbour then gets the momentum-conserving update v_j <- v_j - B_j (v_i^new - v_j^p) / m_j
 * (Eq. 34).  Reading for clamped particles (infinite mass, never moving): a clamped neighbour's
 * velocity is not a variable (its B_j enters sum B and E_i but not sum B_j^2, and it is not updated);
 * the visit of a clamped i damps each free neighbour j against it exactly as the scheme treats a
 * particle whose only neighbour is a wall, v_j <- m v_j / (m - B_j), so every pair, wall pairs
 * included, acts from both of its ends as in the interior. */
/* The local update of D_i alone: particle i (velocity vi, mass m) and its nb neighbours (velocities
 * vj[q * dim ..], coefficients Bj[q], clamped flags cj[q]); vi and vj are updated in place. */
void orc_pbp_local(int dim, double m, int64_t nb, const double *Bj, const unsigned char *cj, double *vi, double *vj)
{
    double sB = 0.0, sB2 = 0.0, E[3] = {0.0, 0.0, 0.0};
    for (int64_t q = 0; q < nb; ++q) {
        sB += Bj[q];
        if (!cj[q]) sB2 += Bj[q] * Bj[q];
        for (int k = 0; k < dim; ++k) E[k] -= Bj[q] * (vi[k] - vj[q * dim + k]);
    }
    double den = (sB - m) * (sB - m) + sB2;
    double kk[3] = {0.0, 0.0, 0.0}, vi_new[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) {
        kk[k] = E[k] / den;
        vi_new[k] = vi[k] + (sB - m) * kk[k];
    }
    for (int64_t q = 0; q < nb; ++q) {
        if (cj[q]) continue;
        for (int k = 0; k < dim; ++k) {
            double vjp = vj[q * dim + k] - Bj[q] * kk[k];
            vj[q * dim + k] = vj[q * dim + k] - Bj[q] * (vi_new[k] - vjp) / m;
        }
    }
    for (int k = 0; k < dim; ++k) vi[k] = vi_new[k];
}

static void damp_particle_pbp(orc_body *b, int64_t i, double eta_t, double tau)
{
    int D = b->dim;
    int64_t lo = b->row_ptr[i], nb = b->row_ptr[i + 1] - lo;
    if (b->clamped[i]) {
        /* a wall particle: each free neighbour is damped against it as a particle whose only
         * neighbour is the wall (the local system of Eq. 29 with one clamped neighbour), which the
         * gradient step solves exactly: v_j <- m v_j / (m - B_j) */
        for (int64_t q = 0; q < nb; ++q) {
            int64_t j = b->col[lo + q];
            if (b->clamped[j]) continue;
            double g[3], r, dW;
            grad_w(b, i, j, g, &r, &dW);
            double Bj = eta_t * tau * (2.0 * b->vol * b->vol * dW / r);
            for (int k = 0; k < D; ++k) b->v[j * D + k] = b->mass * b->v[j * D + k] / (b->mass - Bj);
        }
        return;
    }
    double *Bj = (double *)xcalloc(nb, sizeof(double));
    double *vj = (double *)xcalloc(nb * D, sizeof(double));
    unsigned char *cj = (unsigned char *)xcalloc(nb, 1);
    for (int64_t q = 0; q < nb; ++q) {
        int64_t j = b->col[lo + q];
        double g[3], r, dW;
        grad_w(b, i, j, g, &r, &dW);
        Bj[q] = eta_t * tau * (2.0 * b->vol * b->vol * dW / r);
        cj[q] = b->clamped[j];
        for (int k = 0; k < D; ++k) vj[q * D + k] = b->v[j * D + k];
    }
    orc_pbp_local(D, b->mass, nb, Bj, cj, &b->v[i * D], vj);
    for (int64_t q = 0; q < nb; ++q) {
        int64_t j = b->col[lo + q];
        if (cj[q]) continue;
        for (int k = 0; k < D; ++k) b->v[j * D + k] = vj[q * D + k];
    }
    free(Bj);
    free(vj);
    free(cj);
}

static void damp_visit(orc_body *b, int64_t i, double eta_t, double tau)
{
    if (b->scheme == ORC_PARTICLE) damp_particle_pbp(b, i, eta_t, tau);
    else damp_particle(b, i, eta_t, tau);
}

/* S_d(dt) (Eq. 25): every D_i(dt/2) in the forward order -- colours 0..K-1, cells of a colour
 * ascending, particles of a cell ascending -- then every D_i(dt/2) in exactly the reverse order. */
static void damp_sweep(orc_body *b, double eta_t, double dt)
{
    /* cells of one colour touch disjoint neighbourhoods, so they may run in any order (in parallel) */
    for (int64_t k = 0; k < b->ncolour; ++k) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t q = b->colour_start[k]; q < b->colour_start[k + 1]; ++q) {
            int64_t c = b->colour_cells[q];
            for (int64_t i = b->cell_start[c]; i < b->cell_start[c + 1]; ++i) damp_visit(b, i, eta_t, 0.5 * dt);
        }
    }
    for (int64_t k = b->ncolour - 1; k >= 0; --k) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t q = b->colour_start[k + 1] - 1; q >= b->colour_start[k]; --q) {
            int64_t c = b->colour_cells[q];
            for (int64_t i = b->cell_start[c + 1] - 1; i >= b->cell_start[c]; --i) damp_visit(b, i, eta_t, 0.5 * dt);
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* One relaxation step (Sec. 2.3 Verlet with the Lie-Trotter damping split of Eq. 24)          */
/* ------------------------------------------------------------------------------------------ */
static double neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
    return t;
}

/* force: -1 = random choice, 0 = never damp, 1 = damp (with eta / alpha) */
static int step_once(orc_body *b, int force, int *damped_out)
{
    int D = b->dim;
    if (b->dt <= 0.0) b->dt = time_step(b, max_free_speed(b), b->bmax);
    double dt = b->dt;
    int damped = (force < 0) ? orc_damped_decision(b->seed, b->step, b->alpha) : force;
    /* first half drift (Eq. 15) */
    for (int64_t i = 0; i < b->n; ++i)
        if (!b->clamped[i])
            for (int k = 0; k < D; ++k) b->u[i * D + k] += 0.5 * dt * b->v[i * D + k];
    /* S_m: F, P, T, then force and kick (Eqs. 12, 16) */
    int st = compute_T(b);
    if (st != ORC_OK) return st;
    compute_accel(b);
    double amax = 0.0, asq = 0.0, asq_c = 0.0, bsq = 0.0, bsq_c = 0.0;
    for (int64_t i = 0; i < b->n; ++i) {
        if (b->clamped[i]) continue;
        double an = vnorm(D, &b->acc[i * D]);
        double bn = vnorm(D, &b->bf[i * D]);
        amax = fmax(amax, an);
        neumaier_add(&asq, &asq_c, an * an);
        neumaier_add(&bsq, &bsq_c, bn * bn);
        for (int k = 0; k < D; ++k) b->v[i * D + k] += dt * b->acc[i * D + k];
    }
    /* S_d on the chosen steps (Eq. 40 with eta_t = eta / alpha) */
    if (damped && b->eta > 0.0) damp_sweep(b, b->eta / b->alpha, dt);
    /* second half drift (Eq. 17); clamped particles stay at rest */
    double ek = 0.0, ek_c = 0.0, vmax = 0.0;
    for (int64_t i = 0; i < b->n; ++i) {
        if (b->clamped[i]) {
            for (int k = 0; k < D; ++k) { b->u[i * D + k] = 0.0; b->v[i * D + k] = 0.0; }
            continue;
        }
        for (int k = 0; k < D; ++k) b->u[i * D + k] += 0.5 * dt * b->v[i * D + k];
        double vn2 = b->v[i * D] * b->v[i * D] + b->v[i * D + 1] * b->v[i * D + 1];
        if (D == 3) vn2 = vn2 + b->v[i * D + 2] * b->v[i * D + 2];
        neumaier_add(&ek, &ek_c, 0.5 * b->mass * vn2);
        vmax = fmax(vmax, sqrt(vn2));
        for (int k = 0; k < D; ++k)
            if (!isfinite(b->u[i * D + k]) || !isfinite(b->v[i * D + k])) return ORC_E_NONFINITE;
    }
    ek = ek + ek_c;
    /* residual tracking */
    b->ek_last = ek;
    if (ek > b->ek_peak) b->ek_peak = ek;
    if (b->ek_turn == 0.0 && ek < b->ek_peak) b->ek_turn = b->ek_peak;
    b->ek_win[b->win_pos] = ek;
    b->win_pos = (b->win_pos + 1) % b->win;
    if (b->win_fill < b->win) b->win_fill++;
    double wmax = 0.0;
    for (int64_t q = 0; q < b->win_fill; ++q) wmax = fmax(wmax, b->ek_win[q]);
    b->resid_last = (b->ek_peak > 0.0) ? wmax / b->ek_peak : 1.0;
    asq = asq + asq_c; bsq = bsq + bsq_c;
    b->fres_last = (bsq > 0.0) ? sqrt(asq) / sqrt(bsq) : sqrt(asq);
    b->amax_prev = amax;
    b->dt = time_step(b, vmax, amax);
    b->step += 1;
    if (damped_out) *damped_out = damped;
    /* blow-up: once E_k has turned over, a kinetic energy beyond div_factor times that first peak */
    if (b->ek_turn > 0.0 && ek > b->div_factor * b->ek_turn) return ORC_E_DIVERGED;
    return ORC_OK;
}

int orc_body_step(orc_body *b, int64_t nsteps, int force, int64_t *damped_count)
{
    if (!b || !b->material_set || nsteps < 0) return ORC_E_INVALID;
    int64_t nd = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        int d = 0;
        int st = step_once(b, force, &d);
        if (st != ORC_OK) return st;
        nd += d;
    }
    if (damped_count) *damped_count = nd;
    return ORC_OK;
}

typedef struct {
    int64_t steps, damped_steps;
    double residual, kinetic_energy, force_residual;
    int converged;
} orc_report;

int orc_body_relax(orc_body *b, double tol, int64_t max_steps, orc_report *rep)
{
    if (!b || !b->material_set || max_steps < 0) return ORC_E_INVALID;
    orc_report r;
    memset(&r, 0, sizeof(r));
    int status = ORC_NOT_CONVERGED;
    for (int64_t s = 0; s < max_steps; ++s) {
        int d = 0;
        int st = step_once(b, -1, &d);
        if (st != ORC_OK) { status = st; break; }
        r.steps++;
        r.damped_steps += d;
        if (b->resid_last < tol && b->step >= b->win) { status = ORC_OK; r.converged = 1; break; }
    }
    r.residual = b->resid_last;
    r.kinetic_energy = b->ek_last;
    r.force_residual = b->fres_last;
    if (rep) *rep = r;
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* State access (input order) and diagnostics                                                  */
/* ------------------------------------------------------------------------------------------ */
int64_t orc_body_n(const orc_body *b) { return b->n; }
int64_t orc_body_nnz(const orc_body *b) { return b->row_ptr[b->n]; }
int64_t orc_body_step_index(const orc_body *b) { return b->step; }
double orc_body_dt(const orc_body *b) { return b->dt; }
double orc_body_residual(const orc_body *b) { return b->resid_last; }
double orc_body_kinetic_energy(const orc_body *b) { return b->ek_last; }
double orc_body_ek_peak(const orc_body *b) { return b->ek_peak; }
void orc_body_grid(const orc_body *b, int64_t nc[3], double xmin[3], double *rc)
{
    for (int k = 0; k < 3; ++k) { nc[k] = b->nc[k]; xmin[k] = b->xmin[k]; }
    *rc = b->rc;
}

/* u and v in input order, n x dim (either may be NULL) */
void orc_body_get_state(const orc_body *b, double *u, double *v)
{
    int D = b->dim;
    for (int64_t p = 0; p < b->n; ++p) {
        int64_t i = b->perm[p];
        for (int k = 0; k < D; ++k) {
            if (u) u[i * D + k] = b->u[p * D + k];
            if (v) v[i * D + k] = b->v[p * D + k];
        }
    }
}

/* Sets u, v (input order; clamped entries are forced to zero), the step index and the next dt
 * (dt <= 0: derive it from max|v| and max|b|).  Residual tracking restarts. */
int orc_body_set_state(orc_body *b, const double *u, const double *v, int64_t step, double dt)
{
    if (!b || step < 0) return ORC_E_INVALID;
    int D = b->dim;
    for (int64_t p = 0; p < b->n; ++p) {
        int64_t i = b->perm[p];
        for (int k = 0; k < D; ++k) {
            b->u[p * D + k] = (u && !b->clamped[p]) ? u[i * D + k] : 0.0;
            b->v[p * D + k] = (v && !b->clamped[p]) ? v[i * D + k] : 0.0;
        }
    }
    b->step = step;
    b->dt = dt;
    reset_tracking(b);
    return ORC_OK;
}

/* F of every particle for the current u (input order, n x dim x dim, row-major) */
void orc_body_get_F(const orc_body *b, double *F)
{
    int D = b->dim;
    for (int64_t p = 0; p < b->n; ++p) deformation_gradient(b, p, &F[b->perm[p] * D * D]);
}

/* B0 of every particle (input order) */
void orc_body_get_B0(const orc_body *b, double *B0)
{
    int D = b->dim;
    for (int64_t p = 0; p < b->n; ++p)
        memcpy(&B0[b->perm[p] * D * D], &b->B0[p * D * D], sizeof(double) * D * D);
}

/* S_m acceleration (Eq. 12) of every particle for the current u without advancing the state
 * (input order, n x dim).  T is also returned when non-NULL (n x dim x dim). */
int orc_body_get_accel(orc_body *b, double *acc, double *T)
{
    int D = b->dim;
    if (!b->material_set) return ORC_E_INVALID;
    int st = compute_T(b);
    if (st != ORC_OK) return st;
    compute_accel(b);
    for (int64_t p = 0; p < b->n; ++p) {
        int64_t i = b->perm[p];
        if (acc) for (int k = 0; k < D; ++k) acc[i * D + k] = b->acc[p * D + k];
        if (T) memcpy(&T[i * D * D], &b->T[p * D * D], sizeof(double) * D * D);
    }
    return ORC_OK;
}

/* Von Mises equivalent stress of the Cauchy stress sigma = J^-1 P F^T = J^-1 F S F^T (P = F S is
 * the first Piola-Kirchhoff stress of Sec. 2.1, J = det F): sqrt(3/2 s:s) with s the deviator of
 * the 3x3 sigma, i.e. sqrt(((s11 - s22)^2 + (s22 - s33)^2 + (s33 - s11)^2) / 2 + 3 (s12^2 + s23^2 +
 * s13^2)).  2D is plane strain (F33 = 1, E33 = 0): the out-of-plane normal stress is
 * sigma33 = S33 / J with S33 = lambda tr E (St Venant-Kirchhoff, Eq. 4) or lambda ln J (neo-Hookean,
 * Eq. 7 with C33 = 1).  ORC_E_NONFINITE when J <= 0. */
int orc_von_mises(int dim, int model, double lam, double mu, const double *F, double *vm)
{
    int D = dim;
    double S[9], P[9], sig[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double J = det_n(D, F);
    if (!(J > 0.0)) return ORC_E_NONFINITE;
    int st = orc_stress(D, model, lam, mu, F, S, P);
    if (st != ORC_OK) return st;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += P[a * D + k] * F[b * D + k];
            sig[a][b] = s / J;
        }
    if (D == 2) {
        double S33;
        if (model == ORC_SVK) {
            double trE = 0.0;
            for (int a = 0; a < 2; ++a) {
                double Caa = 0.0;
                for (int k = 0; k < 2; ++k) Caa += F[k * 2 + a] * F[k * 2 + a];
                trE += 0.5 * (Caa - 1.0);
            }
            S33 = lam * trE;
        } else {
            S33 = lam * log(J);
        }
        sig[2][2] = S33 / J;
    }
    double d01 = sig[0][0] - sig[1][1], d12 = sig[1][1] - sig[2][2], d20 = sig[2][2] - sig[0][0];
    double q = 0.5 * (d01 * d01 + d12 * d12 + d20 * d20) +
               3.0 * (sig[0][1] * sig[0][1] + sig[1][2] * sig[1][2] + sig[0][2] * sig[0][2]);
    *vm = sqrt(q);
    return ORC_OK;
}

/* Von Mises stress of every particle for the current u (input order, n values): F of Eq. 9 at
 * each particle, clamped ones included. */
int orc_body_von_mises(orc_body *b, double *out)
{
    if (!b->material_set) return ORC_E_INVALID;
    int status = ORC_OK;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < b->n; ++p) {
        double F[9];
        deformation_gradient(b, p, F);
        int st = orc_von_mises(b->dim, b->model, b->lam, b->mu, F, &out[b->perm[p]]);
        if (st != ORC_OK) {
#pragma omp atomic write
            status = st;
        }
    }
    return status;
}

/* Apply S_d(dt) alone to the current v with viscosity eta_t (for the damping pins). */
void orc_body_damp(orc_body *b, double eta_t, double dt) { damp_sweep(b, eta_t, dt); }

/* Topology in internal order: perm (internal -> input), cell id and colour per particle,
 * row_ptr (n + 1) and col (nnz).  Any pointer may be NULL. */
void orc_body_topology(const orc_body *b, int64_t *perm, int64_t *cell, int64_t *colour, int64_t *row_ptr,
                       int64_t *col)
{
    for (int64_t p = 0; p < b->n; ++p) {
        if (perm) perm[p] = b->perm[p];
        if (cell) cell[p] = b->cell[p];
        if (colour) colour[p] = cell_colour(b, b->cell[p]);
    }
    if (row_ptr) memcpy(row_ptr, b->row_ptr, sizeof(int64_t) * (b->n + 1));
    if (col) memcpy(col, b->col, sizeof(int64_t) * b->row_ptr[b->n]);
}

/* Colour of an arbitrary cell id of this body's grid (for the splitting-CLL pins). */
int64_t orc_body_cell_colour(const orc_body *b, int64_t lin) { return cell_colour(b, lin); }
