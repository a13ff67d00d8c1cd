// api.hip -- host side of the library: the extern "C" entry points of tlsph_dr.h, body lifecycle,
// the per-step launch schedule and the random-choice decisions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tlsph_dr.h"
#include "body.hpp"
#include "internal.hpp"

namespace tlsph {
size_t damp_lds_bytes(int dim, int precision, int hcap, int ecap);

}  // namespace tlsph

using namespace tlsph;

namespace tlsph {

thread_local std::string g_err;

tlsph_status fail(tlsph_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

// ---------------------------------------------------------------------------------------------
// Counter-based generator for the random choice (Sec. 3.3, Eq. 40): Philox4x64 with 10 rounds
// (Salmon et al., SC'11).  Each round multiplies words 0 and 2 by the two Philox constants, and
// the next state is (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key is
// bumped by the two Weyl constants between rounds.
// ---------------------------------------------------------------------------------------------
struct Philox4x64 {
    static constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
    static constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
    static constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
    static constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
    uint64_t key[2];

    static inline void mul128(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
    {
        const __uint128_t p = static_cast<__uint128_t>(a) * b;
        hi = static_cast<uint64_t>(p >> 64);
        lo = static_cast<uint64_t>(p);
    }
    void block(const uint64_t in[4], uint64_t out[4]) const
    {
        uint64_t x[4] = {in[0], in[1], in[2], in[3]};
        uint64_t k0 = key[0], k1 = key[1];
        for (int round = 0; round < 10; ++round) {
            uint64_t h0, l0, h1, l1;
            mul128(kMul0, x[0], h0, l0);
            mul128(kMul1, x[2], h1, l1);
            const uint64_t nx[4] = {h1 ^ x[1] ^ k0, l1, h0 ^ x[3] ^ k1, l0};
            x[0] = nx[0]; x[1] = nx[1]; x[2] = nx[2]; x[3] = nx[3];
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        for (int w = 0; w < 4; ++w) out[w] = x[w];
    }
};

// Step n is damped iff the top 24 bits of output word 0 of counter (n, 0, 0, 0), key (seed, 0),
// fall below ceil(alpha 2^24): probability alpha (Eq. 40 read as phi < alpha).
bool damped_step(uint64_t seed, double alpha, int64_t n)
{
    if (alpha >= 1.0) return true;
    if (!(alpha > 0.0)) return false;
    Philox4x64 g{{seed, 0}};
    const uint64_t ctr[4] = {static_cast<uint64_t>(n), 0, 0, 0};
    uint64_t out[4];
    g.block(ctr, out);
    const uint64_t threshold = static_cast<uint64_t>(ceil(alpha * 16777216.0));
    return (out[0] >> 40) < threshold;
}

void *default_alloc(size_t bytes, void *)
{
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}
void default_free(void *p, void *)
{
    if (p) (void)hipFree(p);
}

}  // namespace tlsph

namespace tlsph {

hipEvent_t pool_event(tlsph_body b)
{
    if (!b->prof_pool.empty()) {
        hipEvent_t e = b->prof_pool.back();
        b->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

struct ProfScope {
    tlsph_body b;
    int pass;
    hipEvent_t a{};
    ProfScope(tlsph_body body, int p) : b(body), pass(p)
    {
        if (b->prof) {
            a = pool_event(b);
            (void)hipEventRecord(a, b->stream);
        }
    }
    ~ProfScope()
    {
        if (b->prof) {
            hipEvent_t e = pool_event(b);
            (void)hipEventRecord(e, b->stream);
            b->prof_pending.push_back({pass, a, e});
        }
    }
};

void prof_collect(tlsph_body b)
{
    for (auto &pe : b->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            b->prof_ms[pe.pass] += ms;
            b->prof_n[pe.pass] += 1;
        }
        b->prof_pool.push_back(pe.a);
        b->prof_pool.push_back(pe.b);
    }
    b->prof_pending.clear();
}

const char *step_error_text(int code)
{
    if (code == TLSPH_E_DIVERGED) return "kinetic energy blew up (beyond the divergence factor times its first peak)";
    return "non-finite state or inverted particle (J <= 0)";
}

tlsph_status hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(TLSPH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return TLSPH_OK;
}

tlsph_status pull_state(tlsph_body b)
{
    tlsph_status s = hip_check(hipMemcpyAsync(b->hst, b->db.st, sizeof(DevState), hipMemcpyDeviceToHost, b->stream),
                               "reading device state");
    if (s != TLSPH_OK) return s;
    return hip_check(hipStreamSynchronize(b->stream), "synchronising the body stream");
}

tlsph_status push_state(tlsph_body b)
{
    tlsph_status s = hip_check(hipMemcpyAsync(b->db.st, b->hst, sizeof(DevState), hipMemcpyHostToDevice, b->stream),
                               "writing device state");
    if (s != TLSPH_OK) return s;
    return hip_check(hipStreamSynchronize(b->stream), "synchronising the body stream");
}

// Time-step criterion of Eq. 18 at rest, and the residual window W = ceil(T_w / dt0) with
// T_w = L_max^2 / (L_min c).
int64_t window_length(tlsph_body b)
{
    const double c = b->P.c;
    double dt0 = INFINITY;
    if (c > 0.0) dt0 = b->h / c;
    if (b->bmax > 0.0) dt0 = fmin(dt0, sqrt(b->h / b->bmax));
    dt0 *= 0.6;
    if (!(c > 0.0) || !isfinite(dt0)) return 1;
    const double Tw = b->extent_max * b->extent_max / (b->extent_min * c);
    int64_t W = (int64_t)ceil(Tw / dt0);
    return W < 1 ? 1 : W;
}

// Resets the residual tracking (E_peak, window) and marks dt for recomputation.
tlsph_status reset_tracking(tlsph_body b, bool recompute_dt)
{
    tlsph_status s = pull_state(b);
    if (s != TLSPH_OK) return s;
    const int64_t W = b->material_set ? window_length(b) : 1;
    if (W != b->hst->win || !b->db.win_buf) {
        b->dput(b->db.win_buf);
        b->db.win_buf = (double *)b->dget(sizeof(double) * W);
        if (!b->db.win_buf) return fail(TLSPH_E_NOMEM, "allocating the residual window (%lld entries)", (long long)W);
    }
    b->hst->win = W;
    b->hst->win_fill = 0;
    b->hst->win_pos = 0;
    b->hst->win_start = b->hst->step;
    b->hst->last_high = b->hst->step;
    b->hst->ek_peak = 0.0;
    b->hst->ek_turn = 0.0;
    b->hst->ek = 0.0;
    b->hst->resid = 1.0;
    b->hst->done = 0;
    b->hst->error = 0;
    b->hst->bad_stress = 0;
    if (recompute_dt) b->dt_valid = false;
    return push_state(b);
}

void enqueue_step(tlsph_body b, bool damped)
{
    const hipStream_t s = b->stream;
    {
        ProfScope ps(b, kPassA);
        launch_passA(b->db, b->P, b->precision, s);
    }
    {
        ProfScope ps(b, kPassB);
        launch_passB(b->db, b->P, b->precision, s);
    }
    if (damped && b->eta > 0.0) {
        const int K = b->dim == 3 ? 27 : 9;
        const double eta_t = b->eta / b->alpha;
        for (int c = 0; c < K; ++c) {
            ProfScope ps(b, kPassD);
            launch_damp_colour(b->db, b->P, b->precision, b->scheme, c, true, eta_t, s);
        }
        for (int c = K - 1; c >= 0; --c) {
            ProfScope ps(b, kPassD);
            launch_damp_colour(b->db, b->P, b->precision, b->scheme, c, false, eta_t, s);
        }
    }
    {
        ProfScope ps(b, kPassC);
        launch_passC(b->db, b->P, b->precision, s);
    }
    {
        ProfScope ps(b, kFinish);
        launch_finish(b->db, b->P, s);
    }
}

bool decision(tlsph_body b, int force, int64_t n)
{
    if (force == 0) return false;
    if (force > 0) return b->damping_set;
    return b->damping_set && damped_step(b->seed, b->alpha, n);
}

tlsph_status run(tlsph_body b, int64_t max_steps, bool relax, double tol, int force, tlsph_report *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!b->material_set) return fail(TLSPH_E_INVALID, "set_material must be called before stepping");
    if (max_steps < 0) return fail(TLSPH_E_INVALID, "negative step count");
    tlsph_status s;
    if (!b->dt_valid) {
        launch_init_dt(b->db, b->P, b->precision, b->bmax, b->dt_given, b->stream);
        b->dt_valid = true;
        b->dt_given = 0.0;
    }
    launch_control(b->db.st, b->db.win_buf, relax ? 1 : 0, tol, INT64_MAX, b->stream);
    int64_t taken = 0, damped = 0;
    int64_t batch = 8;
    bool stop = false;
    tlsph_status result = TLSPH_OK;
    while (taken < max_steps && !stop) {
        const int64_t nb = std::min<int64_t>(batch, max_steps - taken);
        const int64_t n0 = b->step;
        for (int64_t q = 0; q < nb; ++q) enqueue_step(b, decision(b, force, n0 + q));
        launch_resid(b->db, b->stream);
        s = pull_state(b);
        if (s != TLSPH_OK) return s;
        if (b->prof) prof_collect(b);
        const int64_t executed = b->hst->step - n0;
        for (int64_t q = 0; q < executed; ++q) damped += decision(b, force, n0 + q) ? 1 : 0;
        taken += executed;
        b->step = b->hst->step;
        if (b->hst->error) {
            result = fail((tlsph_status)b->hst->error, "%s at step %lld", step_error_text(b->hst->error),
                          (long long)b->step);
            stop = true;
        } else if (b->hst->done || executed < nb) {
            stop = true;
        }
        if (batch < 1024) batch *= 2;
    }
    if (result == TLSPH_OK && relax) {
        const bool conv = b->hst->resid < tol && b->hst->step >= b->hst->win;
        result = conv ? TLSPH_OK : TLSPH_NOT_CONVERGED;
    }
    if (out) {
        out->steps = taken;
        out->damped_steps = damped;
        out->step_index = b->step;
        out->residual = b->hst->resid;
        out->kinetic_energy = b->hst->ek;
        out->force_residual = b->hst->fres;
        out->dt = b->hst->dt;
        out->window = b->hst->win;
        out->converged = (b->hst->resid < tol && b->hst->step >= b->hst->win) ? 1 : 0;
        out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

template <typename R>
void to_internal_soa(const double *in, int64_t n, int D, const std::vector<int32_t> &perm, std::vector<R> &out)
{
    out.assign((size_t)n * D, R(0));
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = perm[p];
        for (int k = 0; k < D; ++k) out[(size_t)k * n + p] = (R)in[i * D + k];
    }
}

tlsph_status upload_field(tlsph_body b, void *dst, const double *src_input_order, bool real, const uint8_t *zero_mask)
{
    const int64_t n = b->n;
    const int D = b->dim;
    if (real && b->precision == 32) {
        std::vector<float> h;
        to_internal_soa<float>(src_input_order, n, D, b->perm, h);
        if (zero_mask)
            for (int64_t p = 0; p < n; ++p)
                if (zero_mask[p])
                    for (int k = 0; k < D; ++k) h[(size_t)k * n + p] = 0.f;
        tlsph_status s = hip_check(hipMemcpyAsync(dst, h.data(), h.size() * 4, hipMemcpyHostToDevice, b->stream), "upload");
        if (s != TLSPH_OK) return s;
        return hip_check(hipStreamSynchronize(b->stream), "upload");
    }
    std::vector<double> h;
    to_internal_soa<double>(src_input_order, n, D, b->perm, h);
    if (zero_mask)
        for (int64_t p = 0; p < n; ++p)
            if (zero_mask[p])
                for (int k = 0; k < D; ++k) h[(size_t)k * n + p] = 0.0;
    tlsph_status s = hip_check(hipMemcpyAsync(dst, h.data(), h.size() * 8, hipMemcpyHostToDevice, b->stream), "upload");
    if (s != TLSPH_OK) return s;
    return hip_check(hipStreamSynchronize(b->stream), "upload");
}

tlsph_status download_field(tlsph_body b, const void *src, bool real, double *dst_input_order)
{
    const int64_t n = b->n;
    const int D = b->dim;
    std::vector<double> h((size_t)n * D);
    if (real && b->precision == 32) {
        std::vector<float> f((size_t)n * D);
        tlsph_status s = hip_check(hipMemcpyAsync(f.data(), src, f.size() * 4, hipMemcpyDeviceToHost, b->stream), "download");
        if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "download");
        if (s != TLSPH_OK) return s;
        for (size_t q = 0; q < h.size(); ++q) h[q] = f[q];
    } else {
        tlsph_status s = hip_check(hipMemcpyAsync(h.data(), src, h.size() * 8, hipMemcpyDeviceToHost, b->stream), "download");
        if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "download");
        if (s != TLSPH_OK) return s;
    }
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = b->perm[p];
        for (int k = 0; k < D; ++k) dst_input_order[i * D + k] = h[(size_t)k * n + p];
    }
    return TLSPH_OK;
}

std::vector<uint8_t> clamped_internal(tlsph_body b)
{
    std::vector<uint8_t> c((size_t)b->n);
    (void)hipMemcpyAsync(c.data(), b->db.clamped, c.size(), hipMemcpyDeviceToHost, b->stream);
    (void)hipStreamSynchronize(b->stream);
    return c;
}

void free_body(tlsph_body b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    DeviceBody &d = b->db;
    void *ptrs[] = {d.X, d.u, d.uh, d.v, d.B0, d.gradsum, d.T, d.accel, d.clamped, d.row_ptr, d.col, d.hslot_a,
                    d.dslot, d.dorder, d.dtouch, d.downr, d.cmap, d.brick_lmax_a, d.gdamp, d.cell_start, d.partB,
                    d.partC, d.partF, d.win_buf, d.st};
    for (void *p : ptrs) b->dput(p);
    // pass B's slot arrays are pass A's when both passes use one brick geometry
    if (d.hslot_b != d.hslot_a) b->dput(d.hslot_b);
    if (d.brick_lmax_b != d.brick_lmax_a) b->dput(d.brick_lmax_b);
    b->dput(d.runs_a);
    if (d.runs_b != d.runs_a) b->dput(d.runs_b);
    if (b->hst && b->hst_owned) (void)hipHostFree(b->hst);
    for (auto &pe : b->prof_pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : b->prof_pool) (void)hipEventDestroy(e);
    delete b;
}

tlsph_status create_body(const tlsph_body_desc *desc, DevState *mirror, tlsph_body *out)
{
    if (!out) return fail(TLSPH_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!desc || !desc->X0) return fail(TLSPH_E_INVALID, "descriptor or X0 is NULL");
    const int D = desc->dim;
    const int64_t n = desc->n;
    if (D != 2 && D != 3) return fail(TLSPH_E_INVALID, "dim must be 2 or 3 (got %d)", D);
    if (n < 1 || n >= ((int64_t)1 << 31) - 1) return fail(TLSPH_E_INVALID, "particle count %lld out of range", (long long)n);
    if (!(desc->dp > 0.0) || !(desc->h_over_dp > 0.0) || !(desc->rho0 > 0.0))
        return fail(TLSPH_E_INVALID, "dp, h_over_dp and rho0 must be positive");
    if (desc->precision != TLSPH_FP32 && desc->precision != TLSPH_FP64)
        return fail(TLSPH_E_INVALID, "precision must be TLSPH_FP32 or TLSPH_FP64");
    double xmin[3] = {0, 0, 0}, xmax[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) xmin[k] = xmax[k] = desc->X0[k];
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < D; ++k) {
            const double x = desc->X0[i * D + k];
            if (!isfinite(x)) return fail(TLSPH_E_INVALID, "X0 holds a non-finite value (particle %lld)", (long long)i);
            xmin[k] = fmin(xmin[k], x);
            xmax[k] = fmax(xmax[k], x);
        }
    tlsph_body b = new (std::nothrow) tlsph_body_s();
    if (!b) return fail(TLSPH_E_NOMEM, "host allocation failed");
    try {
        b->dim = D;
        b->n = n;
        b->precision = desc->precision;
        b->stream = (hipStream_t)desc->stream;
        if (hipGetDevice(&b->device) != hipSuccess) {
            free_body(b);
            return fail(TLSPH_E_DEVICE, "hipGetDevice failed");
        }
        b->alloc = desc->alloc;
        if (!b->alloc.alloc || !b->alloc.free) {
            b->alloc.alloc = default_alloc;
            b->alloc.free = default_free;
            b->alloc.ctx = nullptr;
        }
        b->dp = desc->dp;
        b->rho0 = desc->rho0;
        b->h = desc->h_over_dp * desc->dp;
        b->rc = 2.0 * b->h;
        b->rc2 = b->rc * b->rc;
        for (int k = 0; k < 3; ++k) b->xmin[k] = xmin[k];
        DeviceBody &d = b->db;
        d.dim = D;
        d.n = n;
        d.nc[0] = d.nc[1] = d.nc[2] = 1;
        b->extent_min = INFINITY;
        b->extent_max = 0.0;
        for (int k = 0; k < D; ++k) {
            const double cells = floor((xmax[k] - xmin[k]) / b->rc) + 1.0;
            if (cells > 2e9) {
                free_body(b);
                return fail(TLSPH_E_LIMIT, "cell grid too large along axis %d", k);
            }
            d.nc[k] = (int32_t)cells;
            const double e = (xmax[k] - xmin[k]) + desc->dp;
            b->extent_min = fmin(b->extent_min, e);
            b->extent_max = fmax(b->extent_max, e);
        }
        d.ncell = (int64_t)d.nc[0] * d.nc[1] * d.nc[2];
        if (d.ncell >= ((int64_t)1 << 31) - 1) {
            free_body(b);
            return fail(TLSPH_E_LIMIT, "too many cells (%lld)", (long long)d.ncell);
        }
        const size_t rs = b->precision == 32 ? 4 : 8;
        d.X = (double *)b->dget(sizeof(double) * D * n);
        d.u = (double *)b->dget(sizeof(double) * D * n);
        d.uh = (double *)b->dget(sizeof(double) * D * n);
        d.v = b->dget(rs * D * n);
        d.B0 = b->dget(rs * D * D * n);
        d.gradsum = b->dget(rs * D * n);
        d.T = b->dget(rs * D * D * n);
        d.clamped = (uint8_t *)b->dget(n);
        d.row_ptr = (int64_t *)b->dget(sizeof(int64_t) * (n + 1));
        d.cell_start = (int32_t *)b->dget(sizeof(int32_t) * (d.ncell + 1));
        d.nblocks = (int)((n + kBlock - 1) / kBlock);
        d.partC = (double *)b->dget(sizeof(double) * 4 * d.nblocks);
        d.st = (DevState *)b->dget(sizeof(DevState));
        void *X0d = b->dget(sizeof(double) * D * n);
        void *cld = desc->clamped ? b->dget(n) : nullptr;
        int32_t *permd = (int32_t *)b->dget(sizeof(int32_t) * n);
        if (!d.X || !d.u || !d.uh || !d.v || !d.B0 || !d.gradsum || !d.T || !d.clamped || !d.row_ptr || !d.cell_start ||
            !d.partC || !d.st || !X0d || (desc->clamped && !cld) || !permd) {
            b->dput(X0d);
            b->dput(cld);
            b->dput(permd);
            free_body(b);
            return fail(TLSPH_E_NOMEM, "device allocation failed for a body of %lld particles", (long long)n);
        }
        if (mirror) {
            b->hst = mirror;
            b->hst_owned = false;
        } else if (hipHostMalloc((void **)&b->hst, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
            b->hst = nullptr;
            b->dput(X0d);
            b->dput(cld);
            b->dput(permd);
            free_body(b);
            return fail(TLSPH_E_NOMEM, "pinned host allocation failed");
        }
        memset(b->hst, 0, sizeof(DevState));
        b->hst->win = 1;
        b->hst->resid = 1.0;
        (void)hipMemcpyAsync(d.st, b->hst, sizeof(DevState), hipMemcpyHostToDevice, b->stream);
        (void)hipMemcpyAsync(X0d, desc->X0, sizeof(double) * D * n, hipMemcpyHostToDevice, b->stream);
        if (cld) (void)hipMemcpyAsync(cld, desc->clamped, n, hipMemcpyHostToDevice, b->stream);
        (void)hipMemsetAsync(d.u, 0, sizeof(double) * D * n, b->stream);
        (void)hipMemsetAsync(d.v, 0, rs * D * n, b->stream);
        (void)hipMemsetAsync(d.T, 0, rs * D * D * n, b->stream);
        char msg[256] = {0};
        int st = setup_topology(d, b->precision, (const double *)X0d, (const uint8_t *)cld, xmin, b->rc, b->rc2, b->h,
                                D == 2 ? desc->dp * desc->dp : desc->dp * desc->dp * desc->dp, permd, b->alloc.alloc,
                                b->alloc.free, b->alloc.ctx, b->stream, msg, sizeof msg);
        if (st == 0) {
            b->perm.resize(n);
            if (hipMemcpyAsync(b->perm.data(), permd, sizeof(int32_t) * n, hipMemcpyDeviceToHost, b->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(b->stream) != hipSuccess) {
                st = TLSPH_E_DEVICE;
                snprintf(msg, sizeof msg, "HIP error reading the permutation");
            }
        }
        b->dput(X0d);
        b->dput(cld);
        b->dput(permd);
        if (st != 0) {
            free_body(b);
            return fail((tlsph_status)st, "%s", msg);
        }
        d.partB = (double *)b->dget(sizeof(double) * 2 * (size_t)std::max<int64_t>(1, brick_count(d.gb)));
        if (!d.partB) {
            free_body(b);
            return fail(TLSPH_E_NOMEM, "device allocation failed for the pass-B partials");
        }
        // TLSPH_TWO_STAGE_MIN in the environment at body creation overrides the threshold
        int64_t two_stage_min = kTwoStageMin;
        if (const char *e = getenv("TLSPH_TWO_STAGE_MIN")) {
            char *end = nullptr;
            const long long v = strtoll(e, &end, 10);
            if (end != e && *end == '\0' && v >= 0) two_stage_min = v;
        }
        if (brick_count(d.gb) + d.nblocks > two_stage_min) {
            d.partF = (double *)b->dget(sizeof(double) * 8 * kFinishGroups);
            if (!d.partF) {
                free_body(b);
                return fail(TLSPH_E_NOMEM, "device allocation failed for the finish partials");
            }
        }
        if (d.row_max > kMaxRow) {
            free_body(b);
            return fail(TLSPH_E_LIMIT, "a neighbour row holds %d entries; this build handles at most %d", d.row_max,
                        kMaxRow);
        }
        if (damp_lds_bytes(D, b->precision, d.halo_max, d.cell_pairs_max) > 64 * 1024 || d.halo_max > kMaxHalo) {
            free_body(b);
            return fail(TLSPH_E_LIMIT,
                        "a cell neighbourhood holds %d particles and %d neighbour entries; too many for the damping "
                        "pass's LDS tile", d.halo_max, d.cell_pairs_max);
        }
        if (d.cell_max > kMaxCell) {
            free_body(b);
            return fail(TLSPH_E_LIMIT, "a cell holds %d particles; the damping pass handles at most %d", d.cell_max,
                        kMaxCell);
        }
        // constants of the step
        StepParams &P = b->P;
        P.n = n;
        P.h = b->h;
        P.inv_h = 1.0 / b->h;
        const double aD = D == 2 ? 7.0 / (4.0 * M_PI * b->h * b->h) : 21.0 / (16.0 * M_PI * b->h * b->h * b->h);
        P.kfac = -5.0 * aD / (b->h * b->h);
        P.vol = D == 2 ? desc->dp * desc->dp : desc->dp * desc->dp * desc->dp;
        P.rho0 = desc->rho0;
        P.mass = desc->rho0 * P.vol;
        P.model = TLSPH_NEOHOOKE;
        P.dt_visc = INFINITY;
        P.div_factor = 1e6;
        b->bf_free_norm.clear();
        tlsph_status s2 = reset_tracking(b, true);
        if (s2 != TLSPH_OK) {
            free_body(b);
            return s2;
        }
        *out = b;
        return TLSPH_OK;
    } catch (const std::bad_alloc &) {
        free_body(b);
        return fail(TLSPH_E_NOMEM, "host allocation failed");
    }
}

// Eq. 35: the particle-by-particle scheme needs dt <= 50 h^2 / (nu D), nu = eta / rho0 the
// kinematic viscosity of Eq. 19 (eta itself, not eta / alpha); the pairwise scheme has no such limit.
void update_viscous_limit(tlsph_body b)
{
    if (b->scheme == TLSPH_PARTICLE && b->damping_set && b->eta > 0.0) {
        const double nu_k = b->eta / b->rho0;
        b->P.dt_visc = 50.0 * b->h * b->h / (nu_k * b->dim);
    } else {
        b->P.dt_visc = INFINITY;
    }
}

bool body_damped(tlsph_body b, int64_t n) { return b->damping_set && b->eta > 0.0 && damped_step(b->seed, b->alpha, n); }

void fill_inst(tlsph_body b, Inst &I)
{
    const DeviceBody &d = b->db;
    I.P = b->P;
    I.ga = d.ga;
    I.gb = d.gb;
    I.gd = d.gd;
    for (int k = 0; k < 3; ++k) I.nc[k] = d.nc[k];
    I.halo_a = d.halo_a;
    I.halo_b = d.halo_b;
    I.halo_max = d.halo_max;
    I.row_max = d.row_max;
    I.nbA = (int)brick_count(d.ga);
    I.nbB = (int)brick_count(d.gb);
    I.nbC = d.nblocks;
    I.eta_t = b->damping_set ? b->eta / b->alpha : 0.0;
    I.scheme = b->scheme;
    I.cell_start = d.cell_start;
    I.X = d.X;
    I.u = d.u;
    I.uh = d.uh;
    I.v = d.v;
    I.B0 = d.B0;
    I.T = d.T;
    I.accel = d.accel;
    I.clamped = d.clamped;
    I.row_ptr = d.row_ptr;
    I.hslot_a = d.hslot_a;
    I.hslot_b = d.hslot_b;
    I.brick_lmax_a = d.brick_lmax_a;
    I.brick_lmax_b = d.brick_lmax_b;
    I.dslot = d.dslot;
    I.dorder = d.dorder;
    I.dtouch = d.dtouch;
    I.downr = d.downr;
    I.halo_damp = d.halo_damp;
    I.gdamp = d.gdamp;
    I.gradsum = d.gradsum;
    I.partB = d.partB;
    I.partC = d.partC;
    I.win_buf = d.win_buf;
    I.st = d.st;
}

}  // namespace tlsph

// ---------------------------------------------------------------------------------------------
// Scratch memory of tlsph_get_von_mises_noalloc, for callers that cannot allocate device memory.
// One file-scope array per device, kept until the process ends: the kernel's per-particle values in
// internal order, the same values in input order, and the permutation.  Host code uses the
// address hipGetSymbolAddress returns for each device, never the array's name.  Calls that overlap
// on one device share the array and race.
// ---------------------------------------------------------------------------------------------
constexpr int64_t kScratchMaxParticles = int64_t(1) << 21;
constexpr size_t kScratchInternalOff = 0;
constexpr size_t kScratchInputOff = sizeof(double) * kScratchMaxParticles;
constexpr size_t kScratchPermOff = 2 * sizeof(double) * kScratchMaxParticles;
constexpr size_t kScratchBytes = kScratchPermOff + sizeof(int32_t) * kScratchMaxParticles;   // 40 MiB
constexpr int kScratchMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kScratchMaxDevices] = {};

// Address of the scratch array on `device`, looked up once per device with that device current
// (the caller's current device is restored).
tlsph_status scratch_on_device(int device, unsigned char **out)
{
    if (device < 0 || device >= kScratchMaxDevices) return fail(TLSPH_E_LIMIT, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return fail(TLSPH_E_DEVICE, "hipGetDevice failed");
        if (cur != device && hipSetDevice(device) != hipSuccess)
            return fail(TLSPH_E_DEVICE, "hipSetDevice(%d) failed", device);
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(TLSPH_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                        hipGetErrorString(e));
        g_scratch_ptr[device] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[device];
    return TLSPH_OK;
}

// out_input[perm[p]] = in_internal[p]: internal (cell-sorted) order to the caller's order
__global__ void k_to_input_order(const double *__restrict__ in_internal, const int32_t *__restrict__ perm, int64_t n,
                                 double *__restrict__ out_input)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out_input[perm[p]] = in_internal[p];
}

extern "C" {

const char *tlsph_last_error(void) { return g_err.c_str(); }

const char *tlsph_version(void) { return "tlsph_dr 0.1 (gfx950)"; }

tlsph_status tlsph_damping_decisions(uint64_t seed, double alpha, int64_t n0, int64_t count, uint8_t *out)
{
    if (!out || count < 0 || n0 < 0 || !(alpha > 0.0 && alpha <= 1.0))
        return fail(TLSPH_E_INVALID, "tlsph_damping_decisions: bad arguments");
    for (int64_t q = 0; q < count; ++q) out[q] = damped_step(seed, alpha, n0 + q) ? 1 : 0;
    return TLSPH_OK;
}

tlsph_status tlsph_create_body(const tlsph_body_desc *desc, tlsph_body *out) { return create_body(desc, nullptr, out); }


tlsph_status tlsph_set_material(tlsph_body b, int model, double E, double nu)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (model != TLSPH_SVK && model != TLSPH_NEOHOOKE) return fail(TLSPH_E_INVALID, "unknown material model %d", model);
    if (!(E >= 0.0) || !(nu > -1.0 && nu < 0.5)) return fail(TLSPH_E_INVALID, "need E >= 0 and -1 < nu < 0.5");
    b->E = E;
    b->nu = nu;
    b->P.model = model;
    b->P.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    b->P.mu = E / (2.0 * (1.0 + nu));
    const double K = b->P.lam + 2.0 * b->P.mu / 3.0;
    b->P.c = sqrt(K / b->rho0);
    b->material_set = true;
    return reset_tracking(b, true);
}

tlsph_status tlsph_set_loads(tlsph_body b, const double *g, const double *accel)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!g) return fail(TLSPH_E_INVALID, "g is NULL");
    const int D = b->dim;
    const int64_t n = b->n;
    for (int k = 0; k < 3; ++k) b->P.g[k] = k < D ? g[k] : 0.0;
    if (accel) {
        for (int64_t q = 0; q < n * D; ++q)
            if (!isfinite(accel[q])) return fail(TLSPH_E_INVALID, "accel holds a non-finite value");
        if (!b->db.accel) {
            b->db.accel = b->dget((b->precision == 32 ? 4 : 8) * D * n);
            if (!b->db.accel) return fail(TLSPH_E_NOMEM, "allocating the per-particle load");
        }
        tlsph_status s = upload_field(b, b->db.accel, accel, true, nullptr);
        if (s != TLSPH_OK) return s;
        b->P.has_accel = 1;
    } else {
        b->P.has_accel = 0;
    }
    // max |b| and sum |b|^2 over free particles (FP64, input order)
    std::vector<uint8_t> cl = clamped_internal(b);
    std::vector<uint8_t> cl_in((size_t)n);
    for (int64_t p = 0; p < n; ++p) cl_in[b->perm[p]] = cl[p];
    double bmax = 0.0, bsq = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (cl_in[i]) continue;
        double s = 0.0;
        for (int k = 0; k < D; ++k) {
            const double bk = b->P.g[k] + (accel ? accel[i * D + k] : 0.0);
            s += bk * bk;
        }
        bsq += s;
        bmax = fmax(bmax, sqrt(s));
    }
    b->bmax = bmax;
    b->P.bsq = bsq;
    return reset_tracking(b, true);
}

tlsph_status tlsph_set_damping(tlsph_body b, double eta, double beta, double Lc, double alpha, uint64_t seed)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TLSPH_E_INVALID, "alpha must be in (0, 1]");
    if (!(eta > 0.0)) {
        if (!b->material_set) return fail(TLSPH_E_INVALID, "eta <= 0 needs the material (Eq. 36 uses E)");
        if (!(beta >= 0.0) || !(Lc >= 0.0)) return fail(TLSPH_E_INVALID, "beta and Lc must be >= 0");
        eta = beta / 4.0 * sqrt(b->rho0 * b->E) * Lc;
    }
    b->eta = eta;
    b->alpha = alpha;
    b->seed = seed;
    b->damping_set = true;
    update_viscous_limit(b);
    return TLSPH_OK;
}

tlsph_status tlsph_set_damping_scheme(tlsph_body b, int scheme)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (scheme != TLSPH_PAIRWISE && scheme != TLSPH_PARTICLE)
        return fail(TLSPH_E_INVALID, "unknown damping scheme %d", scheme);
    b->scheme = scheme;
    update_viscous_limit(b);
    return TLSPH_OK;
}

tlsph_status tlsph_set_divergence(tlsph_body b, double factor)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!(factor > 0.0)) return fail(TLSPH_E_INVALID, "the divergence factor must be > 0");
    b->P.div_factor = factor;
    return TLSPH_OK;
}

tlsph_status tlsph_relax_until(tlsph_body b, double tol, int64_t max_steps, tlsph_report *out)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!(tol >= 0.0)) return fail(TLSPH_E_INVALID, "tol must be >= 0");
    return run(b, max_steps, true, tol, -1, out);
}

tlsph_status tlsph_step(tlsph_body b, int64_t nsteps, int force_damping, tlsph_report *out)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (force_damping < -1 || force_damping > 1) return fail(TLSPH_E_INVALID, "force_damping must be -1, 0 or 1");
    return run(b, nsteps, false, 0.0, force_damping, out);
}

tlsph_status tlsph_get_displacement(tlsph_body b, double *u_out)
{
    if (!b || !u_out) return fail(TLSPH_E_INVALID, "body or output is NULL");
    return download_field(b, b->db.u, false, u_out);
}

tlsph_status tlsph_get_von_mises(tlsph_body b, double *vm_out)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!vm_out) return fail(TLSPH_E_INVALID, "vm_out is NULL");
    if (!b->material_set) return fail(TLSPH_E_INVALID, "the von Mises stress needs the material");
    const int64_t n = b->n;
    double *d = (double *)b->dget(sizeof(double) * n);
    if (!d) return fail(TLSPH_E_NOMEM, "allocating the von Mises output (%lld values)", (long long)n);
    launch_von_mises(b->db, b->P, b->precision, d, b->stream);
    std::vector<double> h((size_t)n);
    tlsph_status s = hip_check(hipMemcpyAsync(h.data(), d, h.size() * 8, hipMemcpyDeviceToHost, b->stream), "von Mises");
    if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "von Mises");
    b->dput(d);
    if (s != TLSPH_OK) return s;
    int64_t bad = -1;
    for (int64_t p = 0; p < n; ++p) {
        vm_out[b->perm[p]] = h[(size_t)p];
        if (bad < 0 && !std::isfinite(h[(size_t)p])) bad = b->perm[p];
    }
    if (bad >= 0) return fail(TLSPH_E_NONFINITE, "von Mises stress: J <= 0 or non-finite at particle %lld", (long long)bad);
    return TLSPH_OK;
}

tlsph_status tlsph_get_von_mises_noalloc(tlsph_body b, double *vm_out)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (!vm_out) return fail(TLSPH_E_INVALID, "vm_out is NULL");
    if (!b->material_set) return fail(TLSPH_E_INVALID, "the von Mises stress needs the material");
    const int64_t n = b->n;
    if (n > kScratchMaxParticles)
        return fail(TLSPH_E_LIMIT, "tlsph_get_von_mises_noalloc handles at most %lld particles (body has %lld); "
                    "use tlsph_get_von_mises", (long long)kScratchMaxParticles, (long long)n);
    unsigned char *base = nullptr;
    tlsph_status s = scratch_on_device(b->device, &base);
    if (s != TLSPH_OK) return s;
    // every entry of [0, n) of both value regions and of the permutation is written below before it
    // is read, so nothing needs clearing from an earlier call
    double *vm_internal = (double *)(base + kScratchInternalOff);
    double *vm_input = (double *)(base + kScratchInputOff);
    int32_t *perm = (int32_t *)(base + kScratchPermOff);
    s = hip_check(hipMemcpyAsync(perm, b->perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, b->stream),
                  "von Mises (no allocation): permutation");
    if (s != TLSPH_OK) return s;
    launch_von_mises(b->db, b->P, b->precision, vm_internal, b->stream);
    hipLaunchKernelGGL(k_to_input_order, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, vm_internal, perm,
                       n, vm_input);
    s = hip_check(hipGetLastError(), "von Mises (no allocation): launch");
    if (s == TLSPH_OK)
        s = hip_check(hipMemcpyAsync(vm_out, vm_input, sizeof(double) * n, hipMemcpyDeviceToHost, b->stream),
                      "von Mises (no allocation)");
    if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "von Mises (no allocation)");
    if (s != TLSPH_OK) return s;
    // the same particle as tlsph_get_von_mises reports: the first in internal order
    for (int64_t p = 0; p < n; ++p)
        if (!std::isfinite(vm_out[b->perm[p]]))
            return fail(TLSPH_E_NONFINITE, "von Mises stress: J <= 0 or non-finite at particle %lld",
                        (long long)b->perm[p]);
    return TLSPH_OK;
}

tlsph_status tlsph_get_state(tlsph_body b, double *u, double *v, int64_t *step, double *dt)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    tlsph_status s = TLSPH_OK;
    if (u) s = download_field(b, b->db.u, false, u);
    if (s == TLSPH_OK && v) s = download_field(b, b->db.v, true, v);
    if (s != TLSPH_OK) return s;
    s = pull_state(b);
    if (s != TLSPH_OK) return s;
    if (step) *step = b->step;
    if (dt) *dt = b->dt_valid ? b->hst->dt : (b->dt_given > 0.0 ? b->dt_given : 0.0);
    return TLSPH_OK;
}

tlsph_status tlsph_set_state(tlsph_body b, const double *u, const double *v, int64_t step, double dt)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (step < 0) return fail(TLSPH_E_INVALID, "negative step index");
    const int D = b->dim;
    const int64_t n = b->n;
    std::vector<uint8_t> cl = clamped_internal(b);
    std::vector<double> zero;
    if (!u || !v) zero.assign((size_t)n * D, 0.0);
    tlsph_status s = upload_field(b, b->db.u, u ? u : zero.data(), false, cl.data());
    if (s == TLSPH_OK) s = upload_field(b, b->db.v, v ? v : zero.data(), true, cl.data());
    if (s != TLSPH_OK) return s;
    b->step = step;
    s = pull_state(b);
    if (s != TLSPH_OK) return s;
    b->hst->step = step;
    s = push_state(b);
    if (s != TLSPH_OK) return s;
    s = reset_tracking(b, true);
    b->dt_given = dt > 0.0 ? dt : 0.0;
    return s;
}

tlsph_status tlsph_debug_topology(tlsph_body b, int32_t *perm, int32_t *cell, int32_t *colour, int64_t *row_ptr,
                                  int32_t *col)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    const int64_t n = b->n;
    const DeviceBody &d = b->db;
    if (perm) memcpy(perm, b->perm.data(), sizeof(int32_t) * n);
    if (cell || colour) {
        std::vector<int32_t> cs((size_t)d.ncell + 1);
        tlsph_status s = hip_check(
            hipMemcpyAsync(cs.data(), d.cell_start, sizeof(int32_t) * cs.size(), hipMemcpyDeviceToHost, b->stream),
            "download");
        if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "download");
        if (s != TLSPH_OK) return s;
        for (int64_t c = 0; c < d.ncell; ++c) {
            int32_t col_id;
            if (b->dim == 2) {
                const int64_t cx = c / d.nc[1], cy = c % d.nc[1];
                col_id = (int32_t)(3 * (cx % 3) + (cy % 3));
            } else {
                const int64_t cz = c % d.nc[2], t = c / d.nc[2];
                const int64_t cy = t % d.nc[1], cx = t / d.nc[1];
                col_id = (int32_t)(9 * (cx % 3) + 3 * (cy % 3) + (cz % 3));
            }
            for (int32_t p = cs[c]; p < cs[c + 1]; ++p) {
                if (cell) cell[p] = (int32_t)c;
                if (colour) colour[p] = col_id;
            }
        }
    }
    tlsph_status s = TLSPH_OK;
    if (row_ptr)
        s = hip_check(hipMemcpyAsync(row_ptr, d.row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, b->stream),
                      "download");
    if (s == TLSPH_OK && col && d.nnz > 0)
        s = hip_check(hipMemcpyAsync(col, d.col, sizeof(int32_t) * d.nnz, hipMemcpyDeviceToHost, b->stream), "download");
    if (s == TLSPH_OK) s = hip_check(hipStreamSynchronize(b->stream), "download");
    return s;
}

tlsph_status tlsph_debug_bricks(tlsph_body b, int32_t *cells_a, int32_t *cells_b)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (cells_a) *cells_a = b->db.ga.zb;
    if (cells_b) *cells_b = b->db.gb.zb;
    return TLSPH_OK;
}

tlsph_status tlsph_body_info(tlsph_body b, int64_t *n, int64_t *nnz, int32_t ncell[3], int64_t *window)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    if (n) *n = b->n;
    if (nnz) *nnz = b->db.nnz;
    if (ncell)
        for (int k = 0; k < 3; ++k) ncell[k] = b->db.nc[k];
    if (window) *window = b->hst->win;
    return TLSPH_OK;
}

tlsph_status tlsph_profile(tlsph_body b, int enable)
{
    if (!b) return fail(TLSPH_E_INVALID, "body is NULL");
    (void)hipStreamSynchronize(b->stream);
    prof_collect(b);
    b->prof = enable != 0;
    for (int k = 0; k < kNumPass; ++k) {
        b->prof_ms[k] = 0.0;
        b->prof_n[k] = 0;
    }
    return TLSPH_OK;
}

int tlsph_profile_read(tlsph_body b, double *ms, int64_t *launches, int cap)
{
    if (!b) return 0;
    (void)hipStreamSynchronize(b->stream);
    prof_collect(b);
    for (int k = 0; k < kNumPass && k < cap; ++k) {
        if (ms) ms[k] = b->prof_ms[k];
        if (launches) launches[k] = b->prof_n[k];
    }
    return kNumPass;
}

void tlsph_destroy_body(tlsph_body b) { free_body(b); }

}  // extern "C"
