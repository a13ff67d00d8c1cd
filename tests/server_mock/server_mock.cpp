// Host-only mocks of the HIP runtime, the body API and the batched launchers, for running the
// request server's host logic on the CPU under ThreadSanitizer / AddressSanitizer.  Every batched
// launch checks that the rows it is given are the rows of the group's current table and that each
// row points at a live, set-up body.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "body.hpp"
#include "internal.hpp"
#include "../../include/tlsph_dr.h"

static void die(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vfprintf(stderr, fmt, ap);
    va_end(ap);
    fprintf(stderr, "\n");
    abort();
}

// ---- HIP ----
static std::atomic<int> g_stream_id{1};
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new ihipStream_t{g_stream_id++};
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{
    memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned)
{
    *p = calloc(1, n);
    return *p ? hipSuccess : hipErrorUnknown;
}
hipError_t hipHostFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n)
{
    *p = malloc(n);
    return hipSuccess;
}
hipError_t hipFree(void *p)
{
    free(p);
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "mock"; }

// ---- live bodies ----
static std::mutex g_live_m;
static std::set<const void *> g_live_st;   // DevState pointers of live, armed bodies

namespace tlsph {

thread_local std::string g_err_mock;
tlsph_status fail(tlsph_status st, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err_mock = buf;
    return st;
}

const char *step_error_text(int code) { return code == TLSPH_E_DIVERGED ? "blew up" : "non-finite"; }

bool damped_step(uint64_t seed, double alpha, int64_t n)
{
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + (uint64_t)n * 0xBB67AE8584CAA73Bull;
    x ^= x >> 31;
    x *= 0xD2E7470EE14C6C93ull;
    x ^= x >> 29;
    return (double)(x >> 40) < alpha * 16777216.0;
}

tlsph_status create_body(const tlsph_body_desc *desc, DevState *mirror, tlsph_body *out)
{
    if (desc->n < 4) return fail(TLSPH_E_SINGULAR_B0, "too small (mock)");
    tlsph_body b = new tlsph_body_s();
    b->dim = desc->dim;
    b->n = desc->n;
    b->precision = desc->precision;
    b->stream = (hipStream_t)desc->stream;
    b->alloc = desc->alloc;
    b->hst = mirror;
    b->hst_owned = false;
    DeviceBody &d = b->db;
    d.dim = desc->dim;
    d.n = desc->n;
    const int64_t n = desc->n;
    d.nnz = n * (desc->dim == 3 ? 80 : 20);
    d.nblocks = (int)((n + 255) / 256);
    d.X = (double *)b->dget(8 * n * d.dim);
    d.u = (double *)b->dget(8 * n * d.dim);
    d.uh = (double *)b->dget(8 * n * d.dim);
    d.v = b->dget(4 * n * d.dim);
    d.B0 = b->dget(4 * n * d.dim * d.dim);
    d.T = b->dget(4 * n * d.dim * d.dim);
    d.clamped = (uint8_t *)b->dget(n);
    d.row_ptr = (int64_t *)b->dget(8 * (n + 1));
    d.col = (int32_t *)b->dget(4 * d.nnz);
    d.hslot_a = (uint16_t *)b->dget(2 * d.nnz);
    d.hslot_b = (uint16_t *)b->dget(2 * d.nnz);
    d.dslot = (uint16_t *)b->dget(2 * d.nnz);
    d.gdamp = b->dget(4 * d.nnz);
    d.cell_start = (int32_t *)b->dget(4 * (n / 8 + 2));
    d.partB = (double *)b->dget(16 * (n / 32 + 1));
    d.partC = (double *)b->dget(32 * d.nblocks);
    d.win_buf = (double *)b->dget(8 * 1000);
    d.st = (DevState *)b->dget(sizeof(DevState));
    void *scratch = b->dget(44 * n);   // setup scratch
    if (!d.X || !d.u || !d.uh || !d.v || !d.B0 || !d.T || !d.clamped || !d.row_ptr || !d.col || !d.hslot_a ||
        !d.hslot_b || !d.dslot || !d.gdamp || !d.cell_start || !d.partB || !d.partC || !d.win_buf || !d.st || !scratch) {
        b->dput(scratch);
        free_body(b);
        return fail(TLSPH_E_NOMEM, "pool exhausted (mock)");
    }
    b->dput(scratch);
    memset(d.st, 0, sizeof(DevState));
    d.row_max = desc->dim == 3 ? 80 : 20;
    d.halo_a = d.halo_b = d.halo_max = 100;
    d.ga.zb = 5;
    d.gb.zb = 3;
    b->material_set = true;
    *out = b;
    return TLSPH_OK;
}

void free_body(tlsph_body b)
{
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(g_live_m);
        g_live_st.erase(b->db.st);
    }
    DeviceBody &d = b->db;
    void *ptrs[] = {d.X, d.u, d.uh, d.v, d.B0, d.T, d.accel, d.clamped, d.row_ptr, d.col, d.hslot_a, d.hslot_b,
                    d.dslot, d.gdamp, d.cell_start, d.partB, d.partC, d.win_buf, d.st};
    for (void *p : ptrs) b->dput(p);
    delete b;
}

tlsph_status pull_state(tlsph_body b)
{
    *b->hst = *b->db.st;
    return TLSPH_OK;
}

tlsph_status download_field(tlsph_body b, const void *src, bool, double *dst)
{
    {
        std::lock_guard<std::mutex> lk(g_live_m);
        if (!g_live_st.count(b->db.st)) die("download from a body that is not live");
    }
    (void)src;
    for (int64_t q = 0; q < b->n * b->dim; ++q) dst[q] = 1.0;
    return TLSPH_OK;
}

bool body_damped(tlsph_body b, int64_t n) { return b->damping_set && damped_step(b->seed, b->alpha, n); }

void fill_inst(tlsph_body b, Inst &I)
{
    memset(&I, 0, sizeof I);
    I.P.n = b->n;
    I.row_max = b->db.row_max;
    I.halo_a = b->db.halo_a;
    I.halo_b = b->db.halo_b;
    I.halo_max = b->db.halo_max;
    I.ga = b->db.ga;
    I.gb = b->db.gb;
    I.nbA = 1;
    I.nbB = 1;
    I.nbC = b->db.nblocks;
    I.scheme = b->scheme;
    I.X = b->db.X;
    I.u = b->db.u;
    I.win_buf = b->db.win_buf;
    I.st = b->db.st;
    I.nc[0] = b->dim;   // the dimension, for the launch checks
}

void launch_init_dt(const DeviceBody &, const StepParams &, int, double, double, hipStream_t) {}

void launch_control(DevState *st, const double *, int stop, double tol, int64_t max_step, hipStream_t)
{
    st->stop_on_converge = stop;
    st->tol = tol;
    st->max_step = max_step;
    st->done = 0;
    st->win = 1;
    std::lock_guard<std::mutex> lk(g_live_m);
    g_live_st.insert(st);
}

int damp_pairs_per_lane(int row_max) { return (row_max + 15) / 16; }

static void check_rows(const char *what, const Inst *I, const Inst *h, const int *slots, int count, int dim)
{
    if (count <= 0 || count > kMaxBatch) die("%s: bad count %d", what, count);
    for (int k = 0; k < count; ++k) {
        const Inst &a = I[slots[k]];
        if (h && memcmp(&a, &h[slots[k]], sizeof(Inst)) != 0) die("%s: device table row %d differs from host", what, slots[k]);
        if (dim && a.nc[0] != dim) die("%s: row %d has dim %d, launch dim %d", what, slots[k], a.nc[0], dim);
        std::lock_guard<std::mutex> lk(g_live_m);
        if (!g_live_st.count(a.st)) die("%s: row %d points at a body that is not live", what, slots[k]);
    }
}

void launch_passA_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int, hipStream_t)
{
    check_rows("passA", I, h, slots, count, dim);
}
void launch_passB_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int, hipStream_t)
{
    check_rows("passB", I, h, slots, count, dim);
}
void launch_passC_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int, hipStream_t)
{
    check_rows("passC", I, h, slots, count, dim);
}
void launch_damp_batch(const Inst *I, const Inst *h, const int *slots, int count, int dim, int, int, bool,
                       hipStream_t)
{
    check_rows("damp", I, h, slots, count, dim);
    for (int k = 1; k < count; ++k)
        if (h[slots[k]].scheme != h[slots[0]].scheme) die("damp: one launch mixes damping schemes");
}
void launch_finish_batch(const Inst *I, const int *slots, int count, hipStream_t)
{
    check_rows("finish", I, nullptr, slots, count, 0);
    for (int k = 0; k < count; ++k) {
        DevState *st = I[slots[k]].st;
        if (st->done) continue;
        st->step += 1;
        // converge after a body-specific number of steps
        const int64_t target = 20 + (I[slots[k]].P.n % 97);
        if (st->step >= target) {
            st->resid = 0.0;
            st->done = 1;
        } else {
            st->resid = 1.0;
        }
        if (st->step >= st->max_step) st->done = 1;
    }
}
void launch_gather_state(const Inst *I, const int *slots, int count, DevState *out, hipStream_t)
{
    check_rows("gather", I, nullptr, slots, count, 0);
    for (int k = 0; k < count; ++k) out[k] = *I[slots[k]].st;
}

}  // namespace tlsph

using namespace tlsph;

extern "C" {
const char *tlsph_last_error(void) { return g_err_mock.c_str(); }
tlsph_status tlsph_set_material(tlsph_body b, int, double, double)
{
    b->material_set = true;
    return TLSPH_OK;
}
tlsph_status tlsph_set_loads(tlsph_body, const double *, const double *) { return TLSPH_OK; }
tlsph_status tlsph_set_damping_scheme(tlsph_body b, int scheme)
{
    b->scheme = scheme;
    return TLSPH_OK;
}
tlsph_status tlsph_set_damping(tlsph_body b, double, double, double, double alpha, uint64_t seed)
{
    b->damping_set = true;
    b->eta = 1.0;
    b->alpha = alpha;
    b->seed = seed;
    return TLSPH_OK;
}
}

// ---- stress driver ----
static void *pool_alloc(size_t n, void *) { return malloc(n); }
static void pool_free(void *p, void *) { free(p); }

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? atoi(argv[1]) : 20;
    std::mt19937_64 rng(42);
    for (int round = 0; round < rounds; ++round) {
        const size_t budget = (round % 3 == 0) ? (size_t)(6u << 20) : (size_t)(256u << 20);
        tlsph_allocator al{pool_alloc, pool_free, nullptr};
        tlsph_server S = nullptr;
        const int slots = 1 + (int)(rng() % 32);
        if (tlsph_server_create(budget, slots, 32, nullptr, al, &S) != TLSPH_OK) die("create: %s", tlsph_last_error());
        const int nreq = 10 + (int)(rng() % 40);
        std::vector<int64_t> tickets;
        std::vector<std::vector<double>> X(nreq);
        for (int r = 0; r < nreq; ++r) {
            tlsph_request q{};
            q.body.dim = (rng() & 1) ? 2 : 3;
            q.body.n = (rng() % 10 == 0) ? 2 : 200 + (int64_t)(rng() % 20000);
            X[r].assign((size_t)q.body.n * q.body.dim, 0.0);
            q.body.X0 = X[r].data();
            q.body.dp = 0.002;
            q.body.h_over_dp = 1.3;
            q.body.rho0 = 1000;
            q.model = 1;
            q.E = 1e6;
            q.nu = 0.3;
            q.beta = 1;
            q.Lc = 0.01;
            q.alpha = 0.2;
            q.seed = r;
            q.scheme = (int)(rng() & 1);
            q.tol = 1e-4;
            q.max_steps = (rng() % 5 == 0) ? 7 : 1000;
            int64_t t;
            if (tlsph_server_submit(S, &q, &t) != TLSPH_OK) die("submit: %s", tlsph_last_error());
            tickets.push_back(t);
            if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        }
        int done_ok = 0, failed = 0;
        for (int64_t t : tickets) {
            int done = 0;
            tlsph_status st;
            tlsph_report rep;
            while (!done)
                if (tlsph_server_wait(S, t, 1.0, &done, &st, &rep) != TLSPH_OK) die("wait");
            if (st >= 0) {
                std::vector<double> u(1 << 20);
                ++done_ok;
            } else {
                ++failed;
            }
        }
        tlsph_server_stats ss;
        tlsph_server_stats_get(S, &ss);
        if (ss.completed != nreq) die("completed %lld of %d", (long long)ss.completed, nreq);
        tlsph_server_destroy(S);
        printf("round %d: slots %d, %d requests, %d ok, %d failed, peak active %lld\n", round, slots, nreq, done_ok,
               failed, (long long)ss.peak_active);
    }
    printf("mock server ok\n");
    return 0;
}
