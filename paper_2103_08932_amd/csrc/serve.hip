// serve.hip -- request server: continuous batching of relaxation solves (tlsph_server_* of
// tlsph_dr.h).
//
// Threads and streams:
//   caller    tlsph_server_submit copies a request into the pending queue.
//   worker    admits the oldest pending request when a slot is free and its estimated device
//             footprint fits in the largest free range of the pool, then builds the body (cell
//             binning, neighbour lists, B0, slots; the setup of tlsph_create_body) on the setup
//             stream, sets material / loads / damping, arms the stop rule and hands it to the
//             batch thread.  Setup kernels overlap the batch's steps.
//   batch     runs chunks of steps over every active body: per step, pass A and pass B as one
//             launch per dimension, the damping sweep over the bodies whose random choice picked
//             the step, pass C per dimension and one finish launch (one workgroup per body).
//             3D bodies run on one stream, 2D bodies on another, so their launches overlap.  After
//             a chunk the device states are gathered in one copy; a body that converged, hit its
//             step limit or failed leaves the batch: its displacement is copied out and its
//             memory returned to the pool, which may let the worker admit the next request.
//
// Device memory comes from one pool taken from the caller's allocator at creation and
// sub-allocated here (first fit, coalescing), so serving never calls hipMalloc / hipFree.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tlsph_dr.h"
#include "body.hpp"
#include "internal.hpp"

using namespace tlsph;

namespace {

constexpr size_t kAlign = 256;

// First-fit sub-allocator over one device range.  Thread safe.
class Pool {
  public:
    void init(char *base, size_t size)
    {
        base_ = base;
        size_ = size;
        free_.clear();
        used_.clear();
        if (size) free_[0] = size;
    }
    void *get(size_t bytes)
    {
        bytes = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
        std::lock_guard<std::mutex> lk(m_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_[off] = bytes;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        return nullptr;
    }
    void put(void *p)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(m_);
        const size_t off = (size_t)((char *)p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto nx = free_.lower_bound(off);
        if (nx != free_.begin()) {           // merge with the free range just below
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        nx = free_.find(start + len);        // and with the one just above
        if (nx != free_.end()) {
            len += nx->second;
            free_.erase(nx);
        }
        free_[start] = len;
    }
    size_t largest_free()
    {
        std::lock_guard<std::mutex> lk(m_);
        size_t b = 0;
        for (auto &f : free_) b = std::max(b, f.second);
        return b;
    }
    size_t size() const { return size_; }
    size_t in_use()
    {
        std::lock_guard<std::mutex> lk(m_);
        return in_use_;
    }
    size_t peak()
    {
        std::lock_guard<std::mutex> lk(m_);
        return peak_;
    }
    static void *cb_get(size_t bytes, void *ctx) { return static_cast<Pool *>(ctx)->get(bytes); }
    static void cb_put(void *p, void *ctx) { static_cast<Pool *>(ctx)->put(p); }

  private:
    char *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;             // offset -> length
    std::unordered_map<size_t, size_t> used_;   // offset -> length
    size_t in_use_ = 0, peak_ = 0;
    std::mutex m_;
};

// Upper estimate of a body's device footprint during setup (the peak): per particle the state,
// B0, T, row offsets and setup scratch; per CSR entry the column, two halo slots and the damping
// factor; neighbour rows of a lattice at h = 1.3 dp hold 20 (2D) / 80 (3D) entries, taken with a
// margin for irregular bodies.
size_t estimate_bytes(int dim, int64_t n, int precision, bool accel)
{
    const size_t R = precision == 32 ? 4 : 8, D = (size_t)dim;
    const size_t per_particle = 3 * 8 * D + R * D + 2 * R * D * D + (accel ? R * D : 0) + 1 + 8 + 16 + 32 +
                                8 * D + 1 + 4 + 4 + 4 + 8 + 16;
    const size_t per_pair = 4 + 2 + 2 + R;
    const size_t pairs = (size_t)n * (dim == 3 ? 96 : 26);
    return (size_t)n * per_particle + pairs * per_pair + 64 * kAlign + (1u << 16);
}

double now_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
    int64_t ticket = 0;
    // copied inputs
    int dim = 0;
    int64_t n = 0;
    std::vector<double> X0, accel;
    std::vector<uint8_t> clamped;
    double dp = 0, h_over_dp = 0, rho0 = 0;
    int model = 0;
    double E = 0, nu = 0, g[3] = {0, 0, 0};
    double eta = 0, beta = 0, Lc = 0, alpha = 1;
    uint64_t seed = 0;
    double tol = 0;
    int64_t max_steps = 0;
    size_t need = 0;
    // progress
    tlsph_body body = nullptr;
    int64_t damped = 0;               // damped steps executed so far
    int slot = -1;
    bool done = false;
    tlsph_status status = TLSPH_OK;
    std::string err;
    tlsph_report rep{};
    std::vector<double> u;
    bool result_taken = false;
    double t[4] = {-1, -1, -1, -1};
};

}  // namespace

struct tlsph_server_s {
    int precision = 32;
    int max_slots = 0;
    int device = 0;
    tlsph_allocator alloc{};
    void *pool_mem = nullptr;
    Pool pool;
    hipStream_t s3 = nullptr, s2 = nullptr, ssetup = nullptr;
    bool own_s3 = false;
    std::chrono::steady_clock::time_point t0;

    std::mutex m;
    std::condition_variable cv_worker, cv_batch, cv_done;
    bool stop = false;
    std::deque<Request *> pending;
    std::vector<Request *> ready;
    std::map<int64_t, Request *> reqs;
    std::vector<char> slot_used;
    int64_t next_ticket = 1;
    int64_t retirements = 0;          // bumped whenever memory or a slot is returned
    tlsph_server_stats stats{};
    int in_setup = 0;

    // batch thread
    Inst *table_dev = nullptr, *table_host = nullptr;   // one row per slot
    DevState *st_dev = nullptr, *st_host = nullptr;     // gathered states (one per active body)
    DevState *mirrors = nullptr;                        // pinned state mirror of each slot
    std::vector<Request *> active;
    int chunk = 16;

    std::thread worker, batcher;
};

namespace {

void release_slot_locked(tlsph_server S, int slot)
{
    if (slot >= 0) S->slot_used[slot] = 0;
    S->retirements += 1;
}

int take_slot_locked(tlsph_server S)
{
    for (int k = 0; k < S->max_slots; ++k)
        if (!S->slot_used[k]) {
            S->slot_used[k] = 1;
            return k;
        }
    return -1;
}

void finish_request(tlsph_server S, Request *r, tlsph_status st, const std::string &err)
{
    std::lock_guard<std::mutex> lk(S->m);
    r->status = st;
    r->err = err;
    r->done = true;
    r->t[3] = now_since(S->t0);
    r->rep.wall_s = r->t[3] - r->t[0];
    if (st < 0) S->stats.failed += 1;
    S->stats.completed += 1;
    S->cv_done.notify_all();
}

// Builds, configures and arms the body of `r` on the setup stream.  Returns TLSPH_OK or an error
// (the body is then released).
tlsph_status setup_request(tlsph_server S, Request *r)
{
    tlsph_body_desc d{};
    d.dim = r->dim;
    d.n = r->n;
    d.X0 = r->X0.data();
    d.clamped = r->clamped.empty() ? nullptr : r->clamped.data();
    d.dp = r->dp;
    d.h_over_dp = r->h_over_dp;
    d.rho0 = r->rho0;
    d.precision = S->precision;
    d.stream = S->ssetup;
    d.alloc.alloc = Pool::cb_get;
    d.alloc.free = Pool::cb_put;
    d.alloc.ctx = &S->pool;
    tlsph_body b = nullptr;
    tlsph_status st = create_body(&d, S->mirrors + r->slot, &b);
    if (st != TLSPH_OK) return st;
    st = tlsph_set_material(b, r->model, r->E, r->nu);
    if (st == TLSPH_OK) st = tlsph_set_loads(b, r->g, r->accel.empty() ? nullptr : r->accel.data());
    if (st == TLSPH_OK && (r->eta > 0.0 || r->beta > 0.0))
        st = tlsph_set_damping(b, r->eta, r->beta, r->Lc, r->alpha, r->seed);
    if (st != TLSPH_OK) {
        free_body(b);
        return st;
    }
    // the column indices are only needed to build the slots and the damping factors
    S->pool.put(b->db.col);
    b->db.col = nullptr;
    // the first time step (Eq. 18 at rest) and the stop rule
    launch_init_dt(b->db, b->P, b->precision, b->bmax, 0.0, b->stream);
    b->dt_valid = true;
    launch_control(b->db.st, b->db.win_buf, 1, r->tol, r->max_steps, b->stream);
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        free_body(b);
        return fail(TLSPH_E_DEVICE, "HIP error while arming a served body");
    }
    r->body = b;
    return TLSPH_OK;
}

void worker_main(tlsph_server S)
{
    (void)hipSetDevice(S->device);
    int64_t blocked_at = -1;   // retirement count at the last admission that ran out of memory
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->m);
            S->cv_worker.wait(lk, [&] {
                if (S->stop) return true;
                if (S->pending.empty()) return false;
                if (blocked_at == S->retirements) return false;
                if (std::find(S->slot_used.begin(), S->slot_used.end(), 0) == S->slot_used.end()) return false;
                const bool alone = S->active.empty() && S->ready.empty() && S->in_setup == 0;
                return alone || S->pool.largest_free() >= S->pending.front()->need;
            });
            if (S->stop) return;
            r = S->pending.front();
            S->pending.pop_front();
            r->slot = take_slot_locked(S);
            S->in_setup += 1;
            S->stats.pending -= 1;
            S->stats.in_setup += 1;
            r->t[1] = now_since(S->t0);
        }
        const tlsph_status st = setup_request(S, r);
        const std::string msg = st == TLSPH_OK ? std::string() : std::string(tlsph_last_error());
        if (st == TLSPH_OK) {   // the inputs live on the device now
            std::vector<double>().swap(r->X0);
            std::vector<double>().swap(r->accel);
            std::vector<uint8_t>().swap(r->clamped);
        }
        std::unique_lock<std::mutex> lk(S->m);
        S->in_setup -= 1;
        S->stats.in_setup -= 1;
        if (st == TLSPH_OK) {
            S->ready.push_back(r);
            S->cv_batch.notify_all();
            continue;
        }
        const bool others = !S->active.empty() || !S->ready.empty() || S->in_setup > 0;
        release_slot_locked(S, r->slot);
        r->slot = -1;
        if (st == TLSPH_E_NOMEM && others) {
            // wait for memory to be returned, then try again (the request keeps its place)
            S->pending.push_front(r);
            S->stats.pending += 1;
            blocked_at = S->retirements;
            continue;
        }
        lk.unlock();
        finish_request(S, r, st, msg);
    }
}

// Copies the displacement and the report of a body that left the batch, then releases it.
void retire(tlsph_server S, Request *r, const DevState &ds)
{
    tlsph_body b = r->body;
    *b->hst = ds;
    b->step = ds.step;
    tlsph_status st = TLSPH_OK;
    std::string msg;
    if (ds.error) {
        st = (tlsph_status)ds.error;
        msg = "non-finite state or inverted particle (J <= 0) at step " + std::to_string((long long)ds.step);
    } else {
        const bool conv = ds.resid < r->tol && ds.step >= ds.win;
        st = conv ? TLSPH_OK : TLSPH_NOT_CONVERGED;
        r->u.resize((size_t)r->n * r->dim);
        const tlsph_status s2 = download_field(b, b->db.u, false, r->u.data());
        if (s2 != TLSPH_OK) {
            st = s2;
            msg = tlsph_last_error();
        }
    }
    tlsph_report &rep = r->rep;
    rep.steps = ds.step;
    rep.damped_steps = r->damped;
    rep.step_index = ds.step;
    rep.residual = ds.resid;
    rep.kinetic_energy = ds.ek;
    rep.force_residual = ds.fres;
    rep.dt = ds.dt;
    rep.window = ds.win;
    rep.converged = (ds.resid < r->tol && ds.step >= ds.win) ? 1 : 0;
    free_body(b);
    r->body = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->m);
        release_slot_locked(S, r->slot);
        r->slot = -1;
        S->stats.active -= 1;
        S->cv_worker.notify_all();
    }
    finish_request(S, r, st, msg);
}

// Enqueues nsteps (<= 64) steps of every body in rows[0] (2D) and rows[1] (3D); bit q of
// masks[row] records whether step q of the chunk damps that body.
void enqueue_chunk(tlsph_server S, const std::vector<int> (&rows)[2], const std::vector<int64_t> &step0, int nsteps,
                   std::vector<uint64_t> &masks)
{
    const int prec = S->precision;
    const hipStream_t strm[2] = {S->s2, S->s3};
    std::vector<int> damped;
    for (int q = 0; q < nsteps; ++q) {
        for (int di = 0; di < 2; ++di) {
            const std::vector<int> &L = rows[di];
            if (L.empty()) continue;
            const int dim = di + 2;
            const hipStream_t s = strm[di];
            launch_passA_batch(S->table_dev, S->table_host, L.data(), (int)L.size(), dim, prec, s);
            launch_passB_batch(S->table_dev, S->table_host, L.data(), (int)L.size(), dim, prec, s);
            // the bodies whose random choice picks this step, grouped by the damping kernel's
            // pairs-per-lane so that every body runs the code it runs alone
            damped.clear();
            for (int row : L)
                if (body_damped(S->active[row]->body, step0[row] + q)) {
                    damped.push_back(row);
                    masks[row] |= uint64_t(1) << q;
                }
            if (!damped.empty()) {
                std::map<int, std::vector<int>> groups;
                for (int row : damped) groups[damp_pairs_per_lane(S->table_host[row].row_max)].push_back(row);
                const int K = dim == 3 ? 27 : 9;
                for (auto &gp : groups) {
                    const std::vector<int> &G = gp.second;
                    for (int c = 0; c < K; ++c)
                        launch_damp_batch(S->table_dev, S->table_host, G.data(), (int)G.size(), dim, prec, c, true, s);
                    for (int c = K - 1; c >= 0; --c)
                        launch_damp_batch(S->table_dev, S->table_host, G.data(), (int)G.size(), dim, prec, c, false,
                                          s);
                }
            }
            launch_passC_batch(S->table_dev, S->table_host, L.data(), (int)L.size(), dim, prec, s);
            launch_finish_batch(S->table_dev, L.data(), (int)L.size(), s);
        }
    }
}

void batch_main(tlsph_server S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        // admit the bodies that finished setup
        {
            std::unique_lock<std::mutex> lk(S->m);
            S->cv_batch.wait(lk, [&] { return S->stop || !S->active.empty() || !S->ready.empty(); });
            if (S->stop) return;
            for (Request *r : S->ready) {
                r->t[2] = now_since(S->t0);
                r->body->stream = r->dim == 3 ? S->s3 : S->s2;
                S->active.push_back(r);
                S->stats.active += 1;
            }
            S->ready.clear();
            S->stats.peak_active = std::max<int64_t>(S->stats.peak_active, (int64_t)S->active.size());
        }
        // table rows are the active list's order; rows[0] 2D, rows[1] 3D
        const int na = (int)S->active.size();
        std::vector<int> rows[2];
        std::vector<int64_t> step0(na);
        for (int k = 0; k < na; ++k) {
            Request *r = S->active[k];
            fill_inst(r->body, S->table_host[k]);
            rows[r->dim - 2].push_back(k);
            step0[k] = r->body->step;
        }
        if (hipMemcpyAsync(S->table_dev, S->table_host, sizeof(Inst) * na, hipMemcpyHostToDevice, S->s3) !=
                hipSuccess ||
            hipStreamSynchronize(S->s3) != hipSuccess) {
            // a device failure: fail every active request
            for (Request *r : S->active) {
                free_body(r->body);
                r->body = nullptr;
                {
                    std::lock_guard<std::mutex> lk(S->m);
                    release_slot_locked(S, r->slot);
                    S->stats.active -= 1;
                }
                finish_request(S, r, TLSPH_E_DEVICE, "HIP error uploading the batch table");
            }
            S->active.clear();
            continue;
        }
        std::vector<uint64_t> masks(na, 0);
        enqueue_chunk(S, rows, step0, S->chunk, masks);
        // gather the states: 2D rows on the 2D stream after its chunk, 3D rows on the 3D stream
        const hipStream_t strm[2] = {S->s2, S->s3};
        int off = 0;
        std::vector<int> order;
        bool ok = true;
        for (int di = 0; di < 2; ++di) {
            const std::vector<int> &L = rows[di];
            if (L.empty()) continue;
            launch_gather_state(S->table_dev, L.data(), (int)L.size(), S->st_dev + off, strm[di]);
            ok = ok && hipMemcpyAsync(S->st_host + off, S->st_dev + off, sizeof(DevState) * L.size(),
                                      hipMemcpyDeviceToHost, strm[di]) == hipSuccess;
            for (int row : L) order.push_back(row);
            off += (int)L.size();
        }
        ok = ok && hipStreamSynchronize(S->s2) == hipSuccess && hipStreamSynchronize(S->s3) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(S->m);
            S->stats.chunks += 1;
            S->stats.batch_steps += S->chunk;
        }
        std::vector<Request *> keep;
        std::vector<char> leave(na, 0);
        for (int q = 0; q < (int)order.size(); ++q) {
            const int row = order[q];
            Request *r = S->active[row];
            const DevState &ds = S->st_host[q];
            if (!ok) {
                leave[row] = 1;
                continue;
            }
            const int64_t ran = std::min<int64_t>(std::max<int64_t>(ds.step - step0[row], 0), S->chunk);
            const uint64_t m = ran >= 64 ? masks[row] : masks[row] & ((uint64_t(1) << ran) - 1);
            r->damped += __builtin_popcountll(m);
            r->body->step = ds.step;
            *r->body->hst = ds;
            if (ds.done || ds.error) {
                leave[row] = 1;
                retire(S, r, ds);
            }
        }
        for (int k = 0; k < na; ++k) {
            Request *r = S->active[k];
            if (!ok && leave[k]) {
                free_body(r->body);
                r->body = nullptr;
                {
                    std::lock_guard<std::mutex> lk(S->m);
                    release_slot_locked(S, r->slot);
                    S->stats.active -= 1;
                    S->cv_worker.notify_all();
                }
                finish_request(S, r, TLSPH_E_DEVICE, "HIP error in a batch chunk");
            } else if (!leave[k]) {
                keep.push_back(r);
            }
        }
        S->active.swap(keep);
    }
}

void destroy_server(tlsph_server S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
        S->cv_worker.notify_all();
        S->cv_batch.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (S->batcher.joinable()) S->batcher.join();
    if (S->s3) (void)hipStreamSynchronize(S->s3);
    if (S->s2) (void)hipStreamSynchronize(S->s2);
    if (S->ssetup) (void)hipStreamSynchronize(S->ssetup);
    for (Request *r : S->active)
        if (r->body) free_body(r->body);
    for (Request *r : S->ready)
        if (r->body) free_body(r->body);
    for (auto &kv : S->reqs) delete kv.second;
    S->reqs.clear();
    if (S->pool_mem) S->alloc.free(S->pool_mem, S->alloc.ctx);
    if (S->table_host) (void)hipHostFree(S->table_host);
    if (S->st_host) (void)hipHostFree(S->st_host);
    if (S->mirrors) (void)hipHostFree(S->mirrors);
    if (S->s2) (void)hipStreamDestroy(S->s2);
    if (S->ssetup) (void)hipStreamDestroy(S->ssetup);
    if (S->own_s3 && S->s3) (void)hipStreamDestroy(S->s3);
    delete S;
}

void *hip_alloc(size_t bytes, void *)
{
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void hip_free(void *p, void *)
{
    if (p) (void)hipFree(p);
}

Request *find_locked(tlsph_server S, int64_t ticket)
{
    auto it = S->reqs.find(ticket);
    return it == S->reqs.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

tlsph_status tlsph_server_create(size_t hbm_budget, int max_slots, int precision, void *stream, tlsph_allocator alloc,
                                 tlsph_server *out)
{
    if (!out) return fail(TLSPH_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxBatch)
        return fail(TLSPH_E_INVALID, "max_slots must be in 1..%d (got %d)", kMaxBatch, max_slots);
    if (precision != TLSPH_FP32 && precision != TLSPH_FP64)
        return fail(TLSPH_E_INVALID, "precision must be TLSPH_FP32 or TLSPH_FP64");
    const size_t fixed = 2 * (size_t)max_slots * (sizeof(Inst) + sizeof(DevState)) + 4 * kAlign;
    if (hbm_budget < fixed + (1u << 20)) return fail(TLSPH_E_INVALID, "hbm_budget of %zu bytes is too small", hbm_budget);
    tlsph_server S = new (std::nothrow) tlsph_server_s();
    if (!S) return fail(TLSPH_E_NOMEM, "host allocation failed");
    S->precision = precision;
    S->max_slots = max_slots;
    S->alloc = alloc;
    if (!S->alloc.alloc || !S->alloc.free) {
        S->alloc.alloc = hip_alloc;
        S->alloc.free = hip_free;
        S->alloc.ctx = nullptr;
    }
    S->t0 = std::chrono::steady_clock::now();
    S->slot_used.assign(max_slots, 0);
    if (const char *c = getenv("TLSPH_SERVE_CHUNK")) S->chunk = std::min(64, std::max(1, atoi(c)));
    (void)hipGetDevice(&S->device);
    S->pool_mem = S->alloc.alloc(hbm_budget, S->alloc.ctx);
    if (!S->pool_mem) {
        destroy_server(S);
        return fail(TLSPH_E_NOMEM, "could not allocate the server pool of %zu bytes", hbm_budget);
    }
    S->pool.init((char *)S->pool_mem, hbm_budget);
    S->table_dev = (Inst *)S->pool.get(sizeof(Inst) * max_slots);
    S->st_dev = (DevState *)S->pool.get(sizeof(DevState) * max_slots);
    if (hipHostMalloc((void **)&S->table_host, sizeof(Inst) * max_slots, hipHostMallocDefault) != hipSuccess)
        S->table_host = nullptr;
    if (hipHostMalloc((void **)&S->st_host, sizeof(DevState) * max_slots, hipHostMallocDefault) != hipSuccess)
        S->st_host = nullptr;
    if (hipHostMalloc((void **)&S->mirrors, sizeof(DevState) * max_slots, hipHostMallocDefault) != hipSuccess)
        S->mirrors = nullptr;
    if (!S->table_dev || !S->st_dev || !S->table_host || !S->st_host || !S->mirrors) {
        destroy_server(S);
        return fail(TLSPH_E_NOMEM, "server tables could not be allocated");
    }
    S->s3 = (hipStream_t)stream;
    if (!S->s3) {
        if (hipStreamCreateWithFlags(&S->s3, hipStreamNonBlocking) != hipSuccess) {
            S->s3 = nullptr;
            destroy_server(S);
            return fail(TLSPH_E_DEVICE, "hipStreamCreate failed");
        }
        S->own_s3 = true;
    }
    if (hipStreamCreateWithFlags(&S->s2, hipStreamNonBlocking) != hipSuccess) {
        S->s2 = nullptr;
        destroy_server(S);
        return fail(TLSPH_E_DEVICE, "hipStreamCreate failed");
    }
    if (hipStreamCreateWithFlags(&S->ssetup, hipStreamNonBlocking) != hipSuccess) {
        S->ssetup = nullptr;
        destroy_server(S);
        return fail(TLSPH_E_DEVICE, "hipStreamCreate failed");
    }
    try {
        S->worker = std::thread(worker_main, S);
        S->batcher = std::thread(batch_main, S);
    } catch (...) {
        destroy_server(S);
        return fail(TLSPH_E_NOMEM, "could not start the server threads");
    }
    *out = S;
    return TLSPH_OK;
}

tlsph_status tlsph_server_submit(tlsph_server S, const tlsph_request *q, int64_t *ticket)
{
    if (!S || !q || !ticket) return fail(TLSPH_E_INVALID, "server, request or ticket is NULL");
    const tlsph_body_desc &d = q->body;
    if (d.dim != 2 && d.dim != 3) return fail(TLSPH_E_INVALID, "dim must be 2 or 3 (got %d)", d.dim);
    if (!d.X0 || d.n < 1 || d.n >= ((int64_t)1 << 31) - 1) return fail(TLSPH_E_INVALID, "bad particle arrays");
    if (!(d.dp > 0.0) || !(d.h_over_dp > 0.0) || !(d.rho0 > 0.0))
        return fail(TLSPH_E_INVALID, "dp, h_over_dp and rho0 must be positive");
    if (q->model != TLSPH_SVK && q->model != TLSPH_NEOHOOKE) return fail(TLSPH_E_INVALID, "unknown material model");
    if (!(q->E >= 0.0) || !(q->nu > -1.0 && q->nu < 0.5)) return fail(TLSPH_E_INVALID, "need E >= 0 and -1 < nu < 0.5");
    if ((q->eta > 0.0 || q->beta > 0.0) && !(q->alpha > 0.0 && q->alpha <= 1.0))
        return fail(TLSPH_E_INVALID, "alpha must be in (0, 1]");
    if (!(q->tol >= 0.0) || q->max_steps < 1) return fail(TLSPH_E_INVALID, "need tol >= 0 and max_steps >= 1");
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(TLSPH_E_NOMEM, "host allocation failed");
    try {
        r->dim = d.dim;
        r->n = d.n;
        r->X0.assign(d.X0, d.X0 + (size_t)d.n * d.dim);
        if (d.clamped) r->clamped.assign(d.clamped, d.clamped + d.n);
        if (q->accel) r->accel.assign(q->accel, q->accel + (size_t)d.n * d.dim);
    } catch (const std::bad_alloc &) {
        delete r;
        return fail(TLSPH_E_NOMEM, "host allocation failed");
    }
    r->dp = d.dp;
    r->h_over_dp = d.h_over_dp;
    r->rho0 = d.rho0;
    r->model = q->model;
    r->E = q->E;
    r->nu = q->nu;
    for (int k = 0; k < 3; ++k) r->g[k] = q->g[k];
    r->eta = q->eta;
    r->beta = q->beta;
    r->Lc = q->Lc;
    r->alpha = q->alpha;
    r->seed = q->seed;
    r->tol = q->tol;
    r->max_steps = q->max_steps;
    r->need = estimate_bytes(d.dim, d.n, S->precision, q->accel != nullptr);
    std::lock_guard<std::mutex> lk(S->m);
    r->ticket = S->next_ticket++;
    r->t[0] = now_since(S->t0);
    S->reqs[r->ticket] = r;
    S->pending.push_back(r);
    S->stats.submitted += 1;
    S->stats.pending += 1;
    S->cv_worker.notify_all();
    *ticket = r->ticket;
    return TLSPH_OK;
}

tlsph_status tlsph_server_wait(tlsph_server S, int64_t ticket, double timeout_s, int *done, tlsph_status *status,
                               tlsph_report *report)
{
    if (!S || !done) return fail(TLSPH_E_INVALID, "server or done is NULL");
    std::unique_lock<std::mutex> lk(S->m);
    Request *r = find_locked(S, ticket);
    if (!r) return fail(TLSPH_E_INVALID, "unknown ticket %lld", (long long)ticket);
    if (!r->done && timeout_s > 0.0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; });
    *done = r->done ? 1 : 0;
    if (r->done) {
        if (status) *status = r->status;
        if (report) *report = r->rep;
    }
    return TLSPH_OK;
}

tlsph_status tlsph_server_result(tlsph_server S, int64_t ticket, double *u_out)
{
    if (!S || !u_out) return fail(TLSPH_E_INVALID, "server or output is NULL");
    std::lock_guard<std::mutex> lk(S->m);
    Request *r = find_locked(S, ticket);
    if (!r) return fail(TLSPH_E_INVALID, "unknown ticket %lld", (long long)ticket);
    if (!r->done) return fail(TLSPH_E_INVALID, "request %lld has not finished", (long long)ticket);
    if (r->status < 0) return fail(r->status, "request %lld failed: %s", (long long)ticket, r->err.c_str());
    if (r->result_taken) return fail(TLSPH_E_INVALID, "the result of request %lld was already taken", (long long)ticket);
    memcpy(u_out, r->u.data(), sizeof(double) * r->u.size());
    std::vector<double>().swap(r->u);
    std::vector<double>().swap(r->X0);
    std::vector<double>().swap(r->accel);
    std::vector<uint8_t>().swap(r->clamped);
    r->result_taken = true;
    return TLSPH_OK;
}

tlsph_status tlsph_server_times(tlsph_server S, int64_t ticket, double times[4])
{
    if (!S || !times) return fail(TLSPH_E_INVALID, "server or times is NULL");
    std::lock_guard<std::mutex> lk(S->m);
    Request *r = find_locked(S, ticket);
    if (!r) return fail(TLSPH_E_INVALID, "unknown ticket %lld", (long long)ticket);
    for (int k = 0; k < 4; ++k) times[k] = r->t[k];
    return TLSPH_OK;
}

const char *tlsph_server_error(tlsph_server S, int64_t ticket)
{
    if (!S) return "";
    std::lock_guard<std::mutex> lk(S->m);
    Request *r = find_locked(S, ticket);
    return r ? r->err.c_str() : "";
}

tlsph_status tlsph_server_stats_get(tlsph_server S, tlsph_server_stats *out)
{
    if (!S || !out) return fail(TLSPH_E_INVALID, "server or out is NULL");
    std::lock_guard<std::mutex> lk(S->m);
    *out = S->stats;
    out->pool_bytes = S->pool.size();
    out->pool_used = S->pool.in_use();
    out->pool_peak = S->pool.peak();
    return TLSPH_OK;
}

void tlsph_server_destroy(tlsph_server S) { destroy_server(S); }

}  // extern "C"
