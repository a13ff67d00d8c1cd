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
//   groups    G batch groups (default 8), each with its own thread,
//             stream and launch table; the worker hands a set-up body to a group holding only bodies
//             of its dimension (or none), the fewest bodies first, and mixes dimensions only when no
//             such group exists: a group steps in lock step, so a 2D body grouped with a 3D body
//             would wait every step for the 3D body's launches (its 54-launch damping sweep above
//             all).  A group runs chunks of steps over its bodies: per step, pass A and pass B as
//             one launch per dimension, the damping sweep over the bodies whose random choice
//             picked the step, pass C per dimension and one finish launch (one workgroup per
//             body).  Groups step independently, so the latency-bound launches of one group (the
//             colour-by-colour damping sweep above all) overlap the work of the others, and a
//             damped step of one body holds up only the bodies of its own group.  After a chunk a
//             group gathers its bodies' device states in one copy; a body that converged, hit its
//             step limit or failed leaves the group: its displacement is copied out and its memory
//             returned to the pool, which may let the worker admit the next request.
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
// B0, T, the kernel-gradient row sums, row offsets, the damping cell order and setup scratch; per
// CSR entry the column, three halo slots (the bricks of passes A and B, the damping cells) and the
// damping factor; neighbour rows of a lattice at h = 1.3 dp hold 20 (2D) / 80 (3D) entries, taken
// with a margin for irregular bodies.
size_t estimate_bytes(int dim, int64_t n, int precision, bool accel)
{
    const size_t R = precision == 32 ? 4 : 8, D = (size_t)dim;
    const size_t per_particle = 3 * 8 * D + 2 * R * D + 2 * R * D * D + (accel ? R * D : 0) + 1 + 8 + 16 + 32 +
                                8 * D + 1 + 4 + 4 + 4 + 8 + 16 + 4;
    const size_t per_pair = 4 + 3 * 2 + R;
    const size_t pairs = (size_t)n * (dim == 3 ? 96 : 26);
    // bodies above 1M particles also keep compact pass-B brick maps (16 bytes per 64 neighbourhood
    // slots of a brick, at most 32 bytes per particle), above 2M compact damping neighbourhoods too
    // (132 bytes per cell, at most 36 bytes per particle for cells of 4 or more particles)
    const size_t compact = (n > 1000000 ? (size_t)n * 32 : 0) + (n > 2000000 ? (size_t)n * 36 : 0);
    // run descriptors of the bricks of both pair passes: 96 bytes per 3D brick, 48 per 2D brick,
    // within 16 bytes per particle for bricks of 12 (3D) or 6 (2D) particles or more on average
    const size_t runs = (size_t)n * 16;
    return (size_t)n * per_particle + pairs * per_pair + compact + runs + 64 * kAlign + (1u << 16);
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
    int scheme = 0;
    double tol = 0;
    int64_t max_steps = 0;
    size_t need = 0;
    // progress
    tlsph_body body = nullptr;
    int group = -1;                   // batch group the body was handed to
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

// One batch group: a thread, a stream and a launch table over the bodies it steps.
struct Group {
    int id = 0;
    hipStream_t stream = nullptr;
    bool own_stream = true;
    Inst *table_dev = nullptr, *table_host = nullptr;   // one row per body of the group
    DevState *st_dev = nullptr, *st_host = nullptr;     // gathered states
    std::vector<Request *> ready;                       // handed over by the worker (server mutex)
    std::vector<Request *> active;                      // group thread only
    int load = 0;                                       // bodies handed over, not yet retired (server mutex)
    int load_dim[2] = {0, 0};                           // of which 2D / 3D (server mutex)
    std::condition_variable cv;
    std::thread thread;
};

}  // namespace

struct tlsph_server_s {
    int precision = 32;
    int max_slots = 0;
    int device = 0;
    tlsph_allocator alloc{};
    void *pool_mem = nullptr;
    Pool pool;
    hipStream_t ssetup = nullptr;
    std::chrono::steady_clock::time_point t0;

    std::mutex m;
    std::condition_variable cv_worker, cv_done;
    bool stop = false;
    std::deque<Request *> pending;
    std::map<int64_t, Request *> reqs;
    std::vector<char> slot_used;
    int64_t next_ticket = 1;
    int64_t retirements = 0;          // bumped whenever memory or a slot is returned
    tlsph_server_stats stats{};
    int in_setup = 0;
    int in_groups = 0;                // bodies handed to groups and not yet retired
    DevState *mirrors = nullptr;      // pinned state mirror of each slot
    std::vector<Group *> groups;
    int chunk = 16;

    std::thread worker;
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
    if (st == TLSPH_OK) st = tlsph_set_damping_scheme(b, r->scheme);
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
                const bool alone = S->in_groups == 0 && S->in_setup == 0;
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
            // a group without bodies of the other dimension, the fewest bodies first (ties: the
            // lowest id); a mixed group only when every group holds the other dimension
            const int di = r->dim - 2;
            Group *best = nullptr;
            bool best_mix = false;
            for (Group *g : S->groups) {
                const bool mix = g->load_dim[1 - di] > 0;
                if (!best || (!mix && best_mix) || (mix == best_mix && g->load < best->load)) {
                    best = g;
                    best_mix = mix;
                }
            }
            best->ready.push_back(r);
            best->load += 1;
            best->load_dim[di] += 1;
            r->group = best->id;
            S->in_groups += 1;
            best->cv.notify_all();
            continue;
        }
        const bool others = S->in_groups > 0 || S->in_setup > 0;
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

// Releases a body that left its group and hands the slot back to the worker.
void drop_body(tlsph_server S, Request *r)
{
    free_body(r->body);
    r->body = nullptr;
    std::lock_guard<std::mutex> lk(S->m);
    release_slot_locked(S, r->slot);
    r->slot = -1;
    S->groups[r->group]->load -= 1;
    S->groups[r->group]->load_dim[r->dim - 2] -= 1;
    S->in_groups -= 1;
    S->stats.active -= 1;
    S->cv_worker.notify_all();
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
        msg = std::string(step_error_text(ds.error)) + " at step " + std::to_string((long long)ds.step);
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
    drop_body(S, r);
    finish_request(S, r, st, msg);
}

// Enqueues nsteps (<= 64) steps of every body of the group; bit q of masks[row] records whether
// step q of the chunk damps that body.
void enqueue_chunk(tlsph_server S, Group *G, const std::vector<int> (&rows)[2], const std::vector<int64_t> &step0,
                   int nsteps, std::vector<uint64_t> &masks)
{
    const int prec = S->precision;
    const hipStream_t s = G->stream;
    std::vector<int> damped;
    std::map<int, std::vector<int>> by_p;
    for (int q = 0; q < nsteps; ++q) {
        for (int di = 0; di < 2; ++di) {
            const std::vector<int> &L = rows[di];
            if (L.empty()) continue;
            const int dim = di + 2;
            launch_passA_batch(G->table_dev, G->table_host, L.data(), (int)L.size(), dim, prec, s);
            launch_passB_batch(G->table_dev, G->table_host, L.data(), (int)L.size(), dim, prec, s);
            // the bodies whose random choice picks this step, grouped by the damping kernel's
            // pairs-per-lane and scheme so that every body runs the code it runs alone
            damped.clear();
            for (int row : L)
                if (body_damped(G->active[row]->body, step0[row] + q)) {
                    damped.push_back(row);
                    masks[row] |= uint64_t(1) << q;
                }
            if (!damped.empty()) {
                by_p.clear();
                for (int row : damped)
                    by_p[2 * damp_pairs_per_lane(G->table_host[row].row_max) + G->table_host[row].scheme].push_back(row);
                const int K = dim == 3 ? 27 : 9;
                for (auto &gp : by_p) {
                    const std::vector<int> &B = gp.second;
                    for (int c = 0; c < K; ++c)
                        launch_damp_batch(G->table_dev, G->table_host, B.data(), (int)B.size(), dim, prec, c, true, s);
                    for (int c = K - 1; c >= 0; --c)
                        launch_damp_batch(G->table_dev, G->table_host, B.data(), (int)B.size(), dim, prec, c, false,
                                          s);
                }
            }
            launch_passC_batch(G->table_dev, G->table_host, L.data(), (int)L.size(), dim, prec, s);
            launch_finish_batch(G->table_dev, L.data(), (int)L.size(), s);
        }
    }
}

void group_main(tlsph_server S, Group *G)
{
    (void)hipSetDevice(S->device);
    bool dirty = true;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->m);
            G->cv.wait(lk, [&] { return S->stop || !G->active.empty() || !G->ready.empty(); });
            if (S->stop) return;
            for (Request *r : G->ready) {
                r->t[2] = now_since(S->t0);
                r->body->stream = G->stream;
                G->active.push_back(r);
                S->stats.active += 1;
                dirty = true;
            }
            G->ready.clear();
            S->stats.peak_active = std::max<int64_t>(S->stats.peak_active, S->stats.active);
        }
        // table rows follow the active list; rows[0] 2D, rows[1] 3D
        const int na = (int)G->active.size();
        std::vector<int> rows[2];
        std::vector<int64_t> step0(na);
        for (int k = 0; k < na; ++k) {
            Request *r = G->active[k];
            rows[r->dim - 2].push_back(k);
            step0[k] = r->body->step;
        }
        bool ok = true;
        if (dirty) {
            // the previous upload has completed (every chunk ends with a stream synchronisation)
            for (int k = 0; k < na; ++k) fill_inst(G->active[k]->body, G->table_host[k]);
            ok = hipMemcpyAsync(G->table_dev, G->table_host, sizeof(Inst) * na, hipMemcpyHostToDevice, G->stream) ==
                 hipSuccess;
            dirty = false;
        }
        std::vector<uint64_t> masks(na, 0);
        if (ok) enqueue_chunk(S, G, rows, step0, S->chunk, masks);
        // gather the states, 2D rows first
        std::vector<int> order;
        for (int di = 0; di < 2; ++di)
            for (int row : rows[di]) order.push_back(row);
        if (ok) {
            launch_gather_state(G->table_dev, order.data(), na, G->st_dev, G->stream);
            ok = hipMemcpyAsync(G->st_host, G->st_dev, sizeof(DevState) * na, hipMemcpyDeviceToHost, G->stream) ==
                 hipSuccess;
        }
        ok = ok && hipStreamSynchronize(G->stream) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(S->m);
            S->stats.chunks += 1;
            S->stats.batch_steps += S->chunk;
        }
        // bodies that leave the group; the others keep their rows' order, so the uploaded table
        // stays valid until the membership changes
        std::vector<char> leave(na, 0);
        for (int q = 0; q < na; ++q) {
            const int row = order[q];
            Request *r = G->active[row];
            leave[row] = 1;
            if (!ok) {
                drop_body(S, r);
                finish_request(S, r, TLSPH_E_DEVICE, "HIP error in a batch chunk");
                continue;
            }
            const DevState &ds = G->st_host[q];
            const int64_t ran = std::min<int64_t>(std::max<int64_t>(ds.step - step0[row], 0), S->chunk);
            const uint64_t m = ran >= 64 ? masks[row] : masks[row] & ((uint64_t(1) << ran) - 1);
            r->damped += __builtin_popcountll(m);
            r->body->step = ds.step;
            *r->body->hst = ds;
            if (ds.done || ds.error) {
                retire(S, r, ds);
            } else {
                leave[row] = 0;
            }
        }
        std::vector<Request *> keep;
        for (int k = 0; k < na; ++k)
            if (!leave[k]) keep.push_back(G->active[k]);
        if ((int)keep.size() != na) dirty = true;
        G->active.swap(keep);
    }
}

void destroy_server(tlsph_server S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
        S->cv_worker.notify_all();
        for (Group *g : S->groups) g->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (Group *g : S->groups)
        if (g->thread.joinable()) g->thread.join();
    if (S->ssetup) (void)hipStreamSynchronize(S->ssetup);
    for (Group *g : S->groups) {
        if (g->stream) (void)hipStreamSynchronize(g->stream);
        for (Request *r : g->active)
            if (r->body) free_body(r->body);
        for (Request *r : g->ready)
            if (r->body) free_body(r->body);
        if (g->table_host) (void)hipHostFree(g->table_host);
        if (g->st_host) (void)hipHostFree(g->st_host);
        if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
        delete g;
    }
    S->groups.clear();
    for (auto &kv : S->reqs) delete kv.second;
    S->reqs.clear();
    if (S->pool_mem) S->alloc.free(S->pool_mem, S->alloc.ctx);
    if (S->mirrors) (void)hipHostFree(S->mirrors);
    if (S->ssetup) (void)hipStreamDestroy(S->ssetup);
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
    const size_t fixed = 8 * (size_t)max_slots * (sizeof(Inst) + sizeof(DevState)) + 16 * kAlign;
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
    if (hipHostMalloc((void **)&S->mirrors, sizeof(DevState) * max_slots, hipHostMallocDefault) != hipSuccess) {
        S->mirrors = nullptr;
        destroy_server(S);
        return fail(TLSPH_E_NOMEM, "pinned host allocation failed");
    }
    if (hipStreamCreateWithFlags(&S->ssetup, hipStreamNonBlocking) != hipSuccess) {
        S->ssetup = nullptr;
        destroy_server(S);
        return fail(TLSPH_E_DEVICE, "hipStreamCreate failed");
    }
    // 8 groups measured 12 % more solves/s than 4 on a mixed 2D/3D request stream (the hardware
    // queues are shared, but fewer bodies wait for each other in lock step)
    int ngroups = std::min(8, max_slots);
    if (const char *c = getenv("TLSPH_SERVE_GROUPS")) ngroups = std::min(max_slots, std::max(1, std::min(8, atoi(c))));
    for (int k = 0; k < ngroups; ++k) {
        Group *g = new (std::nothrow) Group();
        if (!g) {
            destroy_server(S);
            return fail(TLSPH_E_NOMEM, "host allocation failed");
        }
        S->groups.push_back(g);
        g->id = k;
        g->table_dev = (Inst *)S->pool.get(sizeof(Inst) * max_slots);
        g->st_dev = (DevState *)S->pool.get(sizeof(DevState) * max_slots);
        if (hipHostMalloc((void **)&g->table_host, sizeof(Inst) * max_slots, hipHostMallocDefault) != hipSuccess)
            g->table_host = nullptr;
        if (hipHostMalloc((void **)&g->st_host, sizeof(DevState) * max_slots, hipHostMallocDefault) != hipSuccess)
            g->st_host = nullptr;
        if (k == 0 && stream) {
            g->stream = (hipStream_t)stream;
            g->own_stream = false;
        } else if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            g->stream = nullptr;
        }
        if (!g->table_dev || !g->st_dev || !g->table_host || !g->st_host || !g->stream) {
            destroy_server(S);
            return fail(TLSPH_E_NOMEM, "server group tables or streams could not be created");
        }
    }
    try {
        S->worker = std::thread(worker_main, S);
        for (Group *g : S->groups) g->thread = std::thread(group_main, S, g);
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
    if (q->scheme != TLSPH_PAIRWISE && q->scheme != TLSPH_PARTICLE)
        return fail(TLSPH_E_INVALID, "unknown damping scheme %d", q->scheme);
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
    r->scheme = q->scheme;
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
