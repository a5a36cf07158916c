// serve.cpp -- continuous-batching request server (include/bem_serve.h).
//
// Worker threads, one per slot, each with its own non-blocking HIP stream,
// take admitted requests and run the whole bem.h path for them; requests that
// arrive while others run are admitted as soon as a slot and a free range of
// the caller's device arena are available.  The arena is managed first-fit
// with coalescing; admission is oldest-first with bounded overtaking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bem_serve.h"
#include "launch.h"

namespace bemk {
void lend_flag_buffers(bem_problem* p, int* pinned, size_t ints, const hipEvent_t* ev);
void freeze_shapes(bem_problem* p, std::shared_ptr<const ShapeSnapshot> snap);
void set_last_error(const std::string& msg);
}

namespace {

constexpr int MAX_SLOTS = 16;
constexpr int MAX_REQ_RHS = 256;
// flag slots per right-hand side: the kernel-by-kernel ring or the captured
// path's GRAPH_MAX_STEPS + 1, whichever is longer
constexpr size_t FLAG_INTS =
    (size_t)(bemk::FLAG_RING > bemk::GRAPH_MAX_STEPS + 1 ? bemk::FLAG_RING : bemk::GRAPH_MAX_STEPS + 1) * MAX_REQ_RHS;

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator over [0, size) in 256-byte units; free ranges coalesce.
class Arena {
  public:
    void init(size_t size)
    {
        size_ = size & ~size_t(255);
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = high_ = 0;
    }
    bool alloc(size_t n, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += n;
            high_ = std::max(high_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
        used_ -= n;
    }
    bool fits(size_t n) const
    {
        for (const auto& f : free_)
            if (f.second >= n) return true;
        return false;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t high() const { return high_; }

  private:
    size_t size_ = 0, used_ = 0, high_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    long long id = 0;
    bem_problem* p = nullptr;
    int n = 0, nrhs = 0;
    std::vector<double> angles;
    bem_z* out = nullptr;
    size_t lda = 0;  // leading dimension of the matrix (n rounded up to 16)
    size_t geom = 0, mat = 0, work = 0, vec = 0, far = 0, footprint = 0;
    double t_submit = 0, t_admit = 0;
    int passed_over = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    int* pinned = nullptr;
    hipEvent_t ev[bemk::FLAG_RING] = {};
    std::thread th;
};

bem_status sfail(bem_status s, const std::string& m)
{
    bemk::set_last_error(m);
    return s;
}

}  // namespace

struct bem_server {
    bem_server_opts o{};
    std::vector<double> dirs;
    // product launch shapes of every request: the tuned table and environment
    // overrides as they were when the server was created
    std::shared_ptr<const bemk::ShapeSnapshot> shapes;
    char* base = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::deque<bem_server_result> done;
    std::vector<Slot> slots;
    bool stop = false;
    long long next_id = 1, submitted = 0;
    int running = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    // Sizes of a request's buffers; false with the bem.h status on failure.
    bem_status size_request(Request& r) const
    {
        size_t g = 0, m = 0, w = 0;
        if (bem_status st = bem_sizes(r.p, (bem_prec)o.prec, r.nrhs, o.solve.restart, &g, &m, &w)) return st;
        r.n = bem_order(r.p);
        // columns start on 128-byte lines (16 complex64 / 8 complex128
        // entries): an unaligned start costs the products one more cache
        // line per column segment a workgroup reads
        r.lda = ((size_t)r.n + 15) / 16 * 16;
        m = bemk::matrix_bytes_ld(o.prec, (size_t)r.n, r.lda);
        r.geom = al(g);
        r.mat = al(m);
        r.work = al(w);
        r.vec = al((size_t)r.n * r.nrhs * sizeof(bem_z));
        r.far = al((size_t)o.ndir * r.nrhs * sizeof(bem_z));
        r.footprint = r.geom + r.mat + r.work + 2 * r.vec + r.far;
        return BEM_OK;
    }

    // Oldest waiting request that fits (caller holds mu).  A request passed
    // over 2 * slots times blocks younger ones.
    Request* pick(size_t* off)
    {
        const int limit = 2 * (int)slots.size();
        for (size_t i = 0; i < queue.size(); ++i) {
            Request* r = queue[i];
            if (arena.alloc(r->footprint, off)) {
                for (size_t j = 0; j < i; ++j) queue[j]->passed_over++;
                queue.erase(queue.begin() + (long)i);
                return r;
            }
            if (r->passed_over >= limit) return nullptr;
        }
        return nullptr;
    }

    // Run the admitted requests of one slot (one, or up to o.fuse with fused
    // Krylov steps): each one's device tables, matrix and right-hand sides,
    // then one bem_solve_batch over those that got that far, then each far
    // field and its copy to the caller.  Every request lends its own part of
    // the slot's pinned flag buffer; the slot's events serve the batch.
    void run_batch(std::vector<Request*>& rs, const std::vector<size_t>& offs, Slot& sl,
                   std::vector<bem_server_result>& res)
    {
        const size_t nb = rs.size();
        std::vector<bem_status> st(nb, BEM_OK);
        std::vector<std::vector<bem_solve_info>> info(nb);
        std::vector<char*> g(nb), A(nb), W(nb), B(nb), X(nb), F(nb);
        for (size_t k = 0; k < nb; ++k) {
            Request* r = rs[k];
            g[k] = base + offs[k];
            A[k] = g[k] + r->geom;
            W[k] = A[k] + r->mat;
            B[k] = W[k] + r->work;
            X[k] = B[k] + r->vec;
            F[k] = X[k] + r->vec;
            info[k].resize((size_t)r->nrhs);
            bemk::lend_flag_buffers(r->p, sl.pinned + k * FLAG_INTS, FLAG_INTS, sl.ev);
            bemk::freeze_shapes(r->p, shapes);
            st[k] = bem_geometry(r->p, g[k], r->geom, sl.stream);
            if (!st[k]) st[k] = bem_assemble(r->p, (bem_prec)o.prec, A[k], r->lda, sl.stream);
            if (!st[k]) st[k] = bem_rhs(r->p, r->nrhs, r->angles.data(), B[k], (size_t)r->n, sl.stream);
            if (st[k]) std::snprintf(res[k].message, sizeof res[k].message, "%s", bem_last_error());
        }
        // the batch: every request whose set-up succeeded
        std::vector<size_t> in;
        std::vector<bem_problem*> ps;
        std::vector<int> nr;
        std::vector<const void*> Bp;
        std::vector<void*> Xp, Wp;
        std::vector<size_t> ld, wb;
        std::vector<bem_solve_info*> ip;
        for (size_t k = 0; k < nb; ++k) {
            if (st[k]) continue;
            in.push_back(k);
            ps.push_back(rs[k]->p);
            nr.push_back(rs[k]->nrhs);
            Bp.push_back(B[k]);
            Xp.push_back(X[k]);
            Wp.push_back(W[k]);
            ld.push_back((size_t)rs[k]->n);
            wb.push_back(rs[k]->work);
            ip.push_back(info[k].data());
        }
        if (!in.empty()) {
            const bem_status sst = bem_solve_batch((int)in.size(), ps.data(), nr.data(), Bp.data(), ld.data(), &o.solve,
                                                   Xp.data(), ld.data(), Wp.data(), wb.data(), ip.data(), sl.stream);
            const std::string msg = sst ? bem_last_error() : "";
            for (size_t k : in) {
                bool conv = true, finite = true;
                for (const auto& i : info[k]) {
                    conv = conv && i.converged;
                    finite = finite && std::isfinite(i.rel_residual);
                }
                // BEM_E_NOCONV / BEM_E_NONFINITE belong to the requests whose
                // columns met them; another error to the whole batch
                if (sst == BEM_E_NONFINITE || sst == BEM_E_NOCONV)
                    st[k] = !finite ? BEM_E_NONFINITE : (!conv ? BEM_E_NOCONV : BEM_OK);
                else
                    st[k] = sst;
                if (st[k] && st[k] != BEM_E_NOCONV)
                    std::snprintf(res[k].message, sizeof res[k].message, "%s", msg.c_str());
            }
        }
        for (size_t k = 0; k < nb; ++k) {
            Request* r = rs[k];
            bem_status s = st[k];
            const bool noconv = s == BEM_E_NOCONV;
            if (!s || noconv)
                s = bem_farfield(r->p, r->nrhs, X[k], (size_t)r->n, o.ndir, dirs.data(), F[k], (size_t)o.ndir, nullptr,
                                 0, sl.stream);
            if (!s) {
                hipError_t e = hipMemcpyAsync(r->out, F[k], (size_t)o.ndir * r->nrhs * sizeof(bem_z),
                                              hipMemcpyDeviceToHost, sl.stream);
                if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
                if (e != hipSuccess) {
                    s = BEM_E_DEVICE;
                    std::snprintf(res[k].message, sizeof res[k].message, "far-field copy: %s", hipGetErrorString(e));
                }
            } else {
                if (!res[k].message[0]) std::snprintf(res[k].message, sizeof res[k].message, "%s", bem_last_error());
                (void)hipStreamSynchronize(sl.stream);
            }
            if (!s && noconv) {
                s = BEM_E_NOCONV;
                std::snprintf(res[k].message, sizeof res[k].message, "%s", "GMRES stopped at max_iter");
            }
            res[k].status = s;
            for (const auto& i : info[k]) {
                res[k].iters_max = std::max(res[k].iters_max, i.iters);
                res[k].refine_max = std::max(res[k].refine_max, i.restarts);
                res[k].rel_residual_max = std::max(res[k].rel_residual_max, i.rel_residual);
            }
        }
    }

    void worker(int k)
    {
        Slot& sl = slots[(size_t)k];
        (void)hipSetDevice(o.device);
        const size_t fuse = (size_t)std::max(1, o.fuse);
        for (;;) {
            std::vector<Request*> rs;
            std::vector<size_t> offs;
            {
                std::unique_lock<std::mutex> lk(mu);
                size_t off = 0;
                Request* r = nullptr;
                for (;;) {
                    if (!queue.empty() && (r = pick(&off)) != nullptr) break;
                    if (stop && queue.empty()) return;
                    cv_work.wait(lk);
                }
                rs.push_back(r);
                offs.push_back(off);
                // more waiting requests that fit join the slot's batch now
                while (rs.size() < fuse && !queue.empty() && (r = pick(&off)) != nullptr) {
                    rs.push_back(r);
                    offs.push_back(off);
                }
                running += (int)rs.size();
                const double t = now();
                for (Request* q : rs) q->t_admit = t;
            }
            std::vector<bem_server_result> res(rs.size());
            for (size_t q = 0; q < rs.size(); ++q) {
                res[q].id = rs[q]->id;
                res[q].n = rs[q]->n;
                res[q].nrhs = rs[q]->nrhs;
                res[q].footprint = rs[q]->footprint;
                res[q].t_submit = rs[q]->t_submit;
                res[q].t_admit = rs[q]->t_admit;
            }
            run_batch(rs, offs, sl, res);
            const double t = now();
            for (size_t q = 0; q < rs.size(); ++q) {
                res[q].t_done = t;
                bem_destroy(rs[q]->p);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                for (size_t q = 0; q < rs.size(); ++q) {
                    arena.release(offs[q], rs[q]->footprint);
                    done.push_back(res[q]);
                }
                running -= (int)rs.size();
            }
            for (Request* q : rs) delete q;
            cv_work.notify_all();
            cv_done.notify_all();
        }
    }
};

extern "C" {

bem_status bem_server_create(const bem_server_opts* opts, bem_server** out)
{
    if (!opts || !out) return sfail(BEM_E_ARG, "null argument");
    *out = nullptr;
    const bem_server_opts& o = *opts;
    if (o.slots < 1 || o.slots > MAX_SLOTS) return sfail(BEM_E_ARG, "slots outside 1..16");
    if (!o.arena_dev || (reinterpret_cast<uintptr_t>(o.arena_dev) & 255) || o.arena_bytes < 256)
        return sfail(BEM_E_ARG, "arena null, unaligned or empty");
    if (o.ndir < 1 || o.ndir > 4096 || !o.dirs) return sfail(BEM_E_ARG, "ndir outside 1..4096 or no directions");
    if (o.prec != BEM_F64 && o.prec != BEM_F32 && o.prec != BEM_MIXED) return sfail(BEM_E_ARG, "unknown precision");
    if (o.solve.restart < 1 || o.solve.max_iter < 1 || !(o.solve.tol > 0.0))
        return sfail(BEM_E_ARG, "bad solve options");
    if (o.fuse < 0 || o.fuse > bemk::MAX_FUSED) return sfail(BEM_E_ARG, "fuse outside 0..8");
    auto* s = new bem_server();
    s->o = o;
    s->dirs.assign(o.dirs, o.dirs + o.ndir);
    s->o.dirs = nullptr;
    s->shapes = bemk::snapshot_shapes();
    s->base = static_cast<char*>(o.arena_dev);
    s->arena.init(o.arena_bytes);
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipSetDevice(o.device);
    s->slots.resize((size_t)o.slots);
    for (Slot& sl : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&sl.pinned),
                              (size_t)std::max(1, o.fuse) * FLAG_INTS * sizeof(int),
                              hipHostMallocMapped | hipHostMallocCoherent);
        for (auto& ev : sl.ev)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        const std::string m = std::string("slot set-up: ") + hipGetErrorString(e);
        s->stop = true;
        bem_server_destroy(s);
        return sfail(BEM_E_DEVICE, m);
    }
    try {
        for (int k = 0; k < o.slots; ++k) s->slots[(size_t)k].th = std::thread(&bem_server::worker, s, k);
    } catch (...) {
        bem_server_destroy(s);
        return sfail(BEM_E_DEVICE, "could not start the slot threads");
    }
    *out = s;
    return BEM_OK;
}

bem_status bem_server_footprint(const bem_server* s, const bem_desc* desc, int nrhs, size_t* bytes)
{
    if (!s || !desc || !bytes) return sfail(BEM_E_ARG, "null argument");
    if (nrhs < 1 || nrhs > MAX_REQ_RHS) return sfail(BEM_E_ARG, "nrhs outside 1..256");
    Request r;
    r.nrhs = nrhs;
    if (bem_status st = bem_create(desc, &r.p)) return sfail(st, bem_last_error());
    const bem_status st = s->size_request(r);
    bem_destroy(r.p);
    if (st) return sfail(st, bem_last_error());
    *bytes = r.footprint;
    return BEM_OK;
}

bem_status bem_server_submit(bem_server* s, const bem_desc* desc, int nrhs, const double* angles,
                             bem_z* farfield_host, long long* id)
{
    if (!s || !desc || !angles || !farfield_host || !id) return sfail(BEM_E_ARG, "null argument");
    if (nrhs < 1 || nrhs > MAX_REQ_RHS) return sfail(BEM_E_ARG, "nrhs outside 1..256");
    auto* r = new Request();
    r->nrhs = nrhs;
    r->angles.assign(angles, angles + nrhs);
    r->out = farfield_host;
    if (bem_status st = bem_create(desc, &r->p)) {
        delete r;
        return sfail(st, bem_last_error());
    }
    if (bem_status st = s->size_request(*r)) {
        bem_destroy(r->p);
        delete r;
        return sfail(st, bem_last_error());
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->footprint > s->arena.size()) {
            bem_destroy(r->p);
            const size_t need = r->footprint;
            delete r;
            return sfail(BEM_E_NOMEM, "request needs " + std::to_string(need) + " arena bytes, the arena has " +
                                          std::to_string(s->arena.size()));
        }
        if (s->stop) {
            bem_destroy(r->p);
            delete r;
            return sfail(BEM_E_STATE, "server is shutting down");
        }
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->queue.push_back(r);
        s->submitted++;
        *id = r->id;
    }
    s->cv_work.notify_one();
    return BEM_OK;
}

bem_status bem_server_poll(bem_server* s, bem_server_result* out, int max, int* count, int wait_ms)
{
    if (!s || !count || (max > 0 && !out)) return sfail(BEM_E_ARG, "null argument");
    *count = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->done.empty() || (s->queue.empty() && s->running == 0); };
    if (wait_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    while (*count < max && !s->done.empty()) {
        out[(*count)++] = s->done.front();
        s->done.pop_front();
    }
    return BEM_OK;
}

bem_status bem_server_stat(bem_server* s, bem_server_stats* out)
{
    if (!s || !out) return sfail(BEM_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->waiting = (long long)s->queue.size();
    out->running = s->running;
    out->unpolled = (long long)s->done.size();
    out->arena_in_use = s->arena.used();
    out->arena_high_water = s->arena.high();
    return BEM_OK;
}

bem_status bem_server_destroy(bem_server* s)
{
    if (!s) return BEM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Slot& sl : s->slots)
        if (sl.th.joinable()) sl.th.join();
    for (Slot& sl : s->slots) {
        for (auto& ev : sl.ev)
            if (ev) (void)hipEventDestroy(ev);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (Request* r : s->queue) {
        bem_destroy(r->p);
        delete r;
    }
    delete s;
    return BEM_OK;
}

}  // extern "C"
