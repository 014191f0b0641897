// Serving runtime (rsilu_serve.h): host setup threads, first-come admission by
// device footprint into one preallocated arena, one stream per solve slot; a
// slot solves the requests it admitted together in batched persistent launches
// (rsilu_batch.h) or one by one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "rsilu.h"
#include "rsilu_batch.h"
#include "rsilu_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

constexpr size_t kAlign = 256;
size_t round_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) of the device arena (offsets only).
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    // offset of a block of `bytes`, or SIZE_MAX when no hole is large enough
    size_t take(size_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void give(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
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
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length, non-adjacent holes
};

struct Job {
    int64_t id = 0;
    rsilu_request_t req{};
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val, b;
    rsilu_handle_t h = nullptr;
    size_t op_bytes = 0, bytes = 0, off = 0;
    Clock::time_point t_submit, t_setup_done, t_admit;
    rsilu_result_t res{};
};

}  // namespace

struct rsilu_server {
    rsilu_server_opts_t opts{};
    void *arena_base = nullptr;
    Arena *arena = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<rsilu_batch_t> batches;  // one per slot when batch_max >= 1
    rsilu_tuner_t tuner = nullptr;       // when tune_slack > 0

    std::mutex mu;
    std::condition_variable cv_setup, cv_ready, cv_done;
    std::deque<Job *> setup_q, ready_q;
    std::deque<rsilu_result_t> results;
    int64_t next_id = 0, completed = 0;
    int64_t in_setup = 0;  // requests taken by a setup thread and not yet ready or finished
    bool stopping = false;
    std::vector<std::thread> threads;

    // streams, batch objects, tuner, arena
    void release_device()
    {
        if (tuner) rsilu_tuner_destroy(tuner);
        tuner = nullptr;
        for (rsilu_batch_t b : batches) rsilu_batch_destroy(b);
        batches.clear();
        for (hipStream_t t : streams) (void)hipStreamDestroy(t);
        streams.clear();
        if (arena_base) (void)hipFree(arena_base);
        arena_base = nullptr;
        delete arena;
        arena = nullptr;
    }

    void finish(Job *j, int32_t status)
    {
        const Clock::time_point now = Clock::now();
        j->res.id = j->id;
        j->res.user = j->req.user;
        j->res.status = status;
        j->res.total_ms = ms_between(j->t_submit, now);
        if (j->h) rsilu_destroy(j->h);
        {
            std::lock_guard<std::mutex> lk(mu);
            results.push_back(j->res);
            ++completed;
        }
        cv_done.notify_all();
        delete j;
    }

    void setup_worker()
    {
        for (;;) {
            Job *j = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_setup.wait(lk, [&] { return stopping || !setup_q.empty(); });
                if (setup_q.empty()) return;
                j = setup_q.front();
                setup_q.pop_front();
                ++in_setup;
            }
            const Clock::time_point t0 = Clock::now();
            rsilu_status_t st = rsilu_factor(j->req.m, j->req.n, j->rowptr.data(), j->col.data(), j->val.data(),
                                             &j->req.params, &j->h);
            j->t_setup_done = Clock::now();
            j->res.setup_ms = ms_between(t0, j->t_setup_done);
            if (st != RSILU_OK) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    --in_setup;
                }
                cv_ready.notify_all();
                finish(j, st);
                continue;
            }
            j->op_bytes = round_up(rsilu_device_bytes(j->h));
            j->bytes = j->op_bytes + round_up(sizeof(double) * (size_t)j->req.m) +
                       round_up(sizeof(double) * (size_t)j->req.n);
            j->res.device_bytes = j->bytes;
            if (j->bytes > opts.hbm_bytes) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    --in_setup;
                }
                cv_ready.notify_all();
                finish(j, RSILU_ENOMEM);
                continue;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                --in_setup;
                ready_q.push_back(j);
            }
            cv_ready.notify_all();
        }
    }

    // Whether the batched kernel accepts a request.
    static bool batchable(const Job &j) { return rsilu_batch_accepts(j.h) == 1; }

    void slot_worker(int slot)
    {
        (void)hipSetDevice(opts.device);
        hipStream_t s = streams[(size_t)slot];
        rsilu_batch_t bt = batches.empty() ? nullptr : batches[(size_t)slot];
        const size_t cap = opts.batch_max > 0 ? (size_t)opts.batch_max : 1;
        for (;;) {
            std::vector<Job *> jobs;
            {
                std::unique_lock<std::mutex> lk(mu);
                // first come, first served: only the head of the ready queue is admitted,
                // then the requests behind it while they fit (up to batch_max)
                cv_ready.wait(lk, [&] {
                    if (ready_q.empty()) return stopping;
                    Job *head = ready_q.front();
                    head->off = arena->take(head->bytes);
                    return head->off != SIZE_MAX;
                });
                if (ready_q.empty()) return;
                jobs.push_back(ready_q.front());
                ready_q.pop_front();
                // batching window: wait a little for requests still in setup
                if (cap >= 2 && opts.batch_wait_ms > 0.0) {
                    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                                          std::chrono::duration<double, std::milli>(opts.batch_wait_ms));
                    cv_ready.wait_until(lk, until, [&] {
                        return stopping || ready_q.size() + 1 >= cap || (in_setup == 0 && setup_q.empty());
                    });
                }
                while (jobs.size() < cap && !ready_q.empty()) {
                    Job *nx = ready_q.front();
                    const size_t off = arena->take(nx->bytes);
                    if (off == SIZE_MAX) break;
                    nx->off = off;
                    jobs.push_back(nx);
                    ready_q.pop_front();
                }
            }
            const size_t k = jobs.size();
            std::vector<rsilu_status_t> st(k, RSILU_OK);
            std::vector<double *> bdev(k), xdev(k);
            for (size_t i = 0; i < k; ++i) {
                Job *j = jobs[i];
                j->t_admit = Clock::now();
                j->res.wait_ms = ms_between(j->t_setup_done, j->t_admit);
                char *base = static_cast<char *>(arena_base) + j->off;
                bdev[i] = reinterpret_cast<double *>(base + j->op_bytes);
                xdev[i] = reinterpret_cast<double *>(base + j->op_bytes + round_up(sizeof(double) * (size_t)j->req.m));
                st[i] = rsilu_upload(j->h, base, j->op_bytes, s);
                if (st[i] == RSILU_OK && hipMemcpyAsync(bdev[i], j->b.data(), sizeof(double) * (size_t)j->req.m,
                                                        hipMemcpyHostToDevice, s) != hipSuccess)
                    st[i] = RSILU_EHIP;
            }
            // path and tile of every request; batched ones grouped by tile
            // Paths: with the autotuner and at least two requests the batched kernel
            // accepts, rsilu_batch_solve_auto splits the admission between one batched
            // launch and the plain path beside it; without the tuner every accepted
            // request shares one launch with the default tile; a lone request, and
            // every request the batched kernel does not accept, takes rsilu_solve.
            std::vector<size_t> ok_idx, acc_idx;
            for (size_t i = 0; i < k; ++i) {
                if (st[i] != RSILU_OK) continue;
                ok_idx.push_back(i);
                jobs[i]->res.path = 1;
                jobs[i]->res.launch_size = 1;
                if (bt && batchable(*jobs[i])) acc_idx.push_back(i);
            }
            std::vector<size_t> plain;
            auto gather = [&](const std::vector<size_t> &ids, std::vector<rsilu_handle_t> &hs,
                              std::vector<const double *> &bb, std::vector<double> &tt, std::vector<double *> &xx) {
                for (size_t i : ids) {
                    hs.push_back(jobs[i]->h);
                    bb.push_back(bdev[i]);
                    tt.push_back(jobs[i]->req.tol);
                    xx.push_back(xdev[i]);
                }
            };
            if (tuner && acc_idx.size() >= 2) {
                std::vector<rsilu_handle_t> hs;
                std::vector<const double *> bb;
                std::vector<double> tt;
                std::vector<double *> xx;
                gather(ok_idx, hs, bb, tt, xx);
                std::vector<rsilu_batch_result_t> rr(ok_idx.size());
                for (rsilu_batch_result_t &r : rr) r.status = RSILU_EINTERNAL;  // overwritten by every problem that ran
                std::vector<int32_t> path(ok_idx.size(), 1);
                rsilu_tile_t tile{};
                const rsilu_status_t rc = rsilu_batch_solve_auto(bt, tuner, (int32_t)ok_idx.size(), hs.data(), bb.data(),
                                                                 tt.data(), xx.data(), rr.data(), path.data(), &tile, s);
                int32_t nb = 0;
                for (int32_t p : path) nb += p == 0;
                for (size_t q = 0; q < ok_idx.size(); ++q) {
                    Job *j = jobs[ok_idx[q]];
                    if (rr[q].status == RSILU_EINTERNAL && rc < 0) {
                        st[ok_idx[q]] = rc;
                        continue;
                    }
                    st[ok_idx[q]] = (rsilu_status_t)rr[q].status;
                    j->res.iters = rr[q].iters;
                    j->res.atr_norm = rr[q].atr_norm;
                    j->res.atr_rel = rr[q].atr_rel;
                    j->res.path = path[q];
                    if (path[q] == 0) {
                        j->res.launch_size = nb;
                        j->res.tile = tile;
                    }
                }
            } else if (!tuner && !acc_idx.empty()) {
                std::vector<rsilu_handle_t> hs;
                std::vector<const double *> bb;
                std::vector<double> tt;
                std::vector<double *> xx;
                gather(acc_idx, hs, bb, tt, xx);
                std::vector<rsilu_batch_result_t> rr(acc_idx.size());
                const rsilu_tile_t tile = {1024, 4, 4, 0};
                const rsilu_status_t rc =
                    rsilu_batch_solve(bt, (int32_t)acc_idx.size(), hs.data(), bb.data(), tt.data(), xx.data(), &tile,
                                      rr.data(), s);
                for (size_t q = 0; q < acc_idx.size(); ++q) {
                    Job *j = jobs[acc_idx[q]];
                    j->res.path = 0;
                    j->res.launch_size = (int32_t)acc_idx.size();
                    j->res.tile = tile;
                    if (rc != RSILU_OK) {
                        st[acc_idx[q]] = rc;
                        continue;
                    }
                    st[acc_idx[q]] = (rsilu_status_t)rr[q].status;
                    j->res.iters = rr[q].iters;
                    j->res.atr_norm = rr[q].atr_norm;
                    j->res.atr_rel = rr[q].atr_rel;
                }
                for (size_t i : ok_idx)
                    if (jobs[i]->res.path == 1) plain.push_back(i);
            } else {
                plain = ok_idx;
            }
            for (size_t i : plain) {
                Job *j = jobs[i];
                st[i] = rsilu_solve(j->h, bdev[i], j->req.tol, xdev[i], &j->res.iters, &j->res.atr_norm,
                                    &j->res.atr_rel, s);
            }
            for (size_t i = 0; i < k; ++i)
                if (st[i] >= 0 && hipMemcpyAsync(jobs[i]->req.x, xdev[i], sizeof(double) * (size_t)jobs[i]->req.n,
                                                 hipMemcpyDeviceToHost, s) != hipSuccess)
                    st[i] = RSILU_EHIP;
            const bool sync_ok = hipStreamSynchronize(s) == hipSuccess;
            const Clock::time_point t_end = Clock::now();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (Job *j : jobs) arena->give(j->off, j->bytes);
            }
            cv_ready.notify_all();
            for (size_t i = 0; i < k; ++i) {
                jobs[i]->res.solve_ms = ms_between(jobs[i]->t_admit, t_end);
                finish(jobs[i], (!sync_ok && st[i] >= 0) ? RSILU_EHIP : st[i]);
            }
        }
    }
};

extern "C" {

rsilu_status_t rsilu_server_create(const rsilu_server_opts_t *opts, rsilu_server_t *out)
{
    if (!opts || !out || opts->slots < 1 || opts->setup_threads < 1 || opts->hbm_bytes < kAlign ||
        opts->batch_max < 0 || opts->batch_max > 65535 || !std::isfinite(opts->tune_slack) || opts->tune_slack < 0.0 ||
        !std::isfinite(opts->batch_wait_ms) || opts->batch_wait_ms < 0.0)
        return RSILU_EINVAL;
    *out = nullptr;
    rsilu_server *s = nullptr;
    try {
        s = new rsilu_server();
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
    s->opts = *opts;
    s->opts.hbm_bytes &= ~(kAlign - 1);
    if (hipSetDevice(opts->device) != hipSuccess) {
        delete s;
        return RSILU_EINVAL;
    }
    if (hipMalloc(&s->arena_base, s->opts.hbm_bytes) != hipSuccess) {
        delete s;
        return RSILU_ENOMEM;
    }
    s->arena = new Arena(s->opts.hbm_bytes);
    for (int i = 0; i < opts->slots; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            s->release_device();
            delete s;
            return RSILU_EHIP;
        }
        s->streams.push_back(st);
    }
    rsilu_status_t rc = RSILU_OK;
    for (int i = 0; i < opts->slots && opts->batch_max > 0 && rc == RSILU_OK; ++i) {
        rsilu_batch_t bt = nullptr;
        rc = rsilu_batch_create(opts->batch_max, &bt);
        if (rc == RSILU_OK) s->batches.push_back(bt);
    }
    if (rc == RSILU_OK && opts->batch_max > 0 && opts->tune_slack > 0.0) rc = rsilu_tuner_create(opts->tune_slack, 4, &s->tuner);
    if (rc != RSILU_OK) {
        s->release_device();
        delete s;
        return rc;
    }
    for (int i = 0; i < opts->setup_threads; ++i) s->threads.emplace_back([s] { s->setup_worker(); });
    for (int i = 0; i < opts->slots; ++i) s->threads.emplace_back([s, i] { s->slot_worker(i); });
    *out = s;
    return RSILU_OK;
}

rsilu_status_t rsilu_server_submit(rsilu_server_t s, const rsilu_request_t *req, int64_t *id)
{
    if (!s || !req || !req->rowptr || !req->b || !req->x || req->m < req->n || req->n < 1) return RSILU_EINVAL;
    const int64_t nnz = req->rowptr[req->m];
    if (nnz < 0 || (nnz > 0 && (!req->colind || !req->val))) return RSILU_EINVAL;
    Job *j = nullptr;
    try {
        j = new Job();
        j->req = *req;
        j->rowptr.assign(req->rowptr, req->rowptr + req->m + 1);
        j->col.assign(req->colind, req->colind + nnz);
        j->val.assign(req->val, req->val + nnz);
        j->b.assign(req->b, req->b + req->m);
    } catch (const std::bad_alloc &) {
        delete j;
        return RSILU_ENOMEM;
    }
    j->t_submit = Clock::now();
    j->res.path = -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete j;
            return RSILU_ESTATE;
        }
        j->id = s->next_id++;
        s->setup_q.push_back(j);
    }
    if (id) *id = j->id;
    s->cv_setup.notify_one();
    return RSILU_OK;
}

int32_t rsilu_server_poll(rsilu_server_t s, rsilu_result_t *out, int32_t max, int32_t wait_ms)
{
    if (!s || !out || max < 1) return 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->results.empty(); });
    int32_t k = 0;
    while (k < max && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    return k;
}

rsilu_status_t rsilu_server_drain(rsilu_server_t s)
{
    if (!s) return RSILU_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->next_id; });
    return RSILU_OK;
}

void rsilu_server_destroy(rsilu_server_t s)
{
    if (!s) return;
    (void)rsilu_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_setup.notify_all();
    s->cv_ready.notify_all();
    for (std::thread &t : s->threads) t.join();
    s->release_device();
    delete s;
}

}  // extern "C"
