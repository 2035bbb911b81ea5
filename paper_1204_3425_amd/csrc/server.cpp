// Continuous-batching solve server (C ABI in include/hubbard.h).
//
// Requests flow through four stages, each owned by one thread:
//   submit -> admission (first fit in arrival order against the HBM budget and
//   the slot limit) -> build (basis and tables on the host, then upload) ->
//   execution -> completion queue.
// Two executors share the device: the batch executor keeps small sectors in
// BatchRunners (two per precision, on two streams) and lets newly built
// requests join between Lanczos steps (so arrivals start while earlier
// requests are still iterating); the solo
// executor runs large sectors one at a time on a second stream with the
// two-pass H.v.  A request's reservation covers its tables and work vectors
// and is released when it completes.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"

namespace hub {
namespace {

struct Job {
    uint64_t id = 0;
    hubbard_request req{};
    std::vector<int32_t> edges;
    size_t reserve = 0;
    hubbard *h = nullptr;
    bool batch = false;
    hubbard_completion done{};
};

// Upper bound of the device bytes a request needs: the two work vectors on
// padded rows, partial sums, the batched engine's coefficient history, and the
// tables with at most n_edges entries per row: up side (row-major entries,
// blocked entries, the entry lines: up to two 128-byte lines per row when a
// row has at most 64 hops (one when 32 slots hold the row and its padding),
// none beyond; counts, states)
// and down side (column-major entries, 64- and 32-bit offset groups, 16-bit
// groups, counts, states, and the FP64 row pass's 16-bit indices split by
// sign: at most w/8 groups of eight + hops and w/4 groups of four - hops).
size_t footprint(const hubbard_request &r)
{
    const uint64_t du = binomial(r.sites, r.n_up), dd = binomial(r.sites, r.n_dn);
    const size_t es = r.precision == HUBBARD_FP64 ? 8 : 4;
    const size_t ld = (size_t)((dd + 63) / 64 * 64);
    const size_t vecs = 2 * es * (size_t)du * ld + 64 * 1024 + 16 * (size_t)std::max(1, r.max_iter);
    const size_t w = (size_t)std::max(1, r.n_edges);
    const size_t lines = w <= 64 ? 256 : 0;  // one or two 128-byte lines
    const size_t up = (size_t)du * (8 * w + 14 + lines);
    const size_t g8 = (w + 7) / 8, g4 = (w + 3) / 4;  // groups of eight or four entries per column
    const size_t dn = (size_t)dd * (14 * w + 56 + 16 * g8 + 16 * g8 + 8 * g4 + 1);
    return vecs + up + dn;
}

}  // namespace
}  // namespace hub

struct hubbard_server {
    size_t budget = 0;
    int max_slots = 1;
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<hub::Job>> pending;   // submitted, not admitted
    std::deque<std::unique_ptr<hub::Job>> to_build;  // admitted, tables not built
    std::deque<std::unique_ptr<hub::Job>> ready_batch, ready_solo;
    std::deque<hubbard_completion> completions;
    size_t reserved = 0, peak_reserved = 0;
    int slots_used = 0;
    uint64_t next_id = 1, admitted = 0, completed = 0, rejected = 0;
    int max_active_batch = 0;
    uint64_t solo_runs = 0;
    bool stop = false;
    std::string fatal;

    hipStream_t s_batch[2] = {nullptr, nullptr}, s_solo = nullptr;
    std::thread t_build, t_batch, t_solo;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace hub {
namespace {

void admit_locked(hubbard_server *S);

void complete(hubbard_server *S, std::unique_ptr<Job> job, int status)
{
    job->done.status = status;
    job->done.t_done = S->now();
    if (job->h)
        hubbard_free(job->h);
    std::lock_guard<std::mutex> lk(S->mu);
    if (job->reserve) {
        S->reserved -= job->reserve;
        S->slots_used--;
    }
    S->completions.push_back(job->done);
    S->completed++;
    admit_locked(S);  // the released memory and slot may let queued requests start
    S->cv.notify_all();
}

// Moves requests from pending to to_build by the admission rule (caller holds mu).
void admit_locked(hubbard_server *S)
{
    std::vector<uint64_t> fp;
    for (auto &j : S->pending)
        fp.push_back(j->reserve);
    std::vector<int32_t> take(fp.size(), 0);
    hubbard_admission_plan(fp.data(), (int)fp.size(), S->budget, S->reserved, S->max_slots - S->slots_used,
                           take.data());
    std::deque<std::unique_ptr<Job>> keep;
    for (size_t k = 0; k < S->pending.size(); k++) {
        auto &j = S->pending[k];
        if (take[k]) {
            S->reserved += j->reserve;
            S->slots_used++;
            S->peak_reserved = std::max(S->peak_reserved, S->reserved);
            S->admitted++;
            j->done.t_admit = S->now();
            S->to_build.push_back(std::move(j));
        } else {
            keep.push_back(std::move(j));
        }
    }
    S->pending.swap(keep);
}

void build_loop(hubbard_server *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::unique_ptr<Job> job;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->to_build.empty(); });
            if (S->stop)
                return;
            job = std::move(S->to_build.front());
            S->to_build.pop_front();
        }
        const hubbard_request &r = job->req;
        hubbard_h h = nullptr;
        int rc = hubbard_build(r.sites, job->edges.data(), r.n_edges, r.n_up, r.n_dn, r.t, r.U, &h);
        if (rc != HUBBARD_OK) {
            complete(S, std::move(job), rc);
            continue;
        }
        job->h = h;
        job->batch = batchable(h, r.precision) && h->dim <= (int64_t)16 * 1024 * 1024;
        std::lock_guard<std::mutex> lk(S->mu);
        (job->batch ? S->ready_batch : S->ready_solo).push_back(std::move(job));
        S->cv.notify_all();
    }
}

hubbard_opts opts_of(const hubbard_request &r)
{
    hubbard_opts o;
    std::memset(&o, 0, sizeof(o));
    o.tol = r.tol;
    o.max_iter = r.max_iter;
    o.precision = r.precision;
    o.seed = r.seed;
    return o;
}

void batch_loop(hubbard_server *S)
{
    (void)hipSetDevice(S->device);
    // two runners per precision (index 2 * precision slot + k) on the two batch
    // streams, so the step launches of one fill the gaps between the other's; a
    // joining request goes to the runner of its precision with fewer solves
    std::unique_ptr<BatchRunner> runners[4];
    std::vector<std::unique_ptr<Job>> running;
    try {
        for (;;) {
            std::vector<std::unique_ptr<Job>> joining;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                bool idle = true;
                for (auto &rn : runners)
                    idle = idle && (!rn || rn->active() == 0);
                if (idle)
                    S->cv.wait(lk, [&] { return S->stop || !S->ready_batch.empty(); });
                if (S->stop)
                    break;
                while (!S->ready_batch.empty()) {
                    joining.push_back(std::move(S->ready_batch.front()));
                    S->ready_batch.pop_front();
                }
            }
            for (auto &job : joining) {
                const int p0 = job->req.precision == HUBBARD_FP64 ? 0 : 2;
                auto load = [&](int i) { return runners[i] ? runners[i]->active() : 0; };
                const int k = load(p0 + 1) < load(p0) ? 1 : 0;
                const int p = p0 + k;
                if (!runners[p])
                    runners[p] = BatchRunner::make(job->req.precision, S->s_batch[k]);
                job->h->stream = S->s_batch[k];
                try {
                    runners[p]->add(job->h, opts_of(job->req), &job->done.result);
                } catch (const Error &e) {
                    // this request could not start (for example its vectors did not
                    // fit after all); the others keep running
                    complete(S, std::move(job), e.code);
                    continue;
                }
                job->done.t_start = S->now();
                running.push_back(std::move(job));
            }
            int active = 0;
            for (auto &rn : runners)
                if (rn)
                    active += rn->active();
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->max_active_batch = std::max(S->max_active_batch, active);
            }
            for (auto &rn : runners) {
                if (!rn || rn->active() == 0)
                    continue;
                std::vector<hubbard_result *> fin = rn->step();
                for (hubbard_result *res : fin) {
                    for (auto &job : running) {
                        if (job && &job->done.result == res) {
                            const int st = res->status;
                            complete(S, std::move(job), st);
                            break;
                        }
                    }
                }
                running.erase(std::remove(running.begin(), running.end(), nullptr), running.end());
            }
        }
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = e.msg;
        S->stop = true;
        S->cv.notify_all();
    }
    for (auto &rn : runners)
        rn.reset();
    for (auto &job : running)
        if (job && job->h)
            hubbard_free(job->h);
}

void solo_loop(hubbard_server *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::unique_ptr<Job> job;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->ready_solo.empty(); });
            if (S->stop)
                return;
            job = std::move(S->ready_solo.front());
            S->ready_solo.pop_front();
        }
        job->h->stream = S->s_solo;
        job->done.t_start = S->now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->solo_runs++;
        }
        int rc;
        try {
            rc = lanczos_impl(job->h, opts_of(job->req), &job->done.result);
        } catch (const Error &e) {
            rc = e.code;
        }
        complete(S, std::move(job), rc);
    }
}

template <typename F>
int guard(F &&f)
{
    try {
        return f();
    } catch (const Error &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return HUBBARD_ENOMEM;
    } catch (...) {
        return HUBBARD_EDEVICE;
    }
}

}  // namespace
}  // namespace hub

using namespace hub;

extern "C" {

int hubbard_admission_plan(const uint64_t *footprints, int n, uint64_t budget, uint64_t used, int free_slots,
                           int32_t *admit)
{
    if (n < 0 || (n > 0 && (!footprints || !admit)))
        return HUBBARD_EINVAL;
    int count = 0;
    uint64_t room = budget > used ? budget - used : 0;
    for (int k = 0; k < n; k++) {
        admit[k] = 0;
        if (count < free_slots && footprints[k] <= room) {
            admit[k] = 1;
            room -= footprints[k];
            count++;
        }
    }
    return count;
}

int hubbard_server_create(size_t hbm_budget, int max_slots, hubbard_server_h *out)
{
    return guard([&]() -> int {
        if (!out || hbm_budget == 0 || max_slots < 1)
            return HUBBARD_EINVAL;
        *out = nullptr;
        std::unique_ptr<hubbard_server> S(new hubbard_server());
        S->budget = hbm_budget;
        S->max_slots = max_slots;
        S->t0 = std::chrono::steady_clock::now();
        HUB_HIP(hipGetDevice(&S->device));
        for (auto &sb : S->s_batch)
            HUB_HIP(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking));
        HUB_HIP(hipStreamCreateWithFlags(&S->s_solo, hipStreamNonBlocking));
        hubbard_server *raw = S.get();
        S->t_build = std::thread(build_loop, raw);
        S->t_batch = std::thread(batch_loop, raw);
        S->t_solo = std::thread(solo_loop, raw);
        *out = S.release();
        return HUBBARD_OK;
    });
}

int hubbard_server_submit(hubbard_server_h S, const hubbard_request *req, uint64_t *id)
{
    return guard([&]() -> int {
        if (!S || !req || !id)
            return HUBBARD_EINVAL;
        if (req->n_edges < 0 || (req->n_edges > 0 && !req->edges) || req->sites < 1 || req->sites > 32 ||
            req->max_iter < 1 || std::isnan(req->tol) ||
            (req->precision != HUBBARD_FP64 && req->precision != HUBBARD_MIXED))
            return HUBBARD_EINVAL;
        auto job = std::make_unique<Job>();
        job->req = *req;
        job->edges.assign(req->edges, req->edges + 2 * (size_t)req->n_edges);
        job->req.edges = nullptr;
        job->reserve = footprint(*req);
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop)
            return HUBBARD_EDEVICE;
        job->id = S->next_id++;
        job->done.id = job->id;
        job->done.tag = req->tag;
        job->done.t_submit = S->now();
        *id = job->id;
        if (job->reserve > S->budget) {
            // can never fit: reported at once, the queue keeps moving
            job->done.status = HUBBARD_ENOMEM;
            job->done.t_admit = job->done.t_start = job->done.t_done = job->done.t_submit;
            S->completions.push_back(job->done);
            S->rejected++;
            S->completed++;
            S->cv.notify_all();
            return HUBBARD_OK;
        }
        S->pending.push_back(std::move(job));
        admit_locked(S);
        S->cv.notify_all();
        return HUBBARD_OK;
    });
}

int hubbard_server_poll(hubbard_server_h S, hubbard_completion *out, int cap, int *n, int timeout_us)
{
    return guard([&]() -> int {
        if (!S || !n || cap < 0 || (cap > 0 && !out))
            return HUBBARD_EINVAL;
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->completions.empty() && timeout_us > 0)
            S->cv.wait_for(lk, std::chrono::microseconds(timeout_us),
                           [&] { return !S->completions.empty() || S->stop; });
        int k = 0;
        while (k < cap && !S->completions.empty()) {
            out[k++] = S->completions.front();
            S->completions.pop_front();
        }
        *n = k;
        if (!S->fatal.empty() && k == 0)
            return HUBBARD_EDEVICE;
        return HUBBARD_OK;
    });
}

int hubbard_server_stats(hubbard_server_h S, hubbard_server_stats_t *st)
{
    return guard([&]() -> int {
        if (!S || !st)
            return HUBBARD_EINVAL;
        std::lock_guard<std::mutex> lk(S->mu);
        std::memset(st, 0, sizeof(*st));
        st->budget = S->budget;
        st->reserved = S->reserved;
        st->peak_reserved = S->peak_reserved;
        st->submitted = S->next_id - 1;
        st->admitted = S->admitted;
        st->completed = S->completed;
        st->rejected = S->rejected;
        st->pending = S->pending.size();
        st->max_active_batch = S->max_active_batch;
        st->slots_used = S->slots_used;
        st->solo_runs = S->solo_runs;
        return HUBBARD_OK;
    });
}

int hubbard_server_destroy(hubbard_server_h S)
{
    return guard([&]() -> int {
        if (!S)
            return HUBBARD_OK;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
        }
        S->t_build.join();
        S->t_batch.join();
        S->t_solo.join();
        for (auto *q : {&S->to_build, &S->ready_batch, &S->ready_solo})
            for (auto &job : *q)
                if (job && job->h)
                    hubbard_free(job->h);
        for (auto sb : S->s_batch)
            (void)hipStreamDestroy(sb);
        (void)hipStreamDestroy(S->s_solo);
        delete S;
        return HUBBARD_OK;
    });
}

}  // extern "C"
