// Host side of the batched Lanczos engine (kernels in batch.hip).
//
// Each call to step() advances every active instance by one step of Alg. 1
// (Sec. 2.2) with two launches.  The first launch of step j also computes
// E_{j-1} and the stop test of step j - 1 on the device and writes every
// instance's {a_{j-1}, b_j, E_{j-1}, code} to a mailbox in mapped host memory;
// the host reads them kLookahead steps behind (after that step's event), so it
// never waits for the device inside a run.  Stopped instances skip later
// steps; the descriptor table is rebuilt when instances join or when every
// listed one has finished.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "batch.h"

namespace hub {

namespace {

struct Dev {
    void *p = nullptr;
    explicit Dev(size_t bytes) { HUB_HIP(hipMalloc(&p, bytes ? bytes : 16)); }
    ~Dev()
    {
        if (p)
            (void)hipFree(p);
    }
    Dev(const Dev &) = delete;
    Dev &operator=(const Dev &) = delete;
};

// Pinned host memory that kernels write directly (mapped, coherent): the
// mailboxes reach the host with no copy in the stream.
struct Pinned {
    void *p = nullptr;
    void *dev = nullptr;  // the same memory's device address
    explicit Pinned(size_t bytes)
    {
        HUB_HIP(hipHostMalloc(&p, bytes ? bytes : 16, hipHostMallocMapped | hipHostMallocCoherent));
        HUB_HIP(hipHostGetDevicePointer(&dev, p, 0));
    }
    ~Pinned()
    {
        if (p)
            (void)hipHostFree(p);
    }
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
};

constexpr int64_t kItemElems = 2048;  // target elements per work item

int64_t rows_per_item(const hubbard *h)
{
    int64_t r = kItemElems / std::max<int64_t>(1, h->dn.dim);
    return std::max<int64_t>(1, std::min<int64_t>(r, h->up.dim));
}

template <typename T>
struct Slot {
    hubbard *h = nullptr;
    hubbard_opts o{};
    hubbard_result *res = nullptr;
    std::unique_ptr<Dev> mem;  // the instance's buffers, carved from one allocation
    void *work = nullptr;
    BatchState *state = nullptr;
    double *part = nullptr, *part2 = nullptr, *hist = nullptr;
    int64_t rpi = 1;
    int nitems = 0;
    int64_t launched = 0;  // steps launched for this instance
    int norm_at = -1;      // pending start vector: index of its squared norm in the host array
    int index = -1;  // position in the current descriptor table, -1 before the first rebuild
    std::vector<double> a, b, e;
    int stop = HUBBARD_STOP_MAXITER;
    bool done = false;
    std::chrono::steady_clock::time_point t0;
};

// Steps the device may run ahead of the host's reading of the mailboxes.
constexpr int kLookahead = 4;

template <typename T>
class Engine : public BatchRunner {
  public:
    explicit Engine(hipStream_t s) : s_(s)
    {
        for (auto &e : ev_)
            HUB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    ~Engine() override
    {
        (void)hipStreamSynchronize(s_);
        for (auto &e : ev_)
            (void)hipEventDestroy(e);
    }

    int active() const override
    {
        int n = 0;
        for (const auto &sl : slots_)
            n += !sl->done;
        return n;
    }

    void add(hubbard *h, const hubbard_opts &o, hubbard_result *res) override
    {
        auto sl = std::make_unique<Slot<T>>();
        sl->h = h;
        sl->o = o;
        sl->res = res;
        sl->t0 = std::chrono::steady_clock::now();
        const int64_t n = h->dim;
        sl->rpi = rows_per_item(h);
        sl->nitems = (int)((h->up.dim + sl->rpi - 1) / sl->rpi);
        const int sb = stream_blocks(n);
        // one allocation: the two vectors, the state, the coefficient history
        // and both sets of partial sums, each on 256 bytes
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t b_work = up(2 * sizeof(T) * (size_t)n), b_state = up(sizeof(BatchState)),
                     b_hist = up(sizeof(double) * 2 * (size_t)o.max_iter),
                     b_part = up(sizeof(double) * (size_t)std::max(sl->nitems, 2 * sb + 8)),
                     b_part2 = up(sizeof(double) * (size_t)sl->nitems);
        sl->mem = std::make_unique<Dev>(b_work + b_state + b_hist + b_part + b_part2);
        char *base = static_cast<char *>(sl->mem->p);
        sl->work = base;
        sl->state = reinterpret_cast<BatchState *>(base + b_work);
        sl->hist = reinterpret_cast<double *>(base + b_work + b_state);
        sl->part = reinterpret_cast<double *>(base + b_work + b_state + b_hist);
        sl->part2 = reinterpret_cast<double *>(base + b_work + b_state + b_hist + b_part);
        // |f_1|^2 from the seed (or the given vector), written straight to host
        // memory; the start vector is filled once all joining instances' norms
        // are known (one wait for all of them)
        if (norms_cap_ <= pending_fill_) {
            // grow before any pending norm is written: the array is only swapped while none is
            (void)hipStreamSynchronize(s_);
            std::unique_ptr<Pinned> bigger = std::make_unique<Pinned>(sizeof(double) * (size_t)(2 * norms_cap_ + 64));
            if (norms_ && pending_fill_ > 0)
                std::memcpy(bigger->p, norms_->p, sizeof(double) * (size_t)pending_fill_);
            norms_ = std::move(bigger);
            norms_cap_ = 2 * norms_cap_ + 64;
        }
        sl->norm_at = pending_fill_++;
        launch_start_norm2(o.start, o.seed, n, sl->part, sb, s_);
        launch_reduce(sl->part, sb, 0, 1, static_cast<double *>(norms_->dev) + sl->norm_at, s_);
        slots_.push_back(std::move(sl));
        dirty_ = true;
    }

    bool empty() const { return active() == 0; }

    // Launches one more step of every active instance (instances that stopped
    // on the device skip it) and reads back the mailboxes of the steps that
    // are more than kLookahead behind; returns the instances found finished.
    std::vector<hubbard_result *> step() override
    {
        std::vector<hubbard_result *> finished;
        if (dirty_)
            rebuild(finished);
        if (table_.empty())
            return finished;
        if (pending_stopped_ < (int)table_.size()) {
            const int k = (int)(launched_ % kRing);
            double *mb = static_cast<double *>(mail_host_->dev) + (size_t)k * 4 * table_.size();
            launch_batch_step<T>(static_cast<BatchInst *>(insts_->p), (int)table_.size(),
                                 static_cast<const BatchItem *>(items_->p), n_items_, lds_, mb, (int)launched_, s_);
            for (Slot<T> *sl : table_)
                sl->launched++;
            HUB_HIP(hipEventRecord(ev_[k], s_));
            launched_++;
        }
        // read back what is kLookahead steps old, or everything when every
        // instance has stopped on the device
        while (read_ < launched_ && (launched_ - read_ > kLookahead || pending_stopped_ == (int)table_.size()))
            read_step(finished);
        if (read_ == launched_ && pending_stopped_ == (int)table_.size()) {
            // every instance in the table is finished: the next step starts a fresh table
            dirty_ = true;
        }
        return finished;
    }

  private:
    static constexpr int kRing = kLookahead + 2;

    void read_step(std::vector<hubbard_result *> &finished)
    {
        const int k = (int)(read_ % kRing);
        HUB_HIP(hipEventSynchronize(ev_[k]));
        const double *mb = static_cast<const double *>(mail_host_->p) + (size_t)k * 4 * table_.size();
        for (size_t i = 0; i < table_.size(); i++) {
            Slot<T> &sl = *table_[i];
            if (sl.done)
                continue;
            const double code = mb[4 * i + 3];
            if (code == kMailStopped || code == kMailNone)
                continue;
            if (code == kMailBad)
                fail(HUBBARD_EDEVICE, "non-finite Lanczos coefficient in a batched solve");
            sl.a.push_back(mb[4 * i]);
            sl.b.push_back(mb[4 * i + 1]);
            sl.e.push_back(mb[4 * i + 2]);
            if (code != kMailRunning) {
                sl.stop = (int)code;
                finalize(sl);
                finished.push_back(sl.res);
                pending_stopped_++;
            }
        }
        read_++;
    }

    void finalize(Slot<T> &sl)
    {
        sl.done = true;
        const int m = (int)sl.a.size();
        std::vector<double> y((size_t)m);
        tridiag_lowest_vector(sl.a.data(), sl.b.data(), m, sl.e.back(), y.data());
        hubbard_result r;
        std::memset(&r, 0, sizeof(r));
        r.e0 = sl.e.back();
        r.residual = -1.0;
        r.rayleigh = NAN;
        // Lanczos estimate of |H psi - E0 psi| for the Ritz pair: b_{m+1} |y_m|
        r.err_est = std::fabs(sl.b.back() * y.back()) / std::fmax(1.0, std::fabs(r.e0));
        r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
        r.seconds_per_iter = r.seconds / m;
        r.n_iter = m;
        r.stop = sl.stop;
        r.status = (sl.stop == HUBBARD_STOP_MAXITER && sl.o.tol >= 0.0) ? HUBBARD_ENOCONV : HUBBARD_OK;
        r.precision = sl.o.precision;
        if (sl.o.a_out)
            std::memcpy(sl.o.a_out, sl.a.data(), sizeof(double) * (size_t)m);
        if (sl.o.b_out)
            std::memcpy(sl.o.b_out, sl.b.data(), sizeof(double) * (size_t)m);
        if (sl.o.e_out)
            std::memcpy(sl.o.e_out, sl.e.data(), sizeof(double) * (size_t)m);
        *sl.res = r;
    }

    // New descriptor table: waits for the steps in flight, reads their
    // mailboxes, drops finished instances (their buffers are free to go once
    // no step in flight refers to them) and lists the work items of the rest.
    void rebuild(std::vector<hubbard_result *> &finished)
    {
        HUB_HIP(hipStreamSynchronize(s_));
        while (read_ < launched_)
            read_step(finished);
        // start vectors of the instances that joined: f_1 = f / |f| (Alg. 1)
        const double *nh = norms_ ? static_cast<const double *>(norms_->p) : nullptr;
        for (auto &slp : slots_) {
            Slot<T> &sl = *slp;
            if (sl.norm_at < 0)
                continue;
            const double nrm2 = nh[sl.norm_at];
            sl.norm_at = -1;
            if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
                fail(HUBBARD_EINVAL, "start vector has zero or non-finite norm");
            const hubbard *h = sl.h;
            T *v0 = static_cast<T *>(sl.work);
            launch_start_fill<T>(sl.o.start, sl.o.seed, 1.0 / std::sqrt(nrm2), v0, v0 + h->dim, h->up.dim, h->dn.dim,
                                 h->dn.dim, s_);
            launch_batch_init_state(sl.state, s_);
        }
        pending_fill_ = 0;
        std::vector<std::unique_ptr<Slot<T>>> keep;
        for (auto &sl : slots_)
            if (!sl->done)
                keep.push_back(std::move(sl));
        slots_.swap(keep);
        table_.clear();
        launched_ = read_ = 0;
        pending_stopped_ = 0;
        dirty_ = false;
        const int n = (int)slots_.size();
        if (n == 0)
            return;
        std::vector<BatchInst> desc((size_t)n);
        std::vector<BatchItem> items;
        size_t lds = 16;
        for (int i = 0; i < n; i++) {
            Slot<T> &sl = *slots_[(size_t)i];
            const hubbard *h = sl.h;
            BatchInst &d = desc[(size_t)i];
            std::memset(&d, 0, sizeof(d));
            d.states_up = h->dev.states_up;
            d.states_dn = h->dev.states_dn;
            d.up_rows = h->dev.up_rows;
            d.dn_cols = h->dev.dn_cols;
            d.nnz_up = h->dev.nnz_up;
            d.nnz_dn = h->dev.nnz_dn;
            d.dim_up = h->up.dim;
            d.dim_dn = h->dn.dim;
            d.dim = h->dim;
            d.w_up = std::max(1, h->up.width);
            d.w_dn = h->dn.width;
            d.t = h->t;
            d.U = h->U;
            T *v0 = static_cast<T *>(sl.work);
            d.vec0 = v0;
            d.vec1 = v0 + h->dim;
            d.st = sl.state;
            d.hist = sl.hist;
            d.part = sl.part;
            d.part2 = sl.part2;
            d.tol = sl.o.tol;
            d.nparts = sl.nitems;
            d.slot = i;
            d.max_iter = sl.o.max_iter;
            d.j0 = (int32_t)sl.launched;
            sl.index = i;
            for (int k = 0; k < sl.nitems; k++) {
                BatchItem it;
                it.inst = i;
                it.part = k;
                it.r0 = (int64_t)k * sl.rpi;
                it.nrows = std::min<int64_t>(sl.rpi, h->up.dim - it.r0);
                items.push_back(it);
            }
            lds = std::max(lds, (size_t)sl.rpi * (size_t)h->dn.dim * sizeof(T));  // one work item's rows
            table_.push_back(&sl);
        }
        if (!insts_ || insts_cap_ < (size_t)n) {
            insts_cap_ = (size_t)n * 2;
            insts_ = std::make_unique<Dev>(sizeof(BatchInst) * insts_cap_);
            mail_host_ = std::make_unique<Pinned>(sizeof(double) * 4 * insts_cap_ * kRing);
        }
        if (!items_ || items_cap_ < items.size()) {
            items_cap_ = items.size() * 2;
            items_ = std::make_unique<Dev>(sizeof(BatchItem) * items_cap_);
        }
        HUB_HIP(hipMemcpyAsync(insts_->p, desc.data(), sizeof(BatchInst) * (size_t)n, hipMemcpyHostToDevice, s_));
        HUB_HIP(hipMemcpyAsync(items_->p, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice, s_));
        HUB_HIP(hipStreamSynchronize(s_));
        n_items_ = (int)items.size();
        lds_ = lds;
    }

    hipStream_t s_;
    std::vector<std::unique_ptr<Slot<T>>> slots_;
    std::vector<Slot<T> *> table_;  // the instances of the current descriptor table, in slot order
    std::unique_ptr<Dev> insts_, items_;
    std::unique_ptr<Pinned> mail_host_;
    std::unique_ptr<Pinned> norms_;  // squared start norms of joining instances (written by the device)
    int norms_cap_ = 0, pending_fill_ = 0;
    hipEvent_t ev_[kRing];
    size_t insts_cap_ = 0, items_cap_ = 0, lds_ = 16;
    int n_items_ = 0;
    int64_t launched_ = 0, read_ = 0;  // steps launched and read back since the last rebuild
    int pending_stopped_ = 0;         // instances of the table found finished
    bool dirty_ = true;
};

}  // namespace

std::unique_ptr<BatchRunner> BatchRunner::make(int precision, hipStream_t s)
{
    if (precision == HUBBARD_FP64)
        return std::make_unique<Engine<double>>(s);
    return std::make_unique<Engine<float>>(s);
}

size_t batch_vector_bytes(const hubbard *h, int precision)
{
    const size_t es = precision == HUBBARD_FP64 ? 8 : 4;
    const int64_t rpi = rows_per_item(h);
    const int64_t items = (h->up.dim + rpi - 1) / rpi;
    return 2 * es * (size_t)h->dim + 8 * sizeof(double) +
           sizeof(double) * (size_t)(std::max<int64_t>(items, 2 * stream_blocks(h->dim) + 8) + items);
}

bool batchable(const hubbard *h, int precision)
{
    const size_t es = precision == HUBBARD_FP64 ? 8 : 4;
    // the batched kernels take one amplitude t for every hop
    return h->device >= 0 && h->tcls.empty() && (size_t)h->dn.dim * es <= 64 * 1024;
}

// The solves of one precision go to kBatchStreams engines on as many streams
// (sorted by size and dealt in snake order, 0, 1, .., k-1, k-1, .., 0, so all
// carry about the same work), stepped in turn: the step launches of one stream
// fill the gaps between those of the others.  Each solve's arithmetic is that
// of an engine of its own.  Two streams: measured on 64 solves, four were
// slower than two (more launches and host work per step for the same gaps).
constexpr int kBatchStreams = 2;

namespace {
struct StreamSet {
    hipStream_t s[kBatchStreams] = {};
    explicit StreamSet(hipStream_t first)
    {
        s[0] = first;
        for (int k = 1; k < kBatchStreams; k++)
            HUB_HIP(hipStreamCreateWithFlags(&s[k], hipStreamNonBlocking));
    }
    ~StreamSet()
    {
        for (int k = 1; k < kBatchStreams; k++)
            if (s[k])
                (void)hipStreamDestroy(s[k]);
    }
};

template <typename T>
void run_group(hubbard **hs, const hubbard_opts *opts, hubbard_result *res, const std::vector<int> &idx,
               const StreamSet &ss)
{
    if (idx.empty())
        return;
    const int ne = std::min<int>(kBatchStreams, (int)idx.size());
    // the other streams start after the work already queued on the first
    hipEvent_t ev;
    HUB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HUB_HIP(hipEventRecord(ev, ss.s[0]));
    for (int k = 1; k < ne; k++)
        HUB_HIP(hipStreamWaitEvent(ss.s[k], ev, 0));
    (void)hipEventDestroy(ev);
    std::vector<int> order = idx;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a]->dim > hs[b]->dim; });
    std::vector<std::unique_ptr<Engine<T>>> eng;
    for (int k = 0; k < ne; k++)
        eng.push_back(std::make_unique<Engine<T>>(ss.s[k]));
    for (size_t q = 0; q < order.size(); q++) {
        const int r = (int)(q % (size_t)(2 * ne));
        const int k = r < ne ? r : 2 * ne - 1 - r;
        eng[(size_t)k]->add(hs[order[q]], opts[order[q]], &res[order[q]]);
    }
    for (bool any = true; any;) {
        any = false;
        for (auto &e : eng)
            if (!e->empty()) {
                e->step();
                any = true;
            }
    }
}
}  // namespace

void run_batch(hubbard **hs, const hubbard_opts *opts, hubbard_result *res, int n, hipStream_t s)
{
    std::vector<int> i64, i32;
    for (int i = 0; i < n; i++)
        (opts[i].precision == HUBBARD_FP64 ? i64 : i32).push_back(i);
    StreamSet ss(s);
    run_group<double>(hs, opts, res, i64, ss);
    run_group<float>(hs, opts, res, i32, ss);
    // the engines synchronise their streams when they end, so the caller's
    // stream sees every solve done
}

}  // namespace hub
