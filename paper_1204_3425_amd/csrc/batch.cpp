// Host side of the batched Lanczos engine (kernels in batch.hip).
//
// Each call to step() advances every active instance by one step of Alg. 1
// (Sec. 2.2) with four launches, then reads every instance's (a_j, b_{j+1})
// from one mailbox copy and applies the energy test.  Converged instances
// leave the batch; the work-item list is rebuilt only when the set changes.
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

struct Pinned {
    void *p = nullptr;
    explicit Pinned(size_t bytes) { HUB_HIP(hipHostMalloc(&p, bytes ? bytes : 16, hipHostMallocDefault)); }
    ~Pinned()
    {
        if (p)
            (void)hipHostFree(p);
    }
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
};

constexpr int64_t kItemElems = 8192;  // target elements per work item

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
    std::unique_ptr<Dev> work, scal, part;
    int64_t rpi = 1;
    int nitems = 0;
    int cur = 0;
    std::vector<double> a, b, e;
    double scale = 0.0;
    int stop = HUBBARD_STOP_MAXITER;
    bool done = false;
    std::chrono::steady_clock::time_point t0;
};

template <typename T>
class Engine : public BatchRunner {
  public:
    explicit Engine(hipStream_t s) : s_(s) {}

    int active() const override { return (int)active_.size(); }

    void add(hubbard *h, const hubbard_opts &o, hubbard_result *res) override
    {
        auto sl = std::make_unique<Slot<T>>();
        sl->h = h;
        sl->o = o;
        sl->res = res;
        sl->t0 = std::chrono::steady_clock::now();
        const int64_t n = h->dim;
        sl->work = std::make_unique<Dev>(2 * sizeof(T) * (size_t)n);
        sl->scal = std::make_unique<Dev>(8 * sizeof(double));
        sl->rpi = rows_per_item(h);
        sl->nitems = (int)((h->up.dim + sl->rpi - 1) / sl->rpi);
        const int sb = stream_blocks(n);
        sl->part = std::make_unique<Dev>(sizeof(double) * (size_t)std::max(sl->nitems, 2 * sb + 8));
        // f_1 from the seed (or the given vector), normalised in FP64 (Alg. 1)
        double *part = static_cast<double *>(sl->part->p);
        double *S = static_cast<double *>(sl->scal->p);
        launch_start_norm2(o.start, o.seed, n, part, sb, s_);
        launch_reduce(part, sb, 0, 1, S + 4, s_);
        double nrm2 = 0.0;
        HUB_HIP(hipMemcpyAsync(&nrm2, S + 4, sizeof(double), hipMemcpyDeviceToHost, s_));
        HUB_HIP(hipStreamSynchronize(s_));
        if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
            fail(HUBBARD_EINVAL, "start vector has zero or non-finite norm");
        T *v0 = static_cast<T *>(sl->work->p);
        launch_start_fill<T>(o.start, o.seed, 1.0 / std::sqrt(nrm2), v0, v0 + n, h->up.dim, h->dn.dim, h->dn.dim, s_);
        launch_init_scalars(S, s_);
        active_.push_back(std::move(sl));
        dirty_ = true;
    }

    bool empty() const { return active_.empty(); }

    // One Lanczos step for every active instance; finished ones are finalised
    // and removed.
    std::vector<hubbard_result *> step() override
    {
        std::vector<hubbard_result *> finished;
        if (active_.empty())
            return finished;
        if (dirty_)
            rebuild();
        const int n = (int)active_.size();
        launch_batch_step<T>(static_cast<BatchInst *>(insts_->p), n, static_cast<const BatchItem *>(items_->p),
                             n_items_, lds_, static_cast<double *>(mail_->p), s_);
        HUB_HIP(hipMemcpyAsync(mail_host_->p, mail_->p, sizeof(double) * 2 * (size_t)n, hipMemcpyDeviceToHost, s_));
        HUB_HIP(hipStreamSynchronize(s_));
        const double *mb = static_cast<const double *>(mail_host_->p);
        bool any_done = false;
        for (int i = 0; i < n; i++) {
            Slot<T> &sl = *active_[(size_t)i];
            sl.cur ^= 1;
            if (check(sl, mb[2 * i], mb[2 * i + 1])) {
                finalize(sl);
                finished.push_back(sl.res);
                any_done = true;
            }
        }
        if (any_done) {
            std::vector<std::unique_ptr<Slot<T>>> keep;
            for (auto &sl : active_)
                if (!sl->done)
                    keep.push_back(std::move(sl));
            active_.swap(keep);
            dirty_ = true;
        }
        return finished;
    }

  private:
    // the energy test of Sec. 2.2 and the breakdown rule, as in the single-instance driver
    bool check(Slot<T> &sl, double a, double b)
    {
        if (!std::isfinite(a) || !std::isfinite(b))
            fail(HUBBARD_EDEVICE, "non-finite Lanczos coefficient in a batched solve");
        sl.a.push_back(a);
        sl.b.push_back(b);
        const int j = (int)sl.a.size();
        const double e = tridiag_lowest(sl.a.data(), sl.b.data(), j);
        sl.e.push_back(e);
        if (sl.o.tol >= 0.0 && j >= 2 && std::fabs(e - sl.e[(size_t)j - 2]) <= sl.o.tol * std::fmax(1.0, std::fabs(e))) {
            sl.stop = HUBBARD_STOP_CONVERGED;
            return true;
        }
        sl.scale = std::fmax(sl.scale, std::fabs(a) + (j > 1 ? sl.b[(size_t)j - 2] : 0.0));
        if (b == 0.0 || b <= 1e-12 * sl.scale) {
            sl.stop = HUBBARD_STOP_BREAKDOWN;
            return true;
        }
        if ((int64_t)j >= sl.h->dim) {
            sl.stop = HUBBARD_STOP_EXHAUSTED;
            return true;
        }
        if (j >= sl.o.max_iter) {
            sl.stop = HUBBARD_STOP_MAXITER;
            return true;
        }
        return false;
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

    void rebuild()
    {
        const int n = (int)active_.size();
        std::vector<BatchInst> desc((size_t)n);
        std::vector<BatchItem> items;
        size_t lds = 16;
        for (int i = 0; i < n; i++) {
            Slot<T> &sl = *active_[(size_t)i];
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
            d.w_up = std::max(1, h->up.width);
            d.w_dn = h->dn.width;
            d.t = h->t;
            d.U = h->U;
            T *v0 = static_cast<T *>(sl.work->p);
            d.vec0 = v0;
            d.vec1 = v0 + h->dim;
            d.S = static_cast<double *>(sl.scal->p);
            d.part = static_cast<double *>(sl.part->p);
            d.nparts = sl.nitems;
            d.cur = sl.cur;
            d.slot = i;
            for (int k = 0; k < sl.nitems; k++) {
                BatchItem it;
                it.inst = i;
                it.part = k;
                it.r0 = (int64_t)k * sl.rpi;
                it.nrows = std::min<int64_t>(sl.rpi, h->up.dim - it.r0);
                items.push_back(it);
            }
            lds = std::max(lds, (size_t)h->dn.dim * sizeof(T));
        }
        if (!insts_ || insts_cap_ < (size_t)n) {
            insts_cap_ = (size_t)n * 2;
            insts_ = std::make_unique<Dev>(sizeof(BatchInst) * insts_cap_);
            mail_ = std::make_unique<Dev>(sizeof(double) * 2 * insts_cap_);
            mail_host_ = std::make_unique<Pinned>(sizeof(double) * 2 * insts_cap_);
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
        dirty_ = false;
    }

    hipStream_t s_;
    std::vector<std::unique_ptr<Slot<T>>> active_;
    std::unique_ptr<Dev> insts_, items_, mail_;
    std::unique_ptr<Pinned> mail_host_;
    size_t insts_cap_ = 0, items_cap_ = 0, lds_ = 16;
    int n_items_ = 0;
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
           sizeof(double) * (size_t)std::max<int64_t>(items, 2 * stream_blocks(h->dim) + 8);
}

bool batchable(const hubbard *h, int precision)
{
    const size_t es = precision == HUBBARD_FP64 ? 8 : 4;
    return h->device >= 0 && (size_t)h->dn.dim * es <= 64 * 1024;
}

void run_batch(hubbard **hs, const hubbard_opts *opts, hubbard_result *res, int n, hipStream_t s)
{
    Engine<double> e64(s);
    Engine<float> e32(s);
    for (int i = 0; i < n; i++) {
        if (opts[i].precision == HUBBARD_FP64)
            e64.add(hs[i], opts[i], &res[i]);
        else
            e32.add(hs[i], opts[i], &res[i]);
    }
    while (!e64.empty())
        e64.step();
    while (!e32.empty())
        e32.step();
}

}  // namespace hub
