// Batched Lanczos: device descriptors and the host engine (not part of the ABI).
#pragma once

#include <memory>
#include <vector>

#include "internal.h"

namespace hub {

// Per-instance state (device memory, owned by the instance; descriptors stay
// read-only between rebuilds).  The step's scalars are not kept here: every
// workgroup derives them from the recorded coefficients and partial sums.
struct BatchState {
    double S[8];     // S[4]: squared norm of the start vector (set up by the host path)
    double scale;    // running max_k |a_k| + b_k (breakdown test)
    double e_prev;   // Ritz value of the previous step
    double e_prev2;  // and of the step before
    int32_t j;       // steps whose coefficients are recorded
    int32_t stopped; // set when the stop test of a step fires
    int32_t cur;     // unused (the vector roles follow the step's parity)
    int32_t pad_;
};

// One instance as the batched kernels see it (plain data, device memory).
struct BatchInst {
    const uint32_t *states_up, *states_dn, *up_rows, *dn_cols;
    const uint16_t *nnz_up, *nnz_dn;
    int64_t dim_up, dim_dn, dim;
    int32_t w_up, w_dn;
    double t, U;
    void *vec0, *vec1;  // the two Lanczos vectors, dense rows
    BatchState *st;
    double *hist;       // a_{k+1} at 2k, b_{k+2} at 2k + 1
    double *part;       // H.v partial sums (y.x), one per work item of this instance
    double *part2;      // update partial sums (|q|^2), one per work item
    double tol;
    int32_t nparts;
    int32_t slot;       // mailbox slot
    int32_t max_iter;
    int32_t j0;         // steps launched for this instance before the table was built
};

// Mailbox entry for every instance, written by the launch that computes the
// Ritz value of the step before (the first launch of step j reports step
// j - 1): {a, b, E, code}; code = -1 running, a HUBBARD_STOP_* value when that
// step stops the instance, kMailStopped when it had stopped before, kMailBad
// when a coefficient is not finite, kMailNone when there is no step before.
constexpr double kMailRunning = -1.0;
constexpr double kMailStopped = -2.0;
constexpr double kMailBad = -3.0;
constexpr double kMailNone = -4.0;

// A work item: rows [r0, r0 + nrows) of instance `inst`, writing partial `part`.
struct BatchItem {
    int32_t inst;
    int32_t part;
    int64_t r0;
    int64_t nrows;
};

// One Lanczos step j of every active instance in two launches: the H.v with
// the three-term update (and, in extra workgroups, the Ritz value and stop
// test of step j - 1), then the q - a_j f_j update with its norm.
template <typename T>
void launch_batch_step(BatchInst *insts_dev, int n_inst, const BatchItem *items_dev, int n_items, size_t lds_bytes,
                       double *mailbox_dev, int j, hipStream_t s);

// zeroes an instance's state and sets S = {1, 1, 0, 0} (f_1 has scale 1, b_1 = 0)
void launch_batch_init_state(BatchState *st, hipStream_t s);

// Largest sector the batched kernels take: a row must fit in 64 KB of LDS.
bool batchable(const hubbard *h, int precision);

// Device bytes a batched solve allocates besides the handle's tables.
size_t batch_vector_bytes(const hubbard *h, int precision);

// A batch that instances can join between steps (the serving loop uses it).
class BatchRunner {
  public:
    virtual ~BatchRunner() = default;
    static std::unique_ptr<BatchRunner> make(int precision, hipStream_t s);
    // allocates the instance's vectors and writes its start vector; res is
    // written when the instance finishes
    virtual void add(hubbard *h, const hubbard_opts &o, hubbard_result *res) = 0;
    // launches one more Lanczos step of every active instance and returns the
    // results that finished in steps the host has read back (the host reads
    // the step mailboxes a few steps behind the device)
    virtual std::vector<hubbard_result *> step() = 0;
    virtual int active() const = 0;
};

// Runs the given solves (all batchable, psi NULL) to completion as one batch.
void run_batch(hubbard **hs, const hubbard_opts *opts, hubbard_result *res, int n, hipStream_t s);

}  // namespace hub
