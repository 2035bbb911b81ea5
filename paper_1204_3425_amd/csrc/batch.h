// Batched Lanczos: device descriptors and the host engine (not part of the ABI).
#pragma once

#include <memory>
#include <vector>

#include "internal.h"

namespace hub {

// One instance as the batched kernels see it (plain data, device memory).
struct BatchInst {
    const uint32_t *states_up, *states_dn, *up_rows, *dn_cols;
    const uint16_t *nnz_up, *nnz_dn;
    int64_t dim_up, dim_dn;
    int32_t w_up, w_dn;
    double t, U;
    void *vec0, *vec1;  // the two Lanczos vectors, dense rows
    double *S;          // {1/s of the current vector, alpha, beta, c, -, -, a_j, b_{j+1}}
    double *part;       // partial sums, one per work item of this instance
    int32_t nparts;
    int32_t cur;        // 0: vec0 holds s f_j, 1: vec1 does
    int32_t slot;       // mailbox slot
    int32_t pad_;
};

// A work item: rows [r0, r0 + nrows) of instance `inst`, writing partial `part`.
struct BatchItem {
    int32_t inst;
    int32_t part;
    int64_t r0;
    int64_t nrows;
};

template <typename T>
void launch_batch_step(BatchInst *insts_dev, int n_inst, const BatchItem *items_dev, int n_items, size_t lds_bytes,
                       double *mailbox_dev, hipStream_t s);

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
    // one Lanczos step of every active instance; returns the results finished in it
    virtual std::vector<hubbard_result *> step() = 0;
    virtual int active() const = 0;
};

// Runs the given solves (all batchable, psi NULL) to completion as one batch.
void run_batch(hubbard **hs, const hubbard_opts *opts, hubbard_result *res, int n, hipStream_t s);

}  // namespace hub
