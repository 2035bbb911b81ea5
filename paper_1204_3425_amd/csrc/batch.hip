// Batched Lanczos for many small sectors (Sec. 2.2, Alg. 1; Sec. 4.3 H.v).
//
// A sector of a few thousand to a million states leaves most of the MI355X
// idle (the paper's Sec. 5 reports the same for small systems on its GPU).
// The batch engine advances every active instance by one Lanczos step with
// four launches in total, whatever the number of instances:
//     batched H.v + three-term update  (work item = rows of one instance)
//     per-instance reduction -> a_j
//     batched q - a_j f_j + partial norms
//     per-instance reduction -> b_{j+1}
// Work items never span two instances and each instance's partial sums are
// added in a fixed order, so an instance's results do not depend on which
// other instances share the launches.
//
// H.v here is the one-pass form: a workgroup stages each row of its work item
// in LDS, gathers the down-spin hops from it and adds the up-spin rows from
// global memory (every vector of a batched instance is small enough to stay in
// the L2 and the Infinity Cache).
#include <hip/hip_runtime.h>

#include "batch.h"

namespace hub {

namespace {

__device__ inline double wg_sum(double v, double *scratch)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); w++)
            s += scratch[w];
    __syncthreads();
    return s;
}

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void batch_hv_kernel(const BatchInst *__restrict__ insts,
                                                            const BatchItem *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kThreads / 64];
    const BatchItem it = items[blockIdx.x];
    const BatchInst &in = insts[it.inst];
    const int64_t ddn = in.dim_dn;
    const T *__restrict__ x = reinterpret_cast<const T *>(in.cur ? in.vec1 : in.vec0);
    T *__restrict__ y = reinterpret_cast<T *>(in.cur ? in.vec0 : in.vec1);
    const double alpha = in.S[1], beta = in.S[2];
    const T a_s = (T)alpha, b_s = (T)beta, tp = (T)in.t, tm = (T)(-in.t), U = (T)in.U;
    double acc = 0.0;
    for (int64_t r = it.r0; r < it.r0 + it.nrows; r++) {
        const T *__restrict__ xr = x + r * ddn;
        for (int64_t d = threadIdx.x; d < ddn; d += blockDim.x)
            xs[d] = xr[d];
        __syncthreads();
        const uint32_t su = in.states_up[r];
        const int nu = in.nnz_up[r];
        const uint32_t *__restrict__ urow = in.up_rows + r * in.w_up;
        for (int64_t d = threadIdx.x; d < ddn; d += blockDim.x) {
            const T xv = xs[d];
            T h = U * (T)__popc(su & in.states_dn[d]) * xv;
            const int nd = in.nnz_dn[d];
            for (int k = 0; k < nd; k++) {
                const uint32_t e = in.dn_cols[(int64_t)k * ddn + d];
                h = fma((e >> 31) ? tp : tm, xs[e & 0x7fffffffu], h);
            }
            for (int k = 0; k < nu; k++) {
                const uint32_t e = urow[k];
                h = fma((e >> 31) ? tp : tm, x[(int64_t)(e & 0x7fffffffu) * ddn + d], h);
            }
            const int64_t J = r * ddn + d;
            const T q = a_s * h + b_s * y[J];
            y[J] = q;
            acc += (double)q * (double)xv;
        }
        __syncthreads();
    }
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0)
        in.part[it.part] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void batch_axpy_kernel(const BatchInst *__restrict__ insts,
                                                              const BatchItem *__restrict__ items)
{
    __shared__ double red[kThreads / 64];
    const BatchItem it = items[blockIdx.x];
    const BatchInst &in = insts[it.inst];
    const T *__restrict__ v = reinterpret_cast<const T *>(in.cur ? in.vec1 : in.vec0);
    T *__restrict__ w = reinterpret_cast<T *>(in.cur ? in.vec0 : in.vec1);
    const T c = (T)in.S[3];
    const int64_t i0 = it.r0 * in.dim_dn, i1 = (it.r0 + it.nrows) * in.dim_dn;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const T q = w[i] - c * v[i];
        w[i] = q;
        acc += (double)q * (double)q;
    }
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0)
        in.part[it.part] = s;
}

// One workgroup per instance: fixed-order sum of its partials, then the same
// scalar updates as the single-instance driver (a_j after the H.v, b_{j+1}
// and the next step's alpha, beta after the update).  The step's (a, b) is
// also written to the instance's slot of the mailbox the host reads, and the
// two vectors swap roles (the updated q holds b_{j+1} f_{j+1}).
__global__ __launch_bounds__(kThreads) void batch_reduce_kernel(BatchInst *__restrict__ insts, int mode,
                                                                double *__restrict__ mailbox)
{
    __shared__ double red[kThreads / 64];
    BatchInst &in = insts[blockIdx.x];
    double acc = 0.0;
    for (int i = threadIdx.x; i < in.nparts; i += blockDim.x)
        acc += in.part[i];
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0) {
        double *S = in.S;
        if (mode == 0) {
            const double a = s * S[0];
            S[3] = a * S[0];
            S[6] = a;
        } else {
            const double b = sqrt(s);
            S[7] = b;
            S[2] = -b * S[0];
            S[0] = b > 0.0 ? 1.0 / b : 0.0;
            S[1] = S[0];
            mailbox[2 * in.slot] = S[6];
            mailbox[2 * in.slot + 1] = b;
            in.cur ^= 1;
        }
    }
}

}  // namespace

template <typename T>
void launch_batch_step(BatchInst *insts_dev, int n_inst, const BatchItem *items_dev, int n_items, size_t lds_bytes,
                       double *mailbox_dev, hipStream_t s)
{
    auto hv = batch_hv_kernel<T>;
    if (lds_bytes > 64 * 1024)
        HUB_HIP(hipFuncSetAttribute((const void *)hv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    hipLaunchKernelGGL(hv, dim3(n_items), dim3(kThreads), lds_bytes, s, insts_dev, items_dev);
    HUB_HIP(hipGetLastError());
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(n_inst), dim3(kThreads), 0, s, insts_dev, 0, mailbox_dev);
    HUB_HIP(hipGetLastError());
    hipLaunchKernelGGL(batch_axpy_kernel<T>, dim3(n_items), dim3(kThreads), 0, s, insts_dev, items_dev);
    HUB_HIP(hipGetLastError());
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(n_inst), dim3(kThreads), 0, s, insts_dev, 1, mailbox_dev);
    HUB_HIP(hipGetLastError());
}

template void launch_batch_step<double>(BatchInst *, int, const BatchItem *, int, size_t, double *, hipStream_t);
template void launch_batch_step<float>(BatchInst *, int, const BatchItem *, int, size_t, double *, hipStream_t);

}  // namespace hub
