// Batched Lanczos for many small sectors (Sec. 2.2, Alg. 1; Sec. 4.3 H.v).
//
// A sector of a few thousand to a million states leaves most of the MI355X
// idle (the paper's Sec. 5 reports the same for small systems on its GPU).
// The batch engine advances every active instance by one Lanczos step with
// two launches in total, whatever the number of instances:
//     batched H.v + three-term update (work item = rows of one instance),
//         and one extra workgroup per instance that finishes the step before:
//         b_j, the Ritz value E_{j-1} of T_j and the stop test of the
//         single-instance driver, with the mailbox entry
//     batched q - a_j f_j update + partial norms
// Each workgroup derives the step's scalars itself: a_j from the instance's
// H.v partial sums and b_j from its update partial sums, summed in the same
// fixed order everywhere, so no launch is spent on reductions alone and the
// Ritz value (a multisection) runs beside the next H.v instead of before it.
// A step that a stop test ends is therefore followed by one more H.v whose
// result is never used.  Work items never span two instances and each
// instance's partial sums are added in a fixed order, so an instance's results
// do not depend on which other instances share the launches.  An instance
// that has stopped skips every kernel of later steps, so the host can read the
// step mailboxes a few steps behind without holding the device.
//
// H.v here is the one-pass form: a workgroup stages the rows of its work item
// in LDS, gathers the down-spin hops from them and adds the up-spin rows from
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

// The work item's rows are staged in LDS at once (each thread issues eight
// loads before its first LDS write); then the item's elements are spread over
// all threads, row by row, so short rows leave no lane idle.  A thread keeps
// its position (r, d) and steps it by the workgroup size.  Down-spin hops read
// LDS, with a column's table entries loaded eight at a time before the
// gathers; up-spin hops read the other rows from global memory, four at a time.
// Fixed-order sum of an instance's n partial sums, returned to every thread
// (every workgroup that needs it gets the same value).
__device__ inline double inst_sum(const double *__restrict__ part, int n, double *red)
{
    __shared__ double total;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        acc += part[i];
    const double s = wg_sum(acc, red);  // in thread 0
    if (threadIdx.x == 0)
        total = s;
    __syncthreads();
    const double r = total;
    __syncthreads();
    return r;
}

__device__ __forceinline__ void ritz_and_stop(const BatchInst &in, int j, double *__restrict__ mailbox);

// Workgroups 0 .. n_inst-1 finish step j - 1 of their instance (ritz_and_stop);
// the others are the work items of step j.
template <typename T>
__global__ __launch_bounds__(kThreads) void batch_hv_kernel(const BatchInst *__restrict__ insts,
                                                            const BatchItem *__restrict__ items, int n_inst, int k,
                                                            double *__restrict__ mailbox)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[kThreads / 64];
    if ((int)blockIdx.x < n_inst) {
        const BatchInst &in = insts[blockIdx.x];
        ritz_and_stop(in, in.j0 + k, mailbox);
        return;
    }
    const BatchItem it = items[blockIdx.x - n_inst];
    const BatchInst &in = insts[it.inst];
    const BatchState *st = in.st;
    // the instance's Ritz workgroup may set the flag during this launch: one
    // read for the whole workgroup, so all its waves agree
    __shared__ int stopped;
    if (threadIdx.x == 0)
        stopped = st->stopped;
    __syncthreads();
    if (stopped)
        return;
    const int j = in.j0 + k;  // this instance's step
    const int ddn = (int)in.dim_dn;
    const int n = (int)(it.nrows * in.dim_dn);  // elements of the item (at most 16384)
    // x = s_j f_j with 1/s_j = S0: vec0 on even steps; y holds s_{j-1} f_{j-1}
    const T *__restrict__ x = reinterpret_cast<const T *>((j & 1) ? in.vec1 : in.vec0);
    T *__restrict__ y = reinterpret_cast<T *>((j & 1) ? in.vec0 : in.vec1);
    // b_j from the update partials of step j - 1; b_{j-1} as recorded
    const double bj = j >= 1 ? sqrt(inst_sum(in.part2, in.nparts, red)) : 1.0;
    const double bjm1 = j >= 2 ? in.hist[2 * j - 3] : 1.0;
    const double s0 = bj > 0.0 ? 1.0 / bj : 0.0, s0_old = bjm1 > 0.0 ? 1.0 / bjm1 : 0.0;
    const double alpha = s0, beta = j >= 1 ? -bj * s0_old : 0.0;
    const T a_s = (T)alpha, b_s = (T)beta, tp = (T)in.t, tm = (T)(-in.t), U = (T)in.U;
    const int64_t base = it.r0 * in.dim_dn;
    for (int i0 = 0; i0 < n; i0 += 8 * kThreads) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int i = i0 + u * kThreads + (int)threadIdx.x;
            v[u] = i < n ? x[base + i] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int i = i0 + u * kThreads + (int)threadIdx.x;
            if (i < n)
                xs[i] = v[u];
        }
    }
    __syncthreads();
    double acc = 0.0;
    int rl = (int)threadIdx.x / ddn, d = (int)threadIdx.x - rl * ddn;
    for (int i = (int)threadIdx.x; i < n; i += kThreads) {
        const int64_t r = it.r0 + rl;
        const T xv = xs[i];
        const T *__restrict__ xrow = xs + (int64_t)rl * ddn;
        T h = U * (T)__popc(in.states_up[r] & in.states_dn[d]) * xv;
        const int nd = in.nnz_dn[d];
        for (int k0 = 0; k0 < nd; k0 += 8) {
            uint32_t e[8];
#pragma unroll
            for (int u = 0; u < 8; u++)
                e[u] = k0 + u < nd ? in.dn_cols[(int64_t)(k0 + u) * ddn + d] : 0u;
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (k0 + u < nd)
                    h = fma((e[u] >> 31) ? tp : tm, xrow[e[u] & 0x7fffffffu], h);
        }
        const int nu = in.nnz_up[r];
        const uint32_t *__restrict__ urow = in.up_rows + r * in.w_up;
        for (int k0 = 0; k0 < nu; k0 += 4) {
            T v[4];
            uint32_t e[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                e[u] = k0 + u < nu ? urow[k0 + u] : 0u;
                v[u] = k0 + u < nu ? x[(int64_t)(e[u] & 0x7fffffffu) * ddn + d] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (k0 + u < nu)
                    h = fma((e[u] >> 31) ? tp : tm, v[u], h);
        }
        const int64_t J = base + i;
        const T q = a_s * h + b_s * y[J];
        y[J] = q;
        acc += (double)q * (double)xv;
        d += kThreads;
        while (d >= ddn) {
            d -= ddn;
            rl++;
        }
    }
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0)
        in.part[it.part] = s;
}

// q <- q - a_j f_j with a_j from the H.v partial sums (recorded by the
// instance's first item), and the partial sums of |q|^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void batch_axpy_kernel(const BatchInst *__restrict__ insts,
                                                              const BatchItem *__restrict__ items, int k)
{
    __shared__ double red[kThreads / 64];
    const BatchItem it = items[blockIdx.x];
    const BatchInst &in = insts[it.inst];
    const BatchState *st = in.st;
    if (st->stopped)
        return;
    const int j = in.j0 + k;
    const T *__restrict__ v = reinterpret_cast<const T *>((j & 1) ? in.vec1 : in.vec0);
    T *__restrict__ w = reinterpret_cast<T *>((j & 1) ? in.vec0 : in.vec1);
    const double bj = j >= 1 ? in.hist[2 * j - 1] : 1.0;
    const double s0 = bj > 0.0 ? 1.0 / bj : 0.0;
    const double a = inst_sum(in.part, in.nparts, red) * s0;
    if (it.part == 0 && threadIdx.x == 0)
        in.hist[2 * j] = a;
    const T c = (T)(a * s0);
    const int64_t i0 = it.r0 * in.dim_dn, i1 = (it.r0 + it.nrows) * in.dim_dn;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const T q = w[i] - c * v[i];
        w[i] = q;
        acc += (double)q * (double)q;
    }
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0)
        in.part2[it.part] = s;
}

// Number of negative pivots of the LDL^T factorisation of T_m - x I (T_m:
// diagonal hist[0], hist[2], ..., off-diagonal hist[1], hist[3], ...), which
// by Sylvester's law of inertia is the number of eigenvalues of T_m below x.
// The pivot recurrence is a serial chain, so the division is the hardware
// reciprocal estimate refined by one Newton step (r' = r + r (1 - p r), which
// squares its relative error to below FP64 rounding) times the squared
// off-diagonal, instead of the longer correctly rounded division sequence.
__device__ inline double recip(double p)
{
    const double r = __builtin_amdgcn_rcp(p);
    return fma(r, fma(-p, r, 1.0), r);
}

// T_m as the pivot recurrence reads it: diagonal dg[i] and squared
// off-diagonal o2[i] (coupling of i-1 and i), staged in LDS when T_m is short
// enough (every step of the recurrence then reads LDS, not global memory),
// else read from the recorded coefficients.
constexpr int kRitzLds = 256;
struct TriView {
    const double *dg, *o2;     // LDS copies (m <= kRitzLds), or null
    const double *hist;        // a at 2i, b at 2i + 1
    __device__ double d(int i) const { return dg ? dg[i] : hist[2 * i]; }
    __device__ double e2(int i) const
    {
        if (o2)
            return o2[i];
        const double e = hist[2 * i - 1];
        return e * e;
    }
};

__device__ int negative_pivots(const TriView &t, int m, double x)
{
    const double floor_piv = 1e-290;
    double piv = t.d(0) - x;
    if (fabs(piv) < floor_piv)
        piv = -floor_piv;
    int neg = piv < 0.0;
    for (int i = 1; i < m; i++) {
        piv = (t.d(i) - x) - t.e2(i) * recip(piv);
        if (fabs(piv) < floor_piv)
            piv = -floor_piv;
        neg += piv < 0.0;
    }
    return neg;
}

// The same count at P points in one pass: the P pivot chains are independent,
// so they hide each other's latency.
template <int P>
__device__ void negative_pivots_p(const TriView &t, int m, const double *x, int *neg)
{
    const double floor_piv = 1e-290;
    double piv[P];
#pragma unroll
    for (int k = 0; k < P; k++) {
        piv[k] = t.d(0) - x[k];
        if (fabs(piv[k]) < floor_piv)
            piv[k] = -floor_piv;
        neg[k] = piv[k] < 0.0;
    }
    for (int i = 1; i < m; i++) {
        const double e2 = t.e2(i), d = t.d(i);
#pragma unroll
        for (int k = 0; k < P; k++) {
            piv[k] = (d - x[k]) - e2 * recip(piv[k]);
            if (fabs(piv[k]) < floor_piv)
                piv[k] = -floor_piv;
            neg[k] += piv[k] < 0.0;
        }
    }
}

// Lowest eigenvalue of T_m by multisection: the workgroup counts the
// eigenvalues below 2 * blockDim.x points of the bracket [lo, hi] (no
// eigenvalue below lo, at least one below hi), and the bracket shrinks to the
// two points around the first count above zero, until no double lies strictly
// inside it.  Returns hi, as the host's bisection does.  The bracket starts
// just below the previous step's value e_prev (by Cauchy interlacing the
// lowest eigenvalue of T_m is at most that of T_{m-1}), four times the last
// change wide, when two counts confirm it; otherwise it is the Gershgorin
// interval.  Either start ends at the same pair of doubles.
__device__ double lowest_eigenvalue(const TriView &t, int m, double e_prev, double e_prev2, double *sh, int *first)
{
    constexpr int P = 2;
    const int np = (int)blockDim.x * P;
    if (threadIdx.x < 2) {
        sh[4 + threadIdx.x] = NAN;
        if (m >= 3) {
            const double scale = fmax(1.0, fabs(e_prev));
            const double width = fmax(4.0 * fabs(e_prev - e_prev2), 1e-12 * scale);
            const double hi = e_prev + 4.0 * 0x1p-52 * scale;
            const double lo = e_prev - width;
            const int c = negative_pivots(t, m, threadIdx.x == 0 ? lo : hi);
            if (threadIdx.x == 0 ? c == 0 : c > 0)
                sh[4 + threadIdx.x] = threadIdx.x == 0 ? lo : hi;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!isnan(sh[4]) && !isnan(sh[5])) {
            sh[0] = sh[4];
            sh[1] = sh[5];
        } else {
            double lo = t.d(0), hi = t.d(0);
            for (int i = 0; i < m; i++) {
                const double rad = (i > 0 ? sqrt(t.e2(i)) : 0.0) + (i < m - 1 ? sqrt(t.e2(i + 1)) : 0.0);
                lo = fmin(lo, t.d(i) - rad);
                hi = fmax(hi, t.d(i) + rad);
            }
            const double pad = 0x1p-52 * (fabs(lo) + fabs(hi)) + 1e-290;
            sh[0] = lo - pad;
            sh[1] = hi + pad;
        }
        sh[2] = nextafter(sh[0], INFINITY) < sh[1] ? 0.0 : 1.0;
    }
    __syncthreads();
    for (int round = 0; round < 64 && sh[2] == 0.0; round++) {
        const double lo = sh[0], hi = sh[1];
        auto point = [&](int t) { return fmin(hi, fmax(lo, lo + (hi - lo) * ((double)(t + 1) / (double)(np + 1)))); };
        double x[P];
        int c[P];
#pragma unroll
        for (int k = 0; k < P; k++)
            x[k] = point((int)threadIdx.x * P + k);
        negative_pivots_p<P>(t, m, x, c);
        if (threadIdx.x == 0)
            *first = np;
        __syncthreads();
        int mine = np;
#pragma unroll
        for (int k = P - 1; k >= 0; k--)
            if (c[k] > 0)
                mine = (int)threadIdx.x * P + k;
        if (mine < np)
            atomicMin(first, mine);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int f = *first;
            const double nlo = f == 0 ? lo : point(f - 1);
            const double nhi = f == np ? hi : point(f);
            // done when a round changed nothing or no double is left strictly inside
            sh[2] = ((nlo == lo && nhi == hi) || !(nextafter(nlo, INFINITY) < nhi)) ? 1.0 : 0.0;
            sh[0] = nlo;
            sh[1] = nhi;
        }
        __syncthreads();
    }
    return sh[1];
}

// One workgroup per instance, beside step j's H.v: the end of step j - 1.
// b_j from the update partials, the Ritz value E_{j-1} of T_j (a_1..a_j,
// b_2..b_j), then the single-instance driver's stop tests in its order; the
// mailbox gets {a, b, E, code}.  A stop keeps every later kernel off the
// instance.
__device__ __forceinline__ void ritz_and_stop(const BatchInst &in, int j, double *__restrict__ mailbox)
{
    __shared__ double red[kThreads / 64];
    __shared__ double sh[6];
    __shared__ int first;
    BatchState *st = in.st;
    double *mb = mailbox + 4 * in.slot;
    if (st->stopped || j == 0) {
        if (threadIdx.x == 0) {
            mb[0] = mb[1] = mb[2] = 0.0;
            mb[3] = st->stopped ? kMailStopped : kMailNone;
        }
        return;
    }
    const int j0 = j - 1;  // the step finished here (0-based)
    const double b = sqrt(inst_sum(in.part2, in.nparts, red));
    const double a = in.hist[2 * j0];
    if (threadIdx.x == 0)
        in.hist[2 * j0 + 1] = b;
    __syncthreads();
    const int m = j0 + 1;
    double code = kMailRunning;
    double e = 0.0;
    if (!isfinite(a) || !isfinite(b)) {
        code = kMailBad;
    } else {
        __shared__ double dg[kRitzLds], o2[kRitzLds];
        TriView t{nullptr, nullptr, in.hist};
        if (m <= kRitzLds) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                dg[i] = in.hist[2 * i];
                const double o = i > 0 ? in.hist[2 * i - 1] : 0.0;
                o2[i] = o * o;
            }
            __syncthreads();
            t.dg = dg;
            t.o2 = o2;
        }
        e = lowest_eigenvalue(t, m, st->e_prev, st->e_prev2, sh, &first);
    }
    if (threadIdx.x == 0) {
        if (code == kMailRunning) {
            if (in.tol >= 0.0 && m >= 2 && fabs(e - st->e_prev) <= in.tol * fmax(1.0, fabs(e))) {
                code = HUBBARD_STOP_CONVERGED;
            } else {
                st->scale = fmax(st->scale, fabs(a) + (m > 1 ? in.hist[2 * j0 - 1] : 0.0));
                if (b == 0.0 || b <= 1e-12 * st->scale)
                    code = HUBBARD_STOP_BREAKDOWN;
                else if ((int64_t)m >= in.dim)
                    code = HUBBARD_STOP_EXHAUSTED;
                else if (m >= in.max_iter)
                    code = HUBBARD_STOP_MAXITER;
            }
        }
        st->e_prev2 = st->e_prev;
        st->e_prev = e;
        st->j = m;
        if (code != kMailRunning)
            st->stopped = 1;
        mb[0] = a;
        mb[1] = b;
        mb[2] = e;
        mb[3] = code;
    }
}

__global__ void batch_init_state_kernel(BatchState *st)
{
    if (threadIdx.x == 0) {
        for (int k = 0; k < 8; k++)
            st->S[k] = 0.0;
        st->S[0] = 1.0;
        st->S[1] = 1.0;
        st->scale = 0.0;
        st->e_prev = 0.0;
        st->e_prev2 = 0.0;
        st->j = 0;
        st->stopped = 0;
        st->cur = 0;
        st->pad_ = 0;
    }
}

}  // namespace

template <typename T>
void launch_batch_step(BatchInst *insts_dev, int n_inst, const BatchItem *items_dev, int n_items, size_t lds_bytes,
                       double *mailbox_dev, int k, hipStream_t s)
{
    auto hv = batch_hv_kernel<T>;
    if (lds_bytes > 64 * 1024)
        HUB_HIP(hipFuncSetAttribute((const void *)hv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    hipLaunchKernelGGL(hv, dim3(n_inst + n_items), dim3(kThreads), lds_bytes, s, insts_dev, items_dev, n_inst, k,
                       mailbox_dev);
    HUB_HIP(hipGetLastError());
    hipLaunchKernelGGL(batch_axpy_kernel<T>, dim3(n_items), dim3(kThreads), 0, s, insts_dev, items_dev, k);
    HUB_HIP(hipGetLastError());
}

template void launch_batch_step<double>(BatchInst *, int, const BatchItem *, int, size_t, double *, int,
                                         hipStream_t);
template void launch_batch_step<float>(BatchInst *, int, const BatchItem *, int, size_t, double *, int,
                                        hipStream_t);

void launch_batch_init_state(BatchState *st, hipStream_t s)
{
    hipLaunchKernelGGL(batch_init_state_kernel, dim3(1), dim3(64), 0, s, st);
    HUB_HIP(hipGetLastError());
}

}  // namespace hub
