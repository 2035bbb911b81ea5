// HIP kernels for gfx950 (CDNA4): the Hubbard H.v product and the vector
// work of the Lanczos recurrence.
//
// H.v (Siro & Harju, Sec. 4.3).  The state vector x of dim = dim_up * dim_dn
// elements (J order, eq. J-formula) is viewed as a row-major dim_up x dim_dn
// matrix X: row r holds the amplitudes with up configuration r (the
// "subvectors" of Fig. slots).  Then
//     (H x)[r, d] = sum_k A_up[r, k] X[c_k(r), d]      (H_up (x) I: a combination of rows)
//                 + sum_k A_dn[d, k] X[r, e_k(d)]      (I (x) H_dn: a gather inside row r)
//                 + U popcount(up_r & dn_d) X[r, d]    (interaction, generated on the fly)
// with every hopping element equal to -t * sgn (Sec. 2.1).  One workgroup
// owns one row at a time: it stages X[r, :] in LDS (a row is at most 160 KB),
// reads the row's up-hopping entries as wave-uniform scalars, and each lane
// produces the outputs of its columns d.  The three terms run in one kernel,
// as the paper prescribes, so x is read from HBM once for the gathers.
//
// Every reduction (the dot products of Alg. 1) is written as one FP64 partial
// per workgroup and summed by a single workgroup in a fixed order, so a run is
// bitwise reproducible and a replayed recurrence retraces the first pass.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hub {

constexpr uint32_t kColMask = 0x7FFFFFFFu;

__device__ inline double block_sum(double v, double *scratch)
{
    // wave64 shuffle tree, then one value per wave through LDS
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; w++)
            s += scratch[w];
    }
    __syncthreads();
    return s;
}

struct HvParams {
    const uint32_t *__restrict__ states_up;
    const uint32_t *__restrict__ states_dn;
    const uint32_t *__restrict__ up_rows;
    const uint32_t *__restrict__ dn_cols;
    const uint16_t *__restrict__ nnz_up;
    const uint16_t *__restrict__ nnz_dn;
    int64_t dim_up, dim_dn;
    int32_t w_up, w_dn;
    double t, U;
    const double *__restrict__ tcls;
    int ncls;
};

// GT: per-bond amplitudes, entry = column | class << 24 | sign << 31 and the
// element is -tcls[class] * sgn; otherwise entry = column | sign << 31 and the
// element is -t * sgn.
template <typename T, int MODE, bool STAGE, bool GT>
__global__ __launch_bounds__(1024) void hv_kernel(HvParams p, const T *__restrict__ x, T *__restrict__ y,
                                                  double alpha, double beta, const double *__restrict__ coef,
                                                  double *__restrict__ partials)
{
    if (MODE == HV_LANCZOS) {
        alpha = coef[0];
        beta = coef[1];
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    __shared__ double red[16];
    // per-bond amplitudes of the classes, for the down-spin gathers (lanes read
    // different classes)
    __shared__ T amp[GT ? kMaxAmpClasses : 1];
    if (GT) {
        for (int c = threadIdx.x; c < p.ncls; c += blockDim.x)
            amp[c] = (T)p.tcls[c];
        __syncthreads();
    }

    const int64_t ddn = p.dim_dn;
    const T tp = (T)p.t, tm = (T)(-p.t), U = (T)p.U;
    const T a_s = (T)alpha, b_s = (T)beta;
    double acc0 = 0.0, acc1 = 0.0;

    for (int64_t r = blockIdx.x; r < p.dim_up; r += gridDim.x) {
        const T *__restrict__ xr = x + r * ddn;
        if (STAGE) {
            for (int64_t d = threadIdx.x; d < ddn; d += blockDim.x)
                xs[d] = xr[d];
            __syncthreads();
        }
        const uint32_t su = p.states_up[r];
        const int nu = p.nnz_up[r];
        const uint32_t *__restrict__ urow = p.up_rows + r * p.w_up;
        for (int64_t d = threadIdx.x; d < ddn; d += blockDim.x) {
            const T xv = STAGE ? xs[d] : xr[d];
            T h = U * (T)__popc(su & p.states_dn[d]) * xv;
            const int nd = p.nnz_dn[d];
            for (int k = 0; k < nd; k++) {
                const uint32_t e = p.dn_cols[(int64_t)k * ddn + d];
                if (GT) {
                    const uint32_t c = e & kClassColMask;
                    const T v = STAGE ? xs[c] : xr[c];
                    const T a = amp[(e >> 24) & 0x7Fu];
                    h = fma((e >> 31) ? a : -a, v, h);
                } else {
                    const T v = STAGE ? xs[e & kColMask] : xr[e & kColMask];
                    h = fma((e >> 31) ? tp : tm, v, h);
                }
            }
            // up-spin hops read other rows of x from memory: eight loads are
            // issued before their products are summed
            auto up_term = [&](uint32_t e, T v) {
                if (GT) {
                    const T a = amp[(e >> 24) & 0x7Fu];
                    return (e >> 31) ? a * v : -a * v;
                }
                return (e >> 31) ? tp * v : tm * v;
            };
            const uint32_t cmask = GT ? kClassColMask : kColMask;
            int k = 0;
            for (; k + 8 <= nu; k += 8) {
                uint32_t e[8];
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    e[u] = urow[k + u];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    v[u] = x[(int64_t)(e[u] & cmask) * ddn + d];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    h += up_term(e[u], v[u]);
            }
            for (; k < nu; k++) {
                const uint32_t e = urow[k];
                h += up_term(e, x[(int64_t)(e & cmask) * ddn + d]);
            }
            const int64_t J = r * ddn + d;
            if (MODE == HV_STORE) {
                y[J] = h;
            } else if (MODE == HV_LANCZOS) {
                const T q = a_s * h + b_s * y[J];
                y[J] = q;
                acc0 += (double)q * (double)xv;
            } else {
                const double res = (double)h - alpha * (double)xv;
                acc0 += res * res;
                acc1 += (double)xv * (double)h;
            }
        }
        if (STAGE)
            __syncthreads();
    }
    if (MODE != HV_STORE) {
        double s0 = block_sum(acc0, red);
        if (threadIdx.x == 0)
            partials[blockIdx.x] = s0;
        if (MODE == HV_RESIDUAL) {
            double s1 = block_sum(acc1, red);
            if (threadIdx.x == 0)
                partials[gridDim.x + blockIdx.x] = s1;
        }
    }
}

static HvParams to_params(const HvArgs &a)
{
    HvParams p;
    p.states_up = a.states_up;
    p.states_dn = a.states_dn;
    p.up_rows = a.up_rows;
    p.dn_cols = a.dn_cols;
    p.nnz_up = a.nnz_up;
    p.nnz_dn = a.nnz_dn;
    p.dim_up = a.dim_up;
    p.dim_dn = a.dim_dn;
    p.w_up = a.w_up;
    p.w_dn = a.w_dn;
    p.t = a.t;
    p.U = a.U;
    p.tcls = a.tcls;
    p.ncls = a.ncls;
    return p;
}

static int hv_threads(int64_t dim_dn)
{
    int64_t t = ((dim_dn + 63) / 64) * 64;
    return (int)(t < 1024 ? t : 1024);
}

// the row must fit in LDS beside the kernel's small static arrays (and the
// amplitude classes of a per-bond handle)
static bool hv_stage(const HvArgs &a, int elem_bytes)
{
    return a.dim_dn * elem_bytes <= 160 * 1024 - 512 - (a.tcls ? 1024 : 0);
}

int hv_blocks(const HvArgs &a, int elem_bytes)
{
    // every workgroup resident at once: LDS bounds how many fit on a CU
    const int64_t lds = hv_stage(a, elem_bytes) ? a.dim_dn * elem_bytes : 0;
    const int threads = hv_threads(a.dim_dn);
    int per_cu = 2048 / threads;
    if (lds > 0) {
        int by_lds = (int)((160 * 1024) / lds);
        per_cu = by_lds < per_cu ? by_lds : per_cu;
    }
    if (per_cu < 1)
        per_cu = 1;
    int64_t n = (int64_t)256 * per_cu;
    return (int)(a.dim_up < n ? a.dim_up : n);
}

template <typename T, int MODE>
static void launch_hv_mode(const HvArgs &a, const T *x, T *y, double alpha, double beta, const double *coef,
                           double *partials, int nblocks, hipStream_t s)
{
    const HvParams p = to_params(a);
    const int threads = hv_threads(a.dim_dn);
    const bool gt = a.tcls != nullptr;
    if (hv_stage(a, sizeof(T))) {
        const size_t lds = (size_t)a.dim_dn * sizeof(T);
        auto k = gt ? hv_kernel<T, MODE, true, true> : hv_kernel<T, MODE, true, false>;
        HUB_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k, dim3(nblocks), dim3(threads), lds, s, p, x, y, alpha, beta, coef, partials);
    } else {
        auto k = gt ? hv_kernel<T, MODE, false, true> : hv_kernel<T, MODE, false, false>;
        hipLaunchKernelGGL(k, dim3(nblocks), dim3(threads), 0, s, p, x, y, alpha, beta, coef, partials);
    }
    HUB_HIP(hipGetLastError());
}

template <typename T>
void launch_hv(const HvArgs &a, const T *x, T *y, int mode, double alpha, const double *coef, double *partials,
               int nblocks, hipStream_t s)
{
    if (mode == HV_STORE)
        launch_hv_mode<T, HV_STORE>(a, x, y, alpha, 0.0, coef, partials, nblocks, s);
    else if (mode == HV_LANCZOS)
        launch_hv_mode<T, HV_LANCZOS>(a, x, y, alpha, 0.0, coef, partials, nblocks, s);
    else
        launch_hv_mode<T, HV_RESIDUAL>(a, x, y, alpha, 0.0, coef, partials, nblocks, s);
}

template void launch_hv<double>(const HvArgs &, const double *, double *, int, double, const double *, double *,
                                int, hipStream_t);
template void launch_hv<float>(const HvArgs &, const float *, float *, int, double, const double *, double *, int,
                               hipStream_t);

// ------------------------------------------------------------ vector kernels

int stream_blocks(int64_t n)
{
    int64_t b = (n + 2047) / 2048;
    if (b > 2048)
        b = 2048;
    return (int)(b < 1 ? 1 : b);
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// q = q - c f with c from the device scalars; partial sums of q.q (Alg. 1:
// q_j <- q_j - a_j f_j, then the norm that becomes b_{j+1}).
template <typename T>
__global__ __launch_bounds__(256) void axpy_norm_kernel(T *__restrict__ w, const T *__restrict__ v,
                                                        const double *__restrict__ coef, int64_t n,
                                                        double *__restrict__ partials)
{
    __shared__ double red[4];
    const T cs = (T)coef[0];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        const T q = w[i] - cs * v[i];
        w[i] = q;
        acc += (double)q * (double)q;
    }
    double s = block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

template <typename T>
void launch_axpy_norm(T *w, const T *v, const double *coef, int64_t n, double *partials, int nblocks,
                      hipStream_t s)
{
    hipLaunchKernelGGL(axpy_norm_kernel<T>, dim3(nblocks), dim3(256), 0, s, w, v, coef, n, partials);
    HUB_HIP(hipGetLastError());
}
template void launch_axpy_norm<double>(double *, const double *, const double *, int64_t, double *, int,
                                       hipStream_t);
template void launch_axpy_norm<float>(float *, const float *, const double *, int64_t, double *, int, hipStream_t);

// Fix-up of a fused step whose expanded norm was flagged as inaccurate
// (S[kFixFlag] set by the RED_FUSED reduction): w <- w - S[3] v, the next
// vector formed explicitly, and partial sums of its squared norm.  A no-op
// (every workgroup returns at once) when the flag is clear.
template <typename T>
__global__ __launch_bounds__(256) void fused_fix_kernel(T *__restrict__ w, const T *__restrict__ v,
                                                        const double *__restrict__ S, int64_t n,
                                                        double *__restrict__ partials)
{
    if (S[kFixFlag] == 0.0)
        return;
    __shared__ double red[4];
    const T cs = (T)S[3];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        const T q = w[i] - cs * v[i];
        w[i] = q;
        acc += (double)q * (double)q;
    }
    double s = block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

template <typename T>
void launch_fused_fix(T *w, const T *v, const double *S, int64_t n, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(fused_fix_kernel<T>, dim3(nblocks), dim3(256), 0, s, w, v, S, n, partials);
    HUB_HIP(hipGetLastError());
}
template void launch_fused_fix<double>(double *, const double *, const double *, int64_t, double *, int, hipStream_t);
template void launch_fused_fix<float>(float *, const float *, const double *, int64_t, double *, int, hipStream_t);

// The same fix-up for a fused deflated step: w <- w - S[3] v - sum_l S[8 + l]
// psi_l (in FP64, rounded once), rows of w and v at stride ld, psi dense;
// partial sums of the new vector's squared norm.
template <typename T>
__global__ __launch_bounds__(256) void fused_fix_defl_kernel(T *__restrict__ w, const T *__restrict__ v,
                                                             const double *__restrict__ S,
                                                             const double *__restrict__ psi, int nd, int64_t pdim,
                                                             int64_t dim_up, int64_t dim_dn, int64_t ld,
                                                             double *__restrict__ partials)
{
    if (S[kFixFlag] == 0.0)
        return;
    __shared__ double red[4];
    const double cs = S[3];
    double g[kMaxDeflate];
    for (int l = 0; l < nd; l++)
        g[l] = S[8 + l];
    double acc = 0.0;
    const int64_t n = dim_up * dim_dn;
    GRID_STRIDE(i, n)
    {
        const int64_t r = i / dim_dn, d = i - r * dim_dn;
        double x = (double)(w[r * ld + d] - (T)cs * v[r * ld + d]);
        for (int l = 0; l < nd; l++)
            x -= g[l] * psi[(int64_t)l * pdim + i];
        const T q = (T)x;
        w[r * ld + d] = q;
        acc += (double)q * (double)q;
    }
    double s = block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

template <typename T>
int launch_fused_fix_defl(T *w, const T *v, const double *S, const double *psi, int nd, int64_t pdim, int64_t dim_up,
                          int64_t dim_dn, int64_t ld, double *partials, hipStream_t s)
{
    const int nb = stream_blocks(dim_up * dim_dn);
    hipLaunchKernelGGL(fused_fix_defl_kernel<T>, dim3(nb), dim3(256), 0, s, w, v, S, psi, nd, pdim, dim_up, dim_dn, ld,
                       partials);
    HUB_HIP(hipGetLastError());
    return nb;
}
template int launch_fused_fix_defl<double>(double *, const double *, const double *, const double *, int, int64_t,
                                           int64_t, int64_t, int64_t, double *, hipStream_t);
template int launch_fused_fix_defl<float>(float *, const float *, const double *, const double *, int, int64_t,
                                          int64_t, int64_t, int64_t, double *, hipStream_t);

// SplitMix64 (Steele, Lea & Flood 2014): output k of the stream started at
// `seed` is the published finaliser applied to seed + k * 0x9E3779B97F4A7C15.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Element J of the random start vector: 2u - 1 with u = top 53 bits / 2^53.
__device__ inline double start_value(uint64_t seed, int64_t J)
{
    const double u = (double)(splitmix64_at(seed, (uint64_t)J + 1) >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

__device__ inline double start_or_given(const double *__restrict__ given, uint64_t seed, int64_t J)
{
    return given ? given[J] : start_value(seed, J);
}

__global__ __launch_bounds__(256) void start_raw_kernel(uint64_t seed, double *__restrict__ f, int64_t n)
{
    GRID_STRIDE(i, n) f[i] = start_value(seed, i);
}

void launch_start_raw(uint64_t seed, double *f, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(start_raw_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, seed, f, n);
    HUB_HIP(hipGetLastError());
}

// partial sums of f.f for the start vector (given, or generated from the seed)
__global__ __launch_bounds__(256) void start_norm2_kernel(const double *__restrict__ given, uint64_t seed, int64_t n,
                                                          double *__restrict__ partials)
{
    __shared__ double red[4];
    double acc = 0.0;
    GRID_STRIDE(i, n)
    {
        const double f = start_or_given(given, seed, i);
        acc += f * f;
    }
    double s = block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

void launch_start_norm2(const double *given, uint64_t seed, int64_t n, double *partials, int nblocks,
                        hipStream_t s)
{
    hipLaunchKernelGGL(start_norm2_kernel, dim3(nblocks), dim3(256), 0, s, given, seed, n, partials);
    HUB_HIP(hipGetLastError());
}

// Row-major fills between the dense J order and the padded internal layout.
#define ROW_LOOP(r, d, dim_up, width)                                                        \
    for (int64_t r = blockIdx.x; r < (dim_up); r += gridDim.x)                               \
        for (int64_t d = threadIdx.x; d < (width); d += blockDim.x)

static int row_blocks(int64_t dim_up) { return (int)(dim_up < 4096 ? dim_up : 4096); }

// out = (T)(c f), the normalised start vector f_1 in the working precision and
// layout (zero in the row padding); zero = the previous vector f_0 = 0 (Alg. 1).
template <typename T>
__global__ __launch_bounds__(256) void start_fill_kernel(const double *__restrict__ given, uint64_t seed, double c,
                                                         T *__restrict__ out, T *__restrict__ zero, int64_t dim_up,
                                                         int64_t dim_dn, int64_t ld)
{
    ROW_LOOP(r, d, dim_up, ld)
    {
        const T v = d < dim_dn ? (T)(c * start_or_given(given, seed, r * dim_dn + d)) : (T)0;
        out[r * ld + d] = v;
        if (zero)
            zero[r * ld + d] = (T)0;
    }
}

template <typename T>
void launch_start_fill(const double *given, uint64_t seed, double c, T *out, T *zero, int64_t dim_up, int64_t dim_dn,
                       int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(start_fill_kernel<T>, dim3(row_blocks(dim_up)), dim3(256), 0, s, given, seed, c, out, zero,
                       dim_up, dim_dn, ld);
    HUB_HIP(hipGetLastError());
}
template void launch_start_fill<double>(const double *, uint64_t, double, double *, double *, int64_t, int64_t,
                                        int64_t, hipStream_t);
template void launch_start_fill<float>(const double *, uint64_t, double, float *, float *, int64_t, int64_t, int64_t,
                                       hipStream_t);

// ------------------------------------------------------------ deflation
// The lower eigenvectors psi_0..psi_{nd-1} (FP64, dense J order, psi_l at
// psi + l * dim) are projected out of every new Lanczos vector, so the
// recurrence runs with P H P, P = 1 - sum_l psi_l psi_l^T, and its lowest Ritz
// value approaches the next eigenvalue (Sec. 2.2: the lowest excited states).
// Vectors in the internal layout are dim_up rows of dim_dn elements at stride
// ld; the padding is left alone (it stays zero).

// Optionally q = q - c v first (c = coef[0]: the q - a_j f_j update of Alg. 1),
// then partial sums of psi_l . q for l < nd, stored at partials[l * grid + block].
template <typename T>
__global__ __launch_bounds__(256) void defl_dots_kernel(T *__restrict__ q, const T *__restrict__ v,
                                                        const double *__restrict__ coef,
                                                        const double *__restrict__ psi, int nd, int64_t dim,
                                                        int64_t dim_up, int64_t dim_dn, int64_t ld,
                                                        double *__restrict__ partials)
{
    __shared__ double red[4];
    double acc[kMaxDeflate];
#pragma unroll
    for (int l = 0; l < kMaxDeflate; l++)
        acc[l] = 0.0;
    const T cs = v ? (T)coef[0] : (T)0;
    ROW_LOOP(r, d, dim_up, dim_dn)
    {
        T x = q[r * ld + d];
        if (v) {
            x = x - cs * v[r * ld + d];
            q[r * ld + d] = x;
        }
        const double xd = (double)x;
        const double *p = psi + r * dim_dn + d;
#pragma unroll
        for (int l = 0; l < kMaxDeflate; l++)
            if (l < nd)
                acc[l] += xd * p[l * dim];
    }
    for (int l = 0; l < nd; l++) {
        const double sl = block_sum(acc[l], red);
        if (threadIdx.x == 0)
            partials[(int64_t)l * gridDim.x + blockIdx.x] = sl;
    }
}

// q = q - sum_l D[l] psi_l (rounded once to T), and partial sums of q.q.
template <typename T>
__global__ __launch_bounds__(256) void defl_update_kernel(T *__restrict__ q, const double *__restrict__ psi,
                                                          const double *__restrict__ D, int nd, int64_t dim,
                                                          int64_t dim_up, int64_t dim_dn, int64_t ld,
                                                          double *__restrict__ partials)
{
    __shared__ double red[4];
    double c[kMaxDeflate];
#pragma unroll
    for (int l = 0; l < kMaxDeflate; l++)
        c[l] = l < nd ? D[l] : 0.0;
    double acc = 0.0;
    ROW_LOOP(r, d, dim_up, dim_dn)
    {
        double x = (double)q[r * ld + d];
        const double *p = psi + r * dim_dn + d;
#pragma unroll
        for (int l = 0; l < kMaxDeflate; l++)
            if (l < nd)
                x -= c[l] * p[l * dim];
        const T xt = (T)x;
        q[r * ld + d] = xt;
        acc += (double)xt * (double)xt;
    }
    const double sq = block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = sq;
}

template <typename T>
int launch_defl_dots(T *q, const T *v, const double *coef, const double *psi, int nd, int64_t dim, int64_t dim_up,
                     int64_t dim_dn, int64_t ld, double *partials, hipStream_t s)
{
    const int nb = row_blocks(dim_up);
    hipLaunchKernelGGL(defl_dots_kernel<T>, dim3(nb), dim3(256), 0, s, q, v, coef, psi, nd, dim, dim_up, dim_dn, ld,
                       partials);
    HUB_HIP(hipGetLastError());
    return nb;
}

template <typename T>
int launch_defl_update(T *q, const double *psi, const double *D, int nd, int64_t dim, int64_t dim_up, int64_t dim_dn,
                       int64_t ld, double *partials, hipStream_t s)
{
    const int nb = row_blocks(dim_up);
    hipLaunchKernelGGL(defl_update_kernel<T>, dim3(nb), dim3(256), 0, s, q, psi, D, nd, dim, dim_up, dim_dn, ld,
                       partials);
    HUB_HIP(hipGetLastError());
    return nb;
}
template int launch_defl_dots<double>(double *, const double *, const double *, const double *, int, int64_t, int64_t,
                                      int64_t, int64_t, double *, hipStream_t);
template int launch_defl_dots<float>(float *, const float *, const double *, const double *, int, int64_t, int64_t,
                                     int64_t, int64_t, double *, hipStream_t);
template int launch_defl_update<double>(double *, const double *, const double *, int, int64_t, int64_t, int64_t,
                                        int64_t, double *, hipStream_t);
template int launch_defl_update<float>(float *, const double *, const double *, int, int64_t, int64_t, int64_t,
                                       int64_t, double *, hipStream_t);

int defl_blocks(int64_t dim_up) { return row_blocks(dim_up); }

// psi += y_j * (1/s) * v, where v holds s f_j and 1/s is the device scalar
// coef[0] (the ground-state vector sum_j y_j f_j of the replayed recurrence).
template <typename T>
__global__ __launch_bounds__(256) void psi_acc_kernel(double *__restrict__ psi, const T *__restrict__ v, double yj,
                                                      const double *__restrict__ coef, int64_t dim_up, int64_t dim_dn,
                                                      int64_t ld, int first)
{
    const double c = yj * coef[0];
    ROW_LOOP(r, d, dim_up, dim_dn)
    {
        const double add = c * (double)v[r * ld + d];
        double *p = psi + r * dim_dn + d;
        *p = first ? add : *p + add;
    }
}

template <typename T>
void launch_psi_acc(double *psi, const T *v, double yj, const double *coef, int64_t dim_up, int64_t dim_dn, int64_t ld,
                    bool first, hipStream_t s)
{
    hipLaunchKernelGGL(psi_acc_kernel<T>, dim3(row_blocks(dim_up)), dim3(256), 0, s, psi, v, yj, coef, dim_up, dim_dn,
                       ld, first ? 1 : 0);
    HUB_HIP(hipGetLastError());
}
template void launch_psi_acc<double>(double *, const double *, double, const double *, int64_t, int64_t, int64_t, bool,
                                     hipStream_t);
template void launch_psi_acc<float>(double *, const float *, double, const double *, int64_t, int64_t, int64_t, bool,
                                    hipStream_t);

// psi = sum_j y_j (1/s_j) v_j over the resident Lanczos vectors, summed in the
// order of the replayed accumulation
template <typename T>
__global__ __launch_bounds__(256) void psi_combine_kernel(double *__restrict__ psi, const T *const *__restrict__ vecs,
                                                          const double *__restrict__ y,
                                                          const double *__restrict__ scale, int m, int64_t dim_up,
                                                          int64_t dim_dn, int64_t ld)
{
    ROW_LOOP(r, d, dim_up, dim_dn)
    {
        double acc = 0.0;
#pragma unroll 8
        for (int j = 0; j < m; j++)
            acc += (y[j] * scale[j]) * (double)vecs[j][r * ld + d];
        psi[r * dim_dn + d] = acc;
    }
}

template <typename T>
void launch_psi_combine(double *psi, const T *const *vecs, const double *y, const double *scale, int m, int64_t dim_up,
                        int64_t dim_dn, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(psi_combine_kernel<T>, dim3(row_blocks(dim_up)), dim3(256), 0, s, psi, vecs, y, scale, m,
                       dim_up, dim_dn, ld);
    HUB_HIP(hipGetLastError());
}
template void launch_psi_combine<double>(double *, const double *const *, const double *, const double *, int, int64_t,
                                         int64_t, int64_t, hipStream_t);
template void launch_psi_combine<float>(double *, const float *const *, const double *, const double *, int, int64_t,
                                        int64_t, int64_t, hipStream_t);

// partial sums of psi.psi and psi.f1
__global__ __launch_bounds__(256) void psi_stats_kernel(const double *__restrict__ psi, const double *__restrict__ given,
                                                        uint64_t seed, int64_t n, double *__restrict__ partials)
{
    __shared__ double red[4];
    double a0 = 0.0, a1 = 0.0;
    GRID_STRIDE(i, n)
    {
        const double v = psi[i];
        a0 += v * v;
        a1 += v * start_or_given(given, seed, i);
    }
    double s0 = block_sum(a0, red);
    double s1 = block_sum(a1, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s0;
        partials[gridDim.x + blockIdx.x] = s1;
    }
}

void launch_psi_stats(const double *psi, const double *given, uint64_t seed, int64_t n, double *partials, int nblocks,
                      hipStream_t s)
{
    hipLaunchKernelGGL(psi_stats_kernel, dim3(nblocks), dim3(256), 0, s, psi, given, seed, n, partials);
    HUB_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void scale_kernel(double *__restrict__ v, double c, int64_t n)
{
    GRID_STRIDE(i, n) v[i] *= c;
}

void launch_scale(double *v, double c, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(scale_kernel, dim3(stream_blocks(n)), dim3(256), 0, s, v, c, n);
    HUB_HIP(hipGetLastError());
}

// Fixed-order sum of `n` partials (block k sums partials[k*stride ...]).
// mode RED_PLAIN: out[k] = sum.
// mode RED_DOT (after the H.v step of iteration j): a_j = sum * S[0];
//   S[3] = a_j * S[0] (the coefficient of the q - a_j f_j update); hist[2j] = a_j.
// mode RED_NORM (after that update): b_{j+1} = sqrt(sum); hist[2j+1] = b_{j+1};
//   the roles of the two vectors swap, so the next H.v gets
//   alpha = 1/b_{j+1}, beta = -b_{j+1} * S[0] (old 1/s), and S[0] = 1/b_{j+1}.
// mode RED_START (after the start vector was projected): S = {1/s, 1/s, 0, 0}
//   with s = sqrt(sum), the norm of the stored start vector.
// mode RED_FUSED (after a fused step, partials [3][n] = shares of y.x, y.y,
//   x.x with x = X_j, the stored vector of norm s, and y = H X_j / s - b_j v_{j-1}):
//   a_j = (y.x) / s, c = a_j / s, and the norm of the next vector
//   X_{j+1} = y - c X_j, which the next step forms, is expanded as
//   |y|^2 - 2 c (y.x) + c^2 |X_j|^2.  The expansion loses the digits of b_{j+1}
//   that cancel against |y|: when it falls below kFixRatio |y|^2 the step is
//   flagged (S[kFixFlag] = 1, the old 1/s kept in S[kFixScale]) and b_{j+1}
//   is left to RED_FIX.
//   A fused deflated step (stride = nd lower vectors, partials [3 + 2l][n] =
//   shares of psi_l.y and [4 + 2l][n] of psi_l.x) projects the next vector,
//   X_{j+1} = y - c X_j - sum_l g_l psi_l with g_l = psi_l.y - c psi_l.x
//   (S[8 + l]), and subtracts sum_l g_l^2 from the expanded norm.
// mode RED_FIX (after fused_fix_kernel, only when the step was flagged):
//   b_{j+1} = |X_{j+1}| from the explicit vector; c = 0 and g = 0, so the
//   next step's row pass keeps X_{j+1} as it is; the flag is cleared.
// S = device scalars {1/s of the current vector, alpha, beta, c, -, -, flag,
// 1/s kept, g_0 .. g_{nd-1}}; RED_START also clears g.
__global__ __launch_bounds__(1024) void reduce_kernel(const double *__restrict__ partials, int n, int stride,
                                                      double *__restrict__ out, int mode, double *__restrict__ S,
                                                      double *__restrict__ hist, int j)
{
    __shared__ double red[16];
    const double *src = partials + (int64_t)blockIdx.x * stride;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        acc += src[i];
    if (mode == RED_FIX && S[kFixFlag] == 0.0)
        return;
    double s = block_sum(acc, red);
    if (mode == RED_FUSED) {
        double acc1 = 0.0, acc2 = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            acc1 += src[n + i];
            acc2 += src[2 * n + i];
        }
        const double qq = block_sum(acc1, red);
        const double xx = block_sum(acc2, red);
        const int nd = stride;  // lower vectors of a deflated step
        double pu[kMaxDeflate], px[kMaxDeflate];
        for (int l = 0; l < nd && l < kMaxDeflate; l++) {
            double au = 0.0, ax = 0.0;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                au += src[(3 + 2 * l) * n + i];
                ax += src[(4 + 2 * l) * n + i];
            }
            pu[l] = block_sum(au, red);
            px[l] = block_sum(ax, red);
        }
        if (threadIdx.x == 0) {
            const double a = s * S[0];
            const double c = a * S[0];
            double b2 = qq - 2.0 * c * s + c * c * xx;
            for (int l = 0; l < nd && l < kMaxDeflate; l++) {
                const double g = pu[l] - c * px[l];
                S[8 + l] = g;
                b2 -= g * g;
            }
            hist[2 * j] = a;
            S[3] = c;
            if (b2 >= kFixRatio * qq) {
                const double b = sqrt(b2);
                hist[2 * j + 1] = b;
                S[2] = -b * S[0];
                S[0] = 1.0 / b;
                S[1] = S[0];
                S[kFixFlag] = 0.0;
            } else {
                S[kFixScale] = S[0];
                S[kFixFlag] = 1.0;
            }
        }
        return;
    }
    if (mode == RED_FIX) {
        if (threadIdx.x == 0) {
            const double b = sqrt(s);
            hist[2 * j + 1] = b;
            S[2] = -b * S[kFixScale];
            S[0] = b > 0.0 ? 1.0 / b : 0.0;
            S[1] = S[0];
            S[3] = 0.0;
            for (int l = 0; l < kMaxDeflate; l++)
                S[8 + l] = 0.0;
            S[kFixFlag] = 0.0;
        }
        return;
    }
    if (threadIdx.x == 0) {
        if (mode == RED_PLAIN) {
            out[blockIdx.x] = s;
        } else if (mode == RED_DOT) {
            const double a = s * S[0];
            S[3] = a * S[0];
            hist[2 * j] = a;
        } else if (mode == RED_START) {
            const double b = sqrt(s);
            S[0] = b > 0.0 ? 1.0 / b : 0.0;
            S[1] = S[0];
            S[2] = 0.0;
            S[3] = 0.0;
            for (int l = 0; l < kMaxDeflate; l++)
                S[8 + l] = 0.0;
        } else {
            const double b = sqrt(s);
            hist[2 * j + 1] = b;
            S[2] = -b * S[0];
            S[0] = b > 0.0 ? 1.0 / b : 0.0;
            S[1] = S[0];
        }
    }
}

void launch_reduce(const double *partials, int n, int stride, int count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(count), dim3(1024), 0, s, partials, n, stride, out, (int)RED_PLAIN,
                       (double *)nullptr, (double *)nullptr, 0);
    HUB_HIP(hipGetLastError());
}

void launch_reduce_step(const double *partials, int n, int mode, double *S, double *hist, int j, hipStream_t s,
                        int nd)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, partials, n, nd, (double *)nullptr, mode, S, hist,
                       j);
    HUB_HIP(hipGetLastError());
}

// S = {1, 1, 0, 0}: f_1 has scale 1 and b_1 = 0 (Alg. 1).
__global__ void init_scalars_kernel(double *S)
{
    if (threadIdx.x == 0) {
        S[0] = 1.0;
        S[1] = 1.0;
        S[2] = 0.0;
        S[3] = 0.0;
        S[kFixFlag] = 0.0;
    }
}

void launch_init_scalars(double *S, hipStream_t s)
{
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, S);
    HUB_HIP(hipGetLastError());
}

}  // namespace hub
