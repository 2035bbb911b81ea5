// Real-time propagation psi <- exp(-i H dt) psi by the Lanczos recurrence of
// Sec. 2.2 (Alg. 1) run on a complex vector: H is real and symmetric, so with
// the Hermitian inner product the coefficients a_j, b_{j+1} are real and a
// complex vector is simply its real and imaginary halves side by side.  The
// Krylov basis stays resident in HBM: slot j of one allocation holds w_j =
// [re | im] in the padded row layout of the H.v (2 * npad doubles), and the
// device scalars sc[4j..4j+3] = {s_j = 1/|w_j|, 0, a_j, b_{j+1}} let every step
// launch without a host round trip (the H.v takes alpha = s_j, beta = 0).
#include <type_traits>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hub {

__device__ inline double prop_block_sum(double v, double *scratch)
{
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

static int prop_row_blocks(int64_t dim_up) { return (int)(dim_up < 4096 ? dim_up : 4096); }

// slot 0 = psi (dense J order -> padded rows, zero padding); partials of |psi|^2
__global__ __launch_bounds__(256) void prop_load_kernel(const double *__restrict__ re, const double *__restrict__ im,
                                                        double *__restrict__ slot, int64_t npad, int64_t dim_up,
                                                        int64_t dim_dn, int64_t ld, double *__restrict__ partials)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t r = blockIdx.x; r < dim_up; r += gridDim.x)
        for (int64_t d = threadIdx.x; d < ld; d += blockDim.x) {
            const bool in = d < dim_dn;
            const double vr = in ? re[r * dim_dn + d] : 0.0, vi = in ? im[r * dim_dn + d] : 0.0;
            slot[r * ld + d] = vr;
            slot[npad + r * ld + d] = vi;
            acc += vr * vr + vi * vi;
        }
    const double s = prop_block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

// y <- y - (a_j s_j) w_j - (b_j s_{j-1}) w_{j-1} over both halves (2 * npad
// doubles, padding included: it stays zero); partials of |y|^2
__global__ __launch_bounds__(256) void prop_update_kernel(double *__restrict__ y, const double *__restrict__ w,
                                                          const double *__restrict__ wp, const double *__restrict__ sc,
                                                          int j, int64_t n, double *__restrict__ partials)
{
    __shared__ double red[4];
    const double ca = sc[4 * j + 2] * sc[4 * j];
    const double cb = wp ? sc[4 * (j - 1) + 3] * sc[4 * (j - 1)] : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = y[i] - ca * w[i];
        if (wp)
            v -= cb * wp[i];
        y[i] = v;
        acc += v * v;
    }
    const double s = prop_block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

// psi = sum_{j < nv} gam_j w_j (complex gam_j = gam[2j] + i gam[2j+1]) into
// slot 0 (the next step's start; each element is read by its own thread before
// it is overwritten) and, after the last step (re, im not null), into the
// caller's dense halves; partials of |psi|^2.  PAIR: a thread takes two
// neighbouring elements of a row with 16-byte loads (even row stride; an odd
// row's last pair reaches into the row's zero padding, which stays zero).
template <bool PAIR>
__global__ __launch_bounds__(256) void prop_combine_kernel(double *__restrict__ basis, int nv, int64_t slot_stride,
                                                           int64_t npad, const double *__restrict__ gam,
                                                           double *__restrict__ re, double *__restrict__ im,
                                                           int64_t dim_up, int64_t dim_dn, int64_t ld,
                                                           double *__restrict__ partials)
{
    __shared__ double red[4];
    constexpr int E = PAIR ? 2 : 1;
    typedef typename std::conditional<PAIR, double2, double>::type V;
    double acc = 0.0;
    const int64_t nu = (dim_dn + E - 1) / E;
    for (int64_t r = blockIdx.x; r < dim_up; r += gridDim.x)
        for (int64_t q = threadIdx.x; q < nu; q += blockDim.x) {
            const int64_t d = q * E, k = r * ld + d;
            double pr[E] = {}, pi[E] = {};
#pragma unroll 4
            for (int j = 0; j < nv; j++) {
                const V vr = *reinterpret_cast<const V *>(basis + j * slot_stride + k);
                const V vi = *reinterpret_cast<const V *>(basis + j * slot_stride + npad + k);
                const double *wr = reinterpret_cast<const double *>(&vr), *wi = reinterpret_cast<const double *>(&vi);
                const double gr = gam[2 * j], gi = gam[2 * j + 1];
#pragma unroll
                for (int e = 0; e < E; e++) {
                    pr[e] += gr * wr[e] - gi * wi[e];
                    pi[e] += gr * wi[e] + gi * wr[e];
                }
            }
            V outr, outi;
            double *orr = reinterpret_cast<double *>(&outr), *oii = reinterpret_cast<double *>(&outi);
#pragma unroll
            for (int e = 0; e < E; e++) {
                orr[e] = pr[e];
                oii[e] = pi[e];
                acc += pr[e] * pr[e] + pi[e] * pi[e];
                if (re && d + e < dim_dn) {
                    re[r * dim_dn + d + e] = pr[e];
                    im[r * dim_dn + d + e] = pi[e];
                }
            }
            *reinterpret_cast<V *>(basis + k) = outr;
            *reinterpret_cast<V *>(basis + npad + k) = outi;
        }
    const double s = prop_block_sum(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

// PROP_START: s_0 = 1/sqrt(sum), beta slot 0.  PROP_DOT: a_j = s_j * sum.
// PROP_NORM: b_{j+1} = sqrt(sum), s_{j+1} = 1/b_{j+1} (0 when b vanishes).
// After a vanishing b the remaining steps of the round compute zeros or
// rounding noise, which the host leaves out of the combination.
__global__ __launch_bounds__(1024) void prop_reduce_kernel(const double *__restrict__ partials, int n, int mode,
                                                           double *__restrict__ sc, int j)
{
    __shared__ double red[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        acc += partials[i];
    const double s = prop_block_sum(acc, red);
    if (threadIdx.x != 0)
        return;
    // 1/b only above 1e-300: an overflow to infinity would leave a slot whose
    // old contents the next H.v multiplies by beta = 0 (giving NaN)
    if (mode == PROP_START) {
        const double b = sqrt(s);
        sc[0] = b > 1e-300 ? 1.0 / b : 0.0;
        sc[1] = 0.0;
    } else if (mode == PROP_DOT) {
        sc[4 * j + 2] = sc[4 * j] * s;
    } else {
        const double b = sqrt(s);
        sc[4 * j + 3] = b;
        sc[4 * (j + 1)] = b > 1e-300 ? 1.0 / b : 0.0;
        sc[4 * (j + 1) + 1] = 0.0;
    }
}

int launch_prop_load(const double *re, const double *im, double *slot, int64_t npad, int64_t dim_up, int64_t dim_dn,
                     int64_t ld, double *partials, hipStream_t s)
{
    const int nb = prop_row_blocks(dim_up);
    hipLaunchKernelGGL(prop_load_kernel, dim3(nb), dim3(256), 0, s, re, im, slot, npad, dim_up, dim_dn, ld, partials);
    HUB_HIP(hipGetLastError());
    return nb;
}

int launch_prop_update(double *y, const double *w, const double *wp, const double *sc, int j, int64_t n,
                       double *partials, hipStream_t s)
{
    const int nb = stream_blocks(n);
    hipLaunchKernelGGL(prop_update_kernel, dim3(nb), dim3(256), 0, s, y, w, wp, sc, j, n, partials);
    HUB_HIP(hipGetLastError());
    return nb;
}

int launch_prop_combine(double *basis, int nv, int64_t slot_stride, int64_t npad, const double *gam, double *re,
                        double *im, int64_t dim_up, int64_t dim_dn, int64_t ld, double *partials, hipStream_t s)
{
    const int nb = prop_row_blocks(dim_up);
    const bool pair = ld % 2 == 0 && npad % 2 == 0 && slot_stride % 2 == 0;
    if (pair)
        hipLaunchKernelGGL(prop_combine_kernel<true>, dim3(nb), dim3(256), 0, s, basis, nv, slot_stride, npad, gam, re,
                           im, dim_up, dim_dn, ld, partials);
    else
        hipLaunchKernelGGL(prop_combine_kernel<false>, dim3(nb), dim3(256), 0, s, basis, nv, slot_stride, npad, gam,
                           re, im, dim_up, dim_dn, ld, partials);
    HUB_HIP(hipGetLastError());
    return nb;
}

void launch_prop_reduce(const double *partials, int n, int mode, double *sc, int j, hipStream_t s)
{
    hipLaunchKernelGGL(prop_reduce_kernel, dim3(1), dim3(1024), 0, s, partials, n, mode, sc, j);
    HUB_HIP(hipGetLastError());
}

}  // namespace hub
