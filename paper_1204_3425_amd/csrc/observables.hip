// Site observables of a state: the occupations n_{i sigma} and their products,
// which are diagonal in the configuration basis (Sec. 1, eq. H; Sec. 2.1: bit i
// of a spin's configuration word is the occupation of site i).
//
// With w_J = psi_J^2 over the dim_up x dim_dn view of psi (J = r * dim_dn + d),
//   UU[i][j] = sum_J w_J bit_i(up_r) bit_j(up_r)     <n_{i up} n_{j up}>
//   DD[i][j] = sum_J w_J bit_i(dn_d) bit_j(dn_d)     <n_{i dn} n_{j dn}>
//   C[i][j]  = sum_J w_J bit_i(up_r) bit_j(dn_d)     <n_{i up} n_{j dn}>
//   norm     = sum_J w_J
// (unnormalised).  One pass reads psi once.  A workgroup of TW threads takes a
// tile of 2 TW down configurations (two per thread) and a strided set of up rows.
// Each thread sums, over those rows, w into q(x) and into A_i(x) for every site i
// occupied in the row's up configuration (a branch that is uniform across the
// workgroup, N_up adds per element).  Per row, the wave's total R of w is formed
// by a butterfly and lane j adds bit_i(up_r) bit_j(up_r) R into column j of UU.
// At the end the workgroup writes A and q to LDS and forms, one (i, j) pair per
// thread, C[i][j] = sum_x A_i(x) bit_j(dn_x) and DD[i][j] = sum_x q(x) bit_i(dn_x)
// bit_j(dn_x) over its tile.  Every workgroup writes one partial of
// 3 * NS * NS + 1 values; a second kernel sums the partials in a fixed order,
// so the result is reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

// wave-wide sum from the ROCm device library (DPP reduction, every lane gets it)
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);

namespace hub {

template <int NS>
constexpr int obs_partial_size()
{
    return 3 * NS * NS + 1;
}

// workgroup width; each thread takes kObsSlots down configurations, so a tile
// is kObsSlots * TW wide.  The LDS image of A (NS x TW doubles, one slot at a
// time) stays within 64 KB.
constexpr int kObsSlots = 2;
template <int NS>
constexpr int obs_threads()
{
    return NS <= 16 ? 256 : 128;
}

template <int NS, int TW>
__global__ __launch_bounds__(TW) void obs_accumulate_kernel(const double *__restrict__ psi,
                                                            const uint32_t *__restrict__ states_up,
                                                            const uint32_t *__restrict__ states_dn, int ns,
                                                            int64_t dim_up, int64_t dim_dn, int ntiles, int nchunks,
                                                            double *__restrict__ part)
{
    constexpr int NW = TW / 64, SL = kObsSlots;
    __shared__ double a_lds[NS][TW];
    __shared__ double q_lds[TW];
    __shared__ uint32_t dn_lds[TW];
    __shared__ double uu_lds[NS][NS];
    __shared__ double nw[NW];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int tile = blockIdx.x % ntiles, chunk = blockIdx.x / ntiles;
    int64_t x[SL];
    bool have[SL];
#pragma unroll
    for (int s = 0; s < SL; s++) {
        x[s] = ((int64_t)tile * SL + s) * TW + t;  // this thread's down configurations
        have[s] = x[s] < dim_dn;
    }

    double A[SL][NS], UU[NS], q[SL];
#pragma unroll
    for (int i = 0; i < NS; i++) {
        UU[i] = 0.0;
#pragma unroll
        for (int s = 0; s < SL; s++)
            A[s][i] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < SL; s++)
        q[s] = 0.0;
    double norm = 0.0;
    // lane j < ns keeps column j of UU; its own occupation as 0 or 1
    const double lbit = lane < ns ? 1.0 : 0.0;
    const int lsite = lane & 31;
    auto row_step = [&](uint32_t up, const double *w) {
        double R = 0.0;
#pragma unroll
        for (int s = 0; s < SL; s++) {
            q[s] += w[s];
            R += w[s];
        }
        // the up word is the same for the whole workgroup: its bits become 0/1
        // factors instead of branches
#pragma unroll
        for (int i = 0; i < NS; i++) {
            const double b = (double)((up >> i) & 1u);
#pragma unroll
            for (int s = 0; s < SL; s++)
                A[s][i] = fma(b, w[s], A[s][i]);
        }
        R = __ockl_wfred_add_f64(R);  // the wave's total of the row
        norm += R;
        const double mine = lbit * (double)((up >> lsite) & 1u) * R;
#pragma unroll
        for (int i = 0; i < NS; i++)
            UU[i] = fma((double)((up >> i) & 1u), mine, UU[i]);
    };
    // a contiguous range of rows (neighbouring rows share address-translation
    // pages); four rows per round, the next round's loads issued before this
    // round's arithmetic
    const int64_t rpb = (dim_up + nchunks - 1) / nchunks;
    const int64_t rbeg = chunk * rpb, rend = rbeg + rpb < dim_up ? rbeg + rpb : dim_up;
    auto load = [&](int64_t r0, double (*v)[SL]) {
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int s = 0; s < SL; s++) {
                const int64_t r = r0 + k;
                v[k][s] = (have[s] && r < rend) ? psi[r * dim_dn + x[s]] : 0.0;
            }
    };
    double v[4][SL], vn[4][SL];
    int64_t r = rbeg;
    if (r < rend)
        load(r, v);
    for (; r < rend; r += 4) {
        if (r + 4 < rend)
            load(r + 4, vn);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int64_t rk = r + k;
            if (rk < rend) {
                double w[SL];
#pragma unroll
                for (int s = 0; s < SL; s++)
                    w[s] = v[k][s] * v[k][s];
                row_step(states_up[rk], w);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int s = 0; s < SL; s++)
                v[k][s] = vn[k][s];
    }

    if (lane == 0)
        nw[wave] = norm;
    // the waves' UU columns, summed through LDS one wave at a time
    for (int k = 0; k < NW; k++) {
        if (wave == k && lane < NS) {
#pragma unroll
            for (int i = 0; i < NS; i++) {
                const double u = lane < ns ? UU[i] : 0.0;
                uu_lds[i][lane] = k == 0 ? u : uu_lds[i][lane] + u;
            }
        }
        __syncthreads();
    }
    // C and DD over the tile, one slot's TW configurations at a time
    double c[(NS * NS + TW - 1) / TW], dd[(NS * NS + TW - 1) / TW];
#pragma unroll
    for (int k = 0; k < (NS * NS + TW - 1) / TW; k++) {
        c[k] = 0.0;
        dd[k] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < SL; s++) {
#pragma unroll
        for (int i = 0; i < NS; i++)
            a_lds[i][t] = A[s][i];
        q_lds[t] = q[s];
        dn_lds[t] = have[s] ? states_dn[x[s]] : 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < (NS * NS + TW - 1) / TW; k++) {
            const int e = t + k * TW;
            const int i = e / NS, j = e % NS;
            if (e < NS * NS && i < ns && j < ns) {
                const uint32_t bj = 1u << j, mask = (1u << i) | bj;
                for (int y = 0; y < TW; y++) {
                    const uint32_t b = dn_lds[y];
                    c[k] += (b & bj) ? a_lds[i][y] : 0.0;
                    dd[k] += (b & mask) == mask ? q_lds[y] : 0.0;
                }
            }
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.x * obs_partial_size<NS>();
#pragma unroll
    for (int k = 0; k < (NS * NS + TW - 1) / TW; k++) {
        const int e = t + k * TW;
        if (e < NS * NS) {
            out[e] = uu_lds[e / NS][e % NS];
            out[NS * NS + e] = dd[k];
            out[2 * NS * NS + e] = c[k];
        }
    }
    if (t == 0) {
        double n = 0.0;
        for (int k = 0; k < NW; k++)
            n += nw[k];
        out[3 * NS * NS] = n;
    }
}

// Sum of the per-workgroup partials in two fixed-order levels: group g of
// kObsGroups adds partials [g * nparts / G, (g + 1) * nparts / G) of element e
// into grp[g][e]; then out[e] adds the groups in order.
constexpr int kObsGroups = 32;

__global__ __launch_bounds__(256) void obs_sum_kernel(const double *__restrict__ part, int nparts, int psize,
                                                      double *__restrict__ grp)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= psize)
        return;
    const int b0 = (int)((int64_t)g * nparts / kObsGroups), b1 = (int)((int64_t)(g + 1) * nparts / kObsGroups);
    double s = 0.0;
    for (int b = b0; b < b1; b++)
        s += part[(int64_t)b * psize + e];
    grp[(int64_t)g * psize + e] = s;
}

__global__ __launch_bounds__(256) void obs_sum_groups_kernel(const double *__restrict__ grp, int psize,
                                                             double *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= psize)
        return;
    double s = 0.0;
    for (int g = 0; g < kObsGroups; g++)
        s += grp[(int64_t)g * psize + e];
    out[e] = s;
}

int obs_ns_max(int sites) { return sites <= 16 ? 16 : 32; }

static void obs_grid(int ns, int64_t dim_up, int64_t dim_dn, int &ntiles, int &nchunks, int max_blocks = 2048)
{
    const int tw = kObsSlots * (ns <= 16 ? obs_threads<16>() : obs_threads<32>());
    ntiles = (int)((dim_dn + tw - 1) / tw);
    int64_t nc = max_blocks / ntiles;
    if (nc < 1)
        nc = 1;
    if (nc > dim_up)
        nc = dim_up;
    nchunks = (int)nc;
}

int obs_partial_count(int ns, int64_t dim_up, int64_t dim_dn, int max_blocks)
{
    int ntiles, nchunks;
    obs_grid(ns, dim_up, dim_dn, ntiles, nchunks, max_blocks);
    return ntiles * nchunks + kObsGroups;  // the workgroups' partials, then the group sums
}

template <int NS>
static void launch_obs(const double *psi, const uint32_t *states_up, const uint32_t *states_dn, int ns, int64_t dim_up,
                       int64_t dim_dn, double *part, double *out, int max_blocks, hipStream_t s)
{
    int ntiles, nchunks;
    obs_grid(ns, dim_up, dim_dn, ntiles, nchunks, max_blocks);
    const int nblocks = ntiles * nchunks;
    constexpr int TW = obs_threads<NS>();
    hipLaunchKernelGGL((obs_accumulate_kernel<NS, TW>), dim3(nblocks), dim3(TW), 0, s, psi, states_up, states_dn, ns,
                       dim_up, dim_dn, ntiles, nchunks, part);
    HUB_HIP(hipGetLastError());
    const int ps = obs_partial_size<NS>();
    double *grp = part + (int64_t)nblocks * ps;
    hipLaunchKernelGGL(obs_sum_kernel, dim3((ps + 255) / 256, kObsGroups), dim3(256), 0, s, part, nblocks, ps, grp);
    HUB_HIP(hipGetLastError());
    hipLaunchKernelGGL(obs_sum_groups_kernel, dim3((ps + 255) / 256), dim3(256), 0, s, grp, ps, out);
    HUB_HIP(hipGetLastError());
}

void launch_observables(const double *psi, const uint32_t *states_up, const uint32_t *states_dn, int ns,
                        int64_t dim_up, int64_t dim_dn, double *part, double *out, int max_blocks, hipStream_t s)
{
    if (ns <= 16)
        launch_obs<16>(psi, states_up, states_dn, ns, dim_up, dim_dn, part, out, max_blocks, s);
    else
        launch_obs<32>(psi, states_up, states_dn, ns, dim_up, dim_dn, part, out, max_blocks, s);
}

// Scratch of the entry point that allocates nothing (hubbard_observables_noalloc):
// the workgroups' partial sums, their group sums and the final sums live in this
// array, one copy per device for the life of the process.  Host code never
// passes the array's name to a kernel: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[kObsScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kObsMaxDevices] = {};

double *obs_scratch(int device)
{
    if (device < 0 || device >= kObsMaxDevices)
        fail(HUBBARD_EDEVICE, "device index out of range for the observables scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(HUBBARD_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    return static_cast<double *>(g_scratch_ptr[device]);
}

int obs_noalloc_blocks(int ns, int64_t dim_up, int64_t dim_dn)
{
    const int ps = ns <= 16 ? obs_partial_size<16>() : obs_partial_size<32>();
    // partials (blocks + groups) and the final sums must fit the scratch
    const int64_t cap = (int64_t)(kObsScratchBytes / sizeof(double)) / ps - kObsGroups - 1;
    int max_blocks = (int)std::min<int64_t>(2048, cap);
    while (max_blocks > 1 && (int64_t)(obs_partial_count(ns, dim_up, dim_dn, max_blocks) + 1) * ps >
                                 (int64_t)(kObsScratchBytes / sizeof(double)))
        max_blocks--;
    return max_blocks;
}

}  // namespace hub
