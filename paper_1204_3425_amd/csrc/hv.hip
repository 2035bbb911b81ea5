// Two-pass H.v for gfx950 (CDNA4).
//
// With the state vector viewed as the dim_up x dim_dn matrix X (Siro &
// Harju, Sec. 4.3, Fig. slots; J = i_up * dim_dn + i_dn),
//     H x = X A_dn^T + U D o X   +   A_up X.
// The two hopping terms want different data movement, so each gets a pass of
// its own:
//
// Row pass (I (x) H_dn and the interaction).  hv_rows64_kernel for FP64 rows that
// fill the LDS (one amplitude), hv_rows_kernel otherwise.  A workgroup stages whole rows of
// X in LDS (RPB rows at once, each followed by a zero slot; every thread loads
// its chunk before writing any of it) and every lane produces the outputs of
// its columns d by gathering X[r, e_k(d)] from LDS.  The down table is stored
// in groups per column d: eight 16-bit entries (element index, sign in bit 15)
// when a row has fewer than 32768 elements, else four 32-bit entries (byte
// offset, sign in bit 31).  All groups of a column are loaded before the first
// gather; padding entries point at the zero slot, so no lane tests how many
// entries it owns; the sign of a hop flips the sign bit of the gathered value.
// The group count is the maximum over the 64 columns of a wave.
//
// Up-spin pass (H_up (x) I).  Output row r is a signed sum of whole rows
// X[c_k(r), :].  Rows are grouped in blocks of equal occupation of the top
// sites (a contiguous range in the ascending order).  Workgroup b handles one
// 128-byte slab of one block, numbered slab-major per XCD (workgroup i runs on
// XCD i mod 8), so the rows that other blocks' hops re-read are still in that
// XCD's 4 MB L2.  The block's slab segment is staged in LDS and serves the
// hops that stay inside the block; the others read global memory.  Eight
// lanes cover one row segment with 16-byte accesses, so a wave updates eight
// rows.  hv_lines_kernel takes a row's entries as one 128-byte line (rows of at
// most 32 hops); hv_blocks_kernel handles longer rows.  Rows that start on 16
// but not on 128 bytes (a caller's dense vector) take the same passes with each
// XCD on a contiguous range of slabs; hv_slabs_kernel serves rows not on 16
// bytes.  The running output is read and written with non-temporal accesses.
//
// Epilogues (both passes together):
//   HV_STORE    y = H x
//   HV_LANCZOS  y = alpha H x + beta y, partial sums of y.x    (alpha, beta on the device)
//   HV_FUSED    x <- x - c y first (row pass), then as HV_LANCZOS, partial sums
//               of y.x, y.y and x.x
//   HV_RESIDUAL z = H x - alpha x (not stored), partial sums of z.z and x.Hx
// Partial sums are one FP64 value per up-spin-pass workgroup, summed later in
// a fixed order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace hub {

namespace {

constexpr int kSlab = 64;       // slab width in elements = one wave
constexpr int kSlabThreads = 256;
constexpr int kLdsBytes = 160 * 1024;

__device__ inline double block_sum2(double v, double *scratch)
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

// wave64 shuffle tree; the sum lands in lane 0
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline float flip_sign(float v, uint32_t sg) { return __int_as_float(__float_as_int(v) ^ (int)sg); }
__device__ inline double flip_sign(double v, uint32_t sg)
{
    return __longlong_as_double(__double_as_longlong(v) ^ ((long long)sg << 32));
}

struct RowArgs {
    const uint4 *__restrict__ groups;  // [g][d] -> 4 entries of 32 bits, or 8 of 16 bits
    const uint8_t *__restrict__ nq;    // groups per 64 columns
    const uint32_t *__restrict__ states_up;
    const uint32_t *__restrict__ states_dn;
    int64_t dim_up, dim_dn;
    int ngroups;
    double t, U;
    double amp[4];  // per-bond amplitude classes (GT kernels)
    void *xc;       // null, or rows at stride ldc that receive a copy of each staged row
    int64_t ldc;
    HvDefl defl;    // HV_FUSED_DEFL
    void *yo;       // fused modes: null (y is overwritten), or rows at stride ldyo for the result
    int64_t ldyo;
    int gmax;       // group slots per column in the table used (groups of eight 16-bit or four 32-bit entries)
};

// Per-bond amplitudes (GT kernels): entries carry a class of at most four
// amplitudes, bits 24..25 of an up-spin entry (row below 2^24) and bits 18..19
// of a row-pass group entry (byte offset below 2^18); the element is
// -amp[class] * sgn, so the class amplitude multiplies the signed value and
// the final factor is -1 instead of -t.
template <typename T>
__device__ inline T class_amp(const T (&a)[4], uint32_t c)
{
    return c == 0 ? a[0] : (c == 1 ? a[1] : (c == 2 ? a[2] : a[3]));
}
constexpr uint32_t kGtRowMask = 0x00FFFFFFu;

// The factor an up-spin entry contributes with: +-1 from its sign bit (the
// high word of +-1.0 built by one and-or), times the class amplitude in the
// per-bond kernels.  acc = fma(factor, x, acc) rounds exactly as acc +- x.
__device__ inline uint32_t and_or(uint32_t a, uint32_t smask, uint32_t vor)
{
    uint32_t r;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(smask), "v"(vor));
    return r;
}
template <typename T, bool GT>
__device__ inline T signed_factor(const T (&a)[4], uint32_t e)
{
    if (GT)
        return flip_sign(class_amp(a, (e >> 24) & 3u), e & 0x80000000u);
    // one instruction: the sign bit of e with the rest of +1.0's (high) word
    const uint32_t hi = and_or(e, 0x80000000u, sizeof(T) == 8 ? 0x3FF00000u : 0x3F800000u);
    if constexpr (sizeof(T) == 8)
        return __hiloint2double((int)hi, 0);
    else
        return __int_as_float((int)hi);
}

// Row pass.  MODE as in the file comment; for HV_RESIDUAL y is the scratch
// vector z and alpha is the shift.
// PF: every column's entries fit four groups (gmax <= 4), so the next column's
// groups, count, down configuration and (modes that read it) y are loaded a
// column ahead, every slot issued (past gmax: slot 0 again, unused; rows past
// the block: its last row) so that the wait counters stay exact.
// s_waitcnt vmcnt(0) with the other counters left alone (gfx9 encoding)
constexpr int kVmcnt0 = 0x0f70;

template <typename T, int RPB, int MODE, bool G16, bool GT, bool PF>
__global__ __launch_bounds__(1024) void hv_rows_kernel(RowArgs p, const T *__restrict__ x, int64_t ldx,
                                                       T *__restrict__ y, int64_t ldy, double alpha, double beta,
                                                       const double *__restrict__ coef)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *xs = reinterpret_cast<T *>(smem_raw);
    constexpr bool FUSED = MODE == HV_FUSED || MODE == HV_FUSED_DEFL;
    double cshift = 0.0;
    if (MODE == HV_LANCZOS) {
        alpha = coef[0];
        beta = coef[1];
    } else if (FUSED) {
        alpha = coef[1];
        beta = coef[2];
        cshift = coef[3];
    }
    double gd[kFusedDefl] = {};
    if (MODE == HV_FUSED_DEFL)
        for (int l = 0; l < p.defl.nd; l++)
            gd[l] = p.defl.g[l];
    const int64_t ddn = p.dim_dn;
    const int64_t slot = ddn + 1;  // staged row length including the zero slot
    const T mt = GT ? (T)(-1) : (T)(-p.t), U = (T)p.U, a_s = (T)alpha, b_s = (T)beta, c_s = (T)cshift;
    const T am[4] = {(T)p.amp[0], (T)p.amp[1], (T)p.amp[2], (T)p.amp[3]};
    // staging: each thread loads CH elements of each of the RPB rows before it
    // writes any of them to LDS, so a row costs one or two memory round trips
    constexpr int CH = (FUSED ? 8 : 16) / RPB;
    const int ddn32 = (int)ddn, nth = (int)blockDim.x;

    for (int64_t r0 = (int64_t)blockIdx.x * RPB; r0 < p.dim_up; r0 += (int64_t)gridDim.x * RPB) {
        const int nr = (int)min((int64_t)RPB, p.dim_up - r0);
        for (int d0 = 0; d0 < ddn32; d0 += CH * nth) {
            T v[RPB][CH], w[RPB][CH];
            double pg[RPB][CH];  // sum_l g_l psi_l (deflated step)
#pragma unroll
            for (int q = 0; q < RPB; q++) {
#pragma unroll
                for (int u = 0; u < CH; u++) {
                    const int d = d0 + u * nth + (int)threadIdx.x;
                    const bool ok = q < nr && d < ddn32;
                    v[q][u] = ok ? x[(r0 + q) * ldx + d] : (T)0;
                    if (FUSED)
                        w[q][u] = ok ? y[(r0 + q) * ldy + d] : (T)0;
                    pg[q][u] = 0.0;
                    if (MODE == HV_FUSED_DEFL && ok)
                        for (int l = 0; l < p.defl.nd; l++)
                            pg[q][u] += gd[l] * p.defl.psi[(int64_t)l * p.defl.pdim + (r0 + q) * ddn + d];
                }
            }
#pragma unroll
            for (int q = 0; q < RPB; q++) {
#pragma unroll
                for (int u = 0; u < CH; u++) {
                    const int d = d0 + u * nth + (int)threadIdx.x;
                    if (q < nr && d < ddn32) {
                        T val = v[q][u];
                        if (FUSED) {
                            // the q - a_j f_j update of the previous step (projected
                            // in the deflated step, rounded once), formed here and kept
                            val = val - c_s * w[q][u];
                            if (MODE == HV_FUSED_DEFL)
                                val = (T)((double)val - pg[q][u]);
                            const_cast<T *>(x)[(r0 + q) * ldx + d] = val;
                        }
                        xs[q * slot + d] = val;
                        if (p.xc)
                            static_cast<T *>(p.xc)[(r0 + q) * p.ldc + d] = val;
                    }
                }
            }
        }
        if (threadIdx.x < RPB)
            xs[threadIdx.x * slot + ddn] = (T)0;
        __syncthreads();
        uint32_t su[RPB];
#pragma unroll
        for (int q = 0; q < RPB; q++)
            su[q] = p.states_up[min(r0 + q, p.dim_up - 1)];

        // 32 entries per batch of table loads: 8 groups of four 32-bit
        // entries, or 4 groups of eight 16-bit entries
        constexpr int GB = G16 ? 4 : 8;
        // one batch of groups: the hops of entries g0 * (G16 ? 8 : 4) on
        auto batch = [&](int g0, int nq, const auto &e4, T (&h)[RPB]) {
            constexpr int N = (int)(sizeof(e4) / sizeof(uint4));
#pragma unroll
            for (int g = 0; g < N; g++) {
                if (g0 + g < nq) {
                    const uint32_t ev[4] = {e4[g].x, e4[g].y, e4[g].z, e4[g].w};
#pragma unroll
                    for (int u = 0; u < (G16 ? 8 : 4); u++) {
                        uint32_t off, sg;
                        if (G16) {
                            const uint32_t e = (ev[u >> 1] >> ((u & 1) * 16)) & 0xffffu;
                            off = (e & 0x7fffu) * (uint32_t)sizeof(T);
                            sg = (e & 0x8000u) << 16;
                        } else {
                            off = ev[u] & (GT ? 0x3ffffu : 0x7fffffffu);
                            sg = ev[u] & 0x80000000u;
                        }
                        const T ac = GT ? class_amp(am, (ev[u] >> 18) & 3u) : (T)1;
#pragma unroll
                        for (int q = 0; q < RPB; q++) {
                            const T v = *reinterpret_cast<const T *>(
                                reinterpret_cast<const unsigned char *>(xs + q * slot) + off);
                            if (GT)
                                h[q] += ac * flip_sign(v, sg);
                            else
                                h[q] += flip_sign(v, sg);
                        }
                    }
                }
            }
        };
        // a column's groups, group count, down configuration and y values (PF)
        constexpr int PB = 4;
        constexpr bool YR = MODE == HV_LANCZOS || FUSED;  // the result reads y
        auto fetch = [&](int64_t dcol, uint4 (&e4)[PB], int &nq, uint32_t &sdc, T (&yv)[RPB]) {
            const int64_t dd = dcol < ddn ? dcol : ddn - 1;
            nq = p.nq[dd >> 6];
#pragma unroll
            for (int g = 0; g < PB; g++)
                e4[g] = p.groups[(int64_t)(g < p.gmax ? g : 0) * ddn + dd];
            sdc = p.states_dn[dd];
#pragma unroll
            for (int q = 0; q < RPB; q++)
                if (YR)
                    yv[q] = y[(r0 + (q < nr ? q : nr - 1)) * ldy + dd];
        };
        // FULL (PF and a whole block of rows): the result is stored without a
        // branch, lanes past the row's end repeating its last column (the same
        // groups, counts and y value, so the same value to the same address),
        // so the wait for the next column's loads never waits for these stores
        auto cols = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            uint4 ec[PB];
            int nqc = 0;
            uint32_t sdc = 0;
            T yc[RPB] = {};
            if (PF) {
                fetch(threadIdx.x, ec, nqc, sdc, yc);
                // these loads complete before the loop: entered with them in
                // flight, the loop would wait for all of its own memory
                // operations (the stores included) at the top of every column
                __builtin_amdgcn_s_waitcnt(kVmcnt0);
            }
            // a wave stops after its last chunk that holds a column of the row,
            // so the lanes that repeat the last column sit in that column's wave
            // (and read y there before it is written)
            for (int64_t d0 = 0; d0 + (int64_t)(threadIdx.x & ~63u) < ddn; d0 += blockDim.x) {
                const int64_t d = d0 + threadIdx.x;
                const bool ok = d < ddn;
                const int64_t dd = ok ? d : ddn - 1;
                T h[RPB];
#pragma unroll
                for (int q = 0; q < RPB; q++)
                    h[q] = (T)0;
                uint32_t sd = sdc;
                T yr[RPB];
#pragma unroll
                for (int q = 0; q < RPB; q++)
                    yr[q] = yc[q];
                if (PF) {
                    uint4 en[PB];
                    int nqn;
                    uint32_t sdn;
                    fetch(d + blockDim.x, en, nqn, sdn, yc);
                    batch(0, nqc, ec, h);
#pragma unroll
                    for (int g = 0; g < PB; g++)
                        ec[g] = en[g];
                    nqc = nqn;
                    sdc = sdn;
                } else {
                    const int nq = p.nq[dd >> 6];
                    const uint4 *__restrict__ gp = p.groups + dd;
                    for (int g0 = 0; g0 < nq; g0 += GB) {
                        uint4 e4[GB];
#pragma unroll
                        for (int g = 0; g < GB; g++)
                            if (g0 + g < nq)
                                e4[g] = gp[(int64_t)(g0 + g) * ddn];
                        batch(g0, nq, e4, h);
                    }
                    sd = p.states_dn[dd];
                }
                if (FULL || ok) {
#pragma unroll
                    for (int q = 0; q < RPB; q++) {
                        if (FULL || q < nr) {
                            const T xv = xs[q * slot + dd];
                            const T hx = fma(mt, h[q], U * (T)__popc(su[q] & sd) * xv);
                            T *yp = y + (r0 + q) * ldy + dd;
                            const T yv = PF ? yr[q] : (YR ? *yp : (T)0);
                            if (MODE == HV_STORE)
                                *yp = hx;
                            else if (FUSED && p.yo)
                                static_cast<T *>(p.yo)[(r0 + q) * p.ldyo + dd] = a_s * hx + b_s * yv;
                            else if (YR)
                                *yp = a_s * hx + b_s * yv;
                            else
                                *yp = hx - a_s * xv;
                        }
                    }
                }
            }
        };
        if (PF && nr == RPB)
            cols(std::true_type());
        else
            cols(std::false_type());
        __syncthreads();
    }
}

// FP64 row pass (one amplitude; rows of at most 13,312 elements).
//
// The same product as hv_rows_kernel with one row per workgroup (an FP64 row
// of the 4x4 lattice fills the LDS), with two instructions per entry and no
// sign handling: a column's hops are split by sign, those of sign + in groups
// of eight 16-bit element indices and those of sign - in groups of four, and
// the gathered value is added to, or subtracted from, the sum (the negation
// is an operand modifier).  The 16-bit index becomes the byte address by one
// shift that reads the half word in place (SDWA).  Padding entries gather the
// zero slot after the row.  Each wave takes 64 columns at a time; the group
// counts of its column chunks sit one per lane of a register and reach the
// wave by a lane read, so no scalar load waits inside the column loop.  The
// row sits in a statically sized LDS array, so an address needs no base.  A
// column's entry groups are loaded one column ahead, and the next row is
// loaded into registers (16-byte loads) while the current one is gathered
// and written to LDS after the barrier that ends it.
constexpr int kRowThreads = 1024;

struct Row64Args {
    const uint4 *__restrict__ pidx;     // [g][d] -> eight 16-bit element indices of + hops
    const uint2 *__restrict__ nidx;     // [g][d] -> four 16-bit element indices of - hops
    const uint8_t *__restrict__ pn;     // per 64 columns: + groups, - groups (two bytes)
    const uint32_t *__restrict__ states_up;
    const uint32_t *__restrict__ states_dn;
    int64_t dim_up;
    int dim_dn;
    double t, U;
    double *xc;  // null, or rows at stride ldc that receive a copy of each staged row
    int64_t ldc;
    HvDefl defl;  // HV_FUSED_DEFL
    double *yo;   // fused modes: null (y is overwritten), or rows at stride ldyo for the result
    int64_t ldyo;
};

__device__ inline uint32_t lds_off_lo(uint32_t e)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(r)
        : "v"(e));
    return r;
}
__device__ inline uint32_t lds_off_hi(uint32_t e)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "=v"(r)
        : "v"(e));
    return r;
}
__device__ inline double lds_at(const double *xs, uint32_t byte)
{
    return *reinterpret_cast<const double *>(reinterpret_cast<const unsigned char *>(xs) + byte);
}

// NP groups of eight + hops and NN groups of four - hops at most per column
template <int MODE, bool VEC, int CH, int NP, int NN>
__global__ __launch_bounds__(kRowThreads) void hv_rows64_kernel(Row64Args p, const double *__restrict__ x, int64_t ldx,
                                                                double *__restrict__ y, int64_t ldy, double alpha,
                                                                double beta, const double *__restrict__ coef)
{
    __shared__ __align__(16) double xs[kRow64Max + 2];
    constexpr bool FUSED = MODE == HV_FUSED || MODE == HV_FUSED_DEFL;
    double cshift = 0.0;
    if (MODE == HV_LANCZOS) {
        alpha = coef[0];
        beta = coef[1];
    } else if (FUSED) {
        alpha = coef[1];
        beta = coef[2];
        cshift = coef[3];
    }
    double gd[kFusedDefl] = {};
    if (MODE == HV_FUSED_DEFL)
        for (int l = 0; l < p.defl.nd; l++)
            gd[l] = p.defl.g[l];
    const int ddn = p.dim_dn, tid = (int)threadIdx.x, lane = tid & 63;
    // staging units: 16-byte pairs (rows 16-byte aligned) or single elements
    typedef typename std::conditional<VEC, double2, double>::type SU;
    const int nu = VEC ? ddn >> 1 : ddn;
    const bool tail = VEC && (ddn & 1) && tid == kRowThreads - 1;  // the odd last element of a VEC row
    SU v[CH], w[CH];
    double vt = 0.0, wt = 0.0;
    auto load_row = [&](int64_t r) {
        const SU *src = reinterpret_cast<const SU *>(x + r * ldx);
        const SU *ysrc = reinterpret_cast<const SU *>(y + r * ldy);
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int i = u * kRowThreads + tid;
            if (i < nu) {
                v[u] = src[i];
                if (FUSED)
                    w[u] = ysrc[i];
            }
        }
        if (tail) {
            vt = x[r * ldx + ddn - 1];
            if (FUSED)
                wt = y[r * ldy + ddn - 1];
        }
    };
    // psi_l at element e of row r (dense rows)
    auto psi_at = [&](int l, int64_t r, int e) -> double {
        return p.defl.psi[(int64_t)l * p.defl.pdim + r * (int64_t)ddn + e];
    };
    auto store_row = [&](int64_t r) {
        SU *xs2 = reinterpret_cast<SU *>(xs);
        SU *xw = reinterpret_cast<SU *>(const_cast<double *>(x) + r * ldx);
        SU *xc = reinterpret_cast<SU *>(p.xc + r * p.ldc);
        // the projection of the deflated step: sum_l g_l psi_l at this
        // thread's elements (all loads issued before the first use)
        SU pg[CH];
        double pgt = 0.0;
        if (MODE == HV_FUSED_DEFL) {
#pragma unroll
            for (int u = 0; u < CH; u++)
                pg[u] = SU{};
            for (int l = 0; l < p.defl.nd; l++) {
#pragma unroll
                for (int u = 0; u < CH; u++) {
                    const int i = u * kRowThreads + tid;
                    if (i < nu) {
                        if constexpr (VEC)
                            pg[u] = pg[u] + gd[l] * SU{psi_at(l, r, 2 * i), psi_at(l, r, 2 * i + 1)};
                        else
                            pg[u] = pg[u] + gd[l] * psi_at(l, r, i);
                    }
                }
                if (tail)
                    pgt += gd[l] * psi_at(l, r, ddn - 1);
            }
        }
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int i = u * kRowThreads + tid;
            if (i < nu) {
                SU val = v[u];
                if (FUSED) {
                    // the q - a_j f_j update of the previous step (projected in
                    // the deflated step), formed here and kept
                    val = val - cshift * w[u];
                    if (MODE == HV_FUSED_DEFL)
                        val = val - pg[u];
                    xw[i] = val;
                } else if (p.xc) {
                    xc[i] = val;
                }
                xs2[i] = val;
            }
        }
        if (tail) {
            double val = vt;
            if (FUSED) {
                val = val - cshift * wt;
                if (MODE == HV_FUSED_DEFL)
                    val = val - pgt;
                const_cast<double *>(x)[r * ldx + ddn - 1] = val;
            } else if (p.xc) {
                p.xc[r * p.ldc + ddn - 1] = val;
            }
            xs[ddn - 1] = val;
        }
        if (tid == 0)
            xs[ddn] = 0.0;  // the zero slot that padding entries point at
    };

    const double mt = -p.t, U = p.U;
    // lane k holds the group counts of this wave's k-th column chunk (chunk
    // wave + 16 k); a wave takes at most 64 chunks (rows of up to 65,536
    // elements).  Chunks past the row's end take the last chunk's counts: their
    // lanes repeat the row's last column (below).
    const int wv = tid >> 6, nchunk = (ddn + 63) >> 6;
    const uint32_t cnt_lane =
        *reinterpret_cast<const uint16_t *>(p.pn + 2 * min(wv + 16 * lane, nchunk - 1));
    auto counts = [&](int k) -> uint32_t { return (uint32_t)__builtin_amdgcn_readlane((int)cnt_lane, k); };
    // a column's entry groups (all of them, so one memory round trip per
    // column).  Every load is issued, slots past the column chunk's counts
    // reading group 0 again (unused): with no skipped loads the wait counters
    // stay exact, and using this column's groups never waits for the loads of
    // the next one.
    auto load_groups = [&](int d, uint32_t c, uint4 (&ep)[NP], uint2 (&en)[NN], uint32_t &sd) {
        const int dd = d < ddn ? d : ddn - 1;
        const int np = (int)(c & 0xffu), nn = (int)(c >> 8);
#pragma unroll
        for (int g = 0; g < NP; g++)
            ep[g] = p.pidx[(size_t)(g < np ? g : 0) * (size_t)ddn + (size_t)dd];
#pragma unroll
        for (int g = 0; g < NN; g++)
            en[g] = p.nidx[(size_t)(g < nn ? g : 0) * (size_t)ddn + (size_t)dd];
        sd = p.states_dn[dd];
    };
    int64_t r = blockIdx.x;
    if (r < p.dim_up)
        load_row(r);
    for (; r < p.dim_up; r += gridDim.x) {
        store_row(r);
        __syncthreads();
        const uint32_t su = p.states_up[r];
        uint32_t c = counts(0);
        uint4 ep[NP];
        uint2 en[NN];
        uint32_t sd = 0;
        load_groups(tid, c, ep, en, sd);
        // the next row's loads stay in flight while this one is gathered;
        // issued after the first column's groups, so that the wait for those
        // (the counters complete in order) does not wait for the row
        if (r + gridDim.x < p.dim_up)
            load_row(r + gridDim.x);
        int k = 0;
        // a wave stops after its last chunk that holds a column of the row, so
        // the lanes that repeat the last column sit in that column's wave (and
        // read y there before it is written)
        for (int d0 = 0; d0 + (wv << 6) < ddn; d0 += kRowThreads, k++) {
            const int d = d0 + tid;
            // the next column's entries load while this one is gathered
            const uint32_t cn = counts(k + 1);
            uint4 epn[NP];
            uint2 enn[NN];
            uint32_t sdn = 0;
            constexpr bool ahead = !FUSED;  // the fused modes have no registers to spare
            if (ahead)
                load_groups(d + kRowThreads, cn, epn, enn, sdn);
            // y at this column (modes that read it) loads while the column is gathered
            constexpr bool YR = MODE == HV_LANCZOS || FUSED;
            double yv = 0.0;
            if (YR)
                yv = y[r * ldy + (d < ddn ? d : ddn - 1)];
            const int np = (int)(c & 0xffu), nn = (int)(c >> 8);
            {
                double h0 = 0.0, h1 = 0.0;
#pragma unroll
                for (int g = 0; g < NP; g++) {
                    if (g < np) {
                        const uint32_t ev[4] = {ep[g].x, ep[g].y, ep[g].z, ep[g].w};
                        double xv[8];
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            xv[u] = lds_at(xs, (u & 1) ? lds_off_hi(ev[u >> 1]) : lds_off_lo(ev[u >> 1]));
#pragma unroll
                        for (int u = 0; u < 8; u += 2) {
                            h0 += xv[u];
                            h1 += xv[u + 1];
                        }
                    }
                }
#pragma unroll
                for (int g = 0; g < NN; g++) {
                    if (g < nn) {
                        const uint32_t ev[2] = {en[g].x, en[g].y};
                        double xv[4];
#pragma unroll
                        for (int u = 0; u < 4; u++)
                            xv[u] = lds_at(xs, (u & 1) ? lds_off_hi(ev[u >> 1]) : lds_off_lo(ev[u >> 1]));
                        h0 -= xv[0];
                        h1 -= xv[1];
                        h0 -= xv[2];
                        h1 -= xv[3];
                    }
                }
                // every lane stores: lanes past the row's end repeat its last
                // column (the same groups, counts and value, to the same
                // address), so no store is skipped and the wait for the next
                // column's loads never waits for this one's store
                {
                    const int dd = d < ddn ? d : ddn - 1;
                    const double xd = xs[dd];
                    const double hx = fma(mt, h0 + h1, U * (double)__popc(su & sd) * xd);
                    double *yp = y + r * ldy + dd;
                    if (MODE == HV_STORE)
                        *yp = hx;
                    else if (FUSED && p.yo)
                        p.yo[r * p.ldyo + dd] = alpha * hx + beta * yv;
                    else if (YR)
                        *yp = alpha * hx + beta * yv;
                    else
                        *yp = hx - alpha * xd;
                }
            }
            c = cn;
            if (ahead) {
#pragma unroll
                for (int g = 0; g < NP; g++)
                    ep[g] = epn[g];
#pragma unroll
                for (int g = 0; g < NN; g++)
                    en[g] = enn[g];
                sd = sdn;
            } else {
                load_groups(d + kRowThreads, cn, ep, en, sd);
            }
        }
        __syncthreads();
    }
}

// FP32 row pass on pairs of rows (one amplitude; rows of at most 13,312
// elements).
//
// hv_rows64_kernel's product for two up configurations at once: rows r and
// r + 1 sit in LDS interleaved, element e of both as one 8-byte pair, so one
// gather at the FP64 kernel's address (the 16-bit index shifted by three)
// fetches a hop's value for both rows and a table entry costs one shift, one
// gather and two adds for two outputs.  The pair fills the LDS as one FP64 row
// does.  Rows are staged in 8-byte units (two elements of a row), written to
// LDS as 16 bytes (the two elements of both rows).  Modes as hv_rows64_kernel
// without the deflated step.
struct Row32Args {
    const uint4 *__restrict__ pidx;  // [g][d] -> eight 16-bit element indices of + hops
    const uint2 *__restrict__ nidx;  // [g][d] -> four 16-bit element indices of - hops
    const uint8_t *__restrict__ pn;  // per 64 columns: + groups, - groups (two bytes)
    const uint32_t *__restrict__ states_up;
    const uint32_t *__restrict__ states_dn;
    int64_t dim_up;
    int dim_dn;
    double t, U;
    float *xc;  // null, or rows at stride ldc that receive a copy of each staged row
    int64_t ldc;
    float *yo;  // fused mode: null (y is overwritten), or rows at stride ldyo for the result
    int64_t ldyo;
};

__device__ inline float2 lds_pair(const float2 *xs, uint32_t byte)
{
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const unsigned char *>(xs) + byte);
}

template <int MODE, bool VEC, int CH, int NP, int NN>
__global__ __launch_bounds__(kRowThreads) void hv_rows32x2_kernel(Row32Args p, const float *__restrict__ x,
                                                                  int64_t ldx, float *__restrict__ y, int64_t ldy,
                                                                  double alpha, double beta,
                                                                  const double *__restrict__ coef)
{
    __shared__ __align__(16) float2 xs[kRow64Max + 2];
    constexpr bool FUSED = MODE == HV_FUSED;
    double cshift = 0.0;
    if (MODE == HV_LANCZOS) {
        alpha = coef[0];
        beta = coef[1];
    } else if (FUSED) {
        alpha = coef[1];
        beta = coef[2];
        cshift = coef[3];
    }
    const float a_s = (float)alpha, b_s = (float)beta, c_s = (float)cshift;
    const int ddn = p.dim_dn, tid = (int)threadIdx.x, lane = tid & 63;
    const int64_t npair = (p.dim_up + 1) / 2;
    // staging units: two elements of a row (rows on 8 bytes) or one element
    typedef typename std::conditional<VEC, float2, float>::type SU;
    const int nu = VEC ? ddn >> 1 : ddn;
    const bool tail = VEC && (ddn & 1) && tid == kRowThreads - 1;  // the odd last element of a VEC row
    SU v0[CH], v1[CH], w0[CH], w1[CH];
    float vt0 = 0.f, vt1 = 0.f, wt0 = 0.f, wt1 = 0.f;
    // units [0, PFU) of the next pair load while the current one is gathered,
    // the rest when it is staged (registers for the whole pair would spill)
    constexpr int PFU = VEC ? 3 : 5;
    // units [u0, u1) of rows r and r1 of a pair (r1 = r for the last pair of an
    // odd count: its second half is computed and not stored)
    auto load_pair = [&](int64_t r, int64_t r1, int u0, int u1) {
        const SU *s0 = reinterpret_cast<const SU *>(x + r * ldx);
        const SU *s1 = reinterpret_cast<const SU *>(x + r1 * ldx);
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int i = u * kRowThreads + tid;
            if (u >= u0 && u < u1 && i < nu) {
                v0[u] = s0[i];
                v1[u] = s1[i];
            }
        }
        if (tail && u1 == CH) {
            vt0 = x[r * ldx + ddn - 1];
            vt1 = x[r1 * ldx + ddn - 1];
        }
    };
    // the fused step's previous y, read when the pair is staged
    auto load_prev = [&](int64_t r, int64_t r1) {
        const SU *s0 = reinterpret_cast<const SU *>(y + r * ldy);
        const SU *s1 = reinterpret_cast<const SU *>(y + r1 * ldy);
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int i = u * kRowThreads + tid;
            if (i < nu) {
                w0[u] = s0[i];
                w1[u] = s1[i];
            }
        }
        if (tail) {
            wt0 = y[r * ldy + ddn - 1];
            wt1 = y[r1 * ldy + ddn - 1];
        }
    };
    auto store_pair = [&](int64_t r, int64_t r1, bool two) {
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int i = u * kRowThreads + tid;
            if (i < nu) {
                SU a = v0[u], b = v1[u];
                if (FUSED) {
                    // the q - a_j f_j update of the previous step, formed here and kept
                    if constexpr (VEC) {
                        a = make_float2(a.x - c_s * w0[u].x, a.y - c_s * w0[u].y);
                        b = make_float2(b.x - c_s * w1[u].x, b.y - c_s * w1[u].y);
                    } else {
                        a = a - c_s * w0[u];
                        b = b - c_s * w1[u];
                    }
                    reinterpret_cast<SU *>(const_cast<float *>(x) + r * ldx)[i] = a;
                    if (two)
                        reinterpret_cast<SU *>(const_cast<float *>(x) + r1 * ldx)[i] = b;
                } else if (p.xc) {
                    reinterpret_cast<SU *>(p.xc + r * p.ldc)[i] = a;
                    if (two)
                        reinterpret_cast<SU *>(p.xc + r1 * p.ldc)[i] = b;
                }
                if constexpr (VEC)
                    reinterpret_cast<float4 *>(xs)[i] = make_float4(a.x, b.x, a.y, b.y);
                else
                    xs[i] = make_float2(a, b);
            }
        }
        if (tail) {
            float a = vt0, b = vt1;
            if (FUSED) {
                a = a - c_s * wt0;
                b = b - c_s * wt1;
                const_cast<float *>(x)[r * ldx + ddn - 1] = a;
                if (two)
                    const_cast<float *>(x)[r1 * ldx + ddn - 1] = b;
            } else if (p.xc) {
                p.xc[r * p.ldc + ddn - 1] = a;
                if (two)
                    p.xc[r1 * p.ldc + ddn - 1] = b;
            }
            xs[ddn - 1] = make_float2(a, b);
        }
        if (tid == 0)
            xs[ddn] = make_float2(0.f, 0.f);  // the zero slot that padding entries point at
    };

    const float mt = (float)(-p.t), U = (float)p.U;
    // counts of a wave's column chunks, one per lane (as in hv_rows64_kernel)
    const int wv = tid >> 6, nchunk = (ddn + 63) >> 6;
    const uint32_t cnt_lane =
        *reinterpret_cast<const uint16_t *>(p.pn + 2 * min(wv + 16 * lane, nchunk - 1));
    auto counts = [&](int k) -> uint32_t { return (uint32_t)__builtin_amdgcn_readlane((int)cnt_lane, k); };
    auto load_groups = [&](int d, uint32_t c, uint4 (&ep)[NP], uint2 (&en)[NN], uint32_t &sd) {
        const int dd = d < ddn ? d : ddn - 1;
        const int np = (int)(c & 0xffu), nn = (int)(c >> 8);
#pragma unroll
        for (int g = 0; g < NP; g++)
            ep[g] = p.pidx[(size_t)(g < np ? g : 0) * (size_t)ddn + (size_t)dd];
#pragma unroll
        for (int g = 0; g < NN; g++)
            en[g] = p.nidx[(size_t)(g < nn ? g : 0) * (size_t)ddn + (size_t)dd];
        sd = p.states_dn[dd];
    };
    int64_t pr = blockIdx.x;
    if (pr < npair)
        load_pair(2 * pr, min(2 * pr + 1, p.dim_up - 1), 0, PFU);
    for (; pr < npair; pr += gridDim.x) {
        const int64_t r = 2 * pr, r1 = min(r + 1, p.dim_up - 1);
        const bool two = r + 1 < p.dim_up;
        load_pair(r, r1, PFU, CH);
        if (FUSED)
            load_prev(r, r1);
        store_pair(r, r1, two);
        __syncthreads();
        const uint32_t su0 = p.states_up[r], su1 = p.states_up[r1];
        // the pair's rows of y (read) and of the result (uniform bases, so an
        // access needs only the column offset)
        const float *yin0 = y + r * ldy, *yin1 = y + r1 * ldy;
        float *yout0 = (FUSED && p.yo) ? p.yo + r * p.ldyo : y + r * ldy;
        float *yout1 = (FUSED && p.yo) ? p.yo + r1 * p.ldyo : y + r1 * ldy;
        uint32_t c = counts(0);
        uint4 ep[NP];
        uint2 en[NN];
        uint32_t sd = 0;
        load_groups(tid, c, ep, en, sd);
        if (pr + gridDim.x < npair)
            load_pair(2 * (pr + gridDim.x), min(2 * (pr + gridDim.x) + 1, p.dim_up - 1), 0, PFU);
        int k = 0;
        for (int d0 = 0; d0 + (wv << 6) < ddn; d0 += kRowThreads, k++) {
            const int d = d0 + tid;
            const uint32_t cn = counts(k + 1);
            uint4 epn[NP];
            uint2 enn[NN];
            uint32_t sdn = 0;
            // the next column's groups load after this one's gathers: loaded a
            // column ahead they would need registers the pair does not leave
            constexpr bool ahead = false;
            if (ahead)
                load_groups(d + kRowThreads, cn, epn, enn, sdn);
            constexpr bool YR = MODE == HV_LANCZOS || FUSED;
            const int dd = d < ddn ? d : ddn - 1;
            float yv0 = 0.f, yv1 = 0.f;
            if (YR) {
                yv0 = yin0[dd];
                yv1 = yin1[dd];
            }
            const int np = (int)(c & 0xffu), nn = (int)(c >> 8);
            float2 h0 = make_float2(0.f, 0.f), h1 = make_float2(0.f, 0.f);
#pragma unroll
            for (int g = 0; g < NP; g++) {
                if (g < np) {
                    const uint32_t ev[4] = {ep[g].x, ep[g].y, ep[g].z, ep[g].w};
                    float2 xv[8];
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        xv[u] = lds_pair(xs, (u & 1) ? lds_off_hi(ev[u >> 1]) : lds_off_lo(ev[u >> 1]));
#pragma unroll
                    for (int u = 0; u < 8; u += 2) {
                        h0.x += xv[u].x;
                        h0.y += xv[u].y;
                        h1.x += xv[u + 1].x;
                        h1.y += xv[u + 1].y;
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < NN; g++) {
                if (g < nn) {
                    const uint32_t ev[2] = {en[g].x, en[g].y};
                    float2 xv[4];
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        xv[u] = lds_pair(xs, (u & 1) ? lds_off_hi(ev[u >> 1]) : lds_off_lo(ev[u >> 1]));
#pragma unroll
                    for (int u = 0; u < 4; u += 2) {
                        h0.x -= xv[u].x;
                        h0.y -= xv[u].y;
                        h1.x -= xv[u + 1].x;
                        h1.y -= xv[u + 1].y;
                    }
                }
            }
            // every lane stores (lanes past the row's end repeat its last
            // column); the second row of an odd count's last pair is not stored
            {
                const float2 xd = xs[dd];
                const float hx0 = fmaf(mt, h0.x + h1.x, U * (float)__popc(su0 & sd) * xd.x);
                const float hx1 = fmaf(mt, h0.y + h1.y, U * (float)__popc(su1 & sd) * xd.y);
                float o0, o1;
                if (MODE == HV_STORE) {
                    o0 = hx0;
                    o1 = hx1;
                } else if (YR) {
                    o0 = a_s * hx0 + b_s * yv0;
                    o1 = a_s * hx1 + b_s * yv1;
                } else {
                    o0 = hx0 - a_s * xd.x;
                    o1 = hx1 - a_s * xd.y;
                }
                yout0[dd] = o0;
                if (two)
                    yout1[dd] = o1;
            }
            c = cn;
            if (ahead) {
#pragma unroll
                for (int g = 0; g < NP; g++)
                    ep[g] = epn[g];
#pragma unroll
                for (int g = 0; g < NN; g++)
                    en[g] = enn[g];
                sd = sdn;
            } else {
                load_groups(d + kRowThreads, cn, ep, en, sd);
            }
        }
        __syncthreads();
    }
}

struct SlabArgs {
    const uint32_t *__restrict__ up_rows;  // row-major entries (column | sign<<31)
    const uint16_t *__restrict__ nnz_up;
    int64_t dim_up, dim_dn;
    int w_up, rows_per_wg, nslab;
    double t;
    double amp[4];
};

// Slab pass.  y holds the row-pass result and receives the complete product.
template <typename T, int MODE, bool GT>
__global__ __launch_bounds__(kSlabThreads) void hv_slabs_kernel(SlabArgs p, const T *__restrict__ x, int64_t ldx,
                                                                T *__restrict__ y, int64_t ldy, double alpha,
                                                                const double *__restrict__ coef,
                                                                double *__restrict__ partials)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint32_t *ent = reinterpret_cast<uint32_t *>(smem_raw);
    int *nn = reinterpret_cast<int *>(ent + (size_t)p.rows_per_wg * p.w_up);
    __shared__ double red[4];
    if (MODE == HV_LANCZOS)
        alpha = coef[0];
    const T a_s = (T)alpha, tp = (T)p.t;
    const T am[4] = {(T)p.amp[0], (T)p.amp[1], (T)p.amp[2], (T)p.amp[3]};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xcd = blockIdx.x & 7;
    const int64_t local = blockIdx.x >> 3;
    const int64_t r0 = local * p.rows_per_wg;
    const int nr = (int)max((int64_t)0, min((int64_t)p.rows_per_wg, p.dim_up - r0));
    double acc0 = 0.0, acc1 = 0.0;

    for (int i = threadIdx.x; i < nr * p.w_up; i += blockDim.x) {
        const int q = i / p.w_up, k = i - q * p.w_up;
        ent[i] = p.up_rows[(r0 + q) * p.w_up + k];
    }
    for (int i = threadIdx.x; i < nr; i += blockDim.x)
        nn[i] = p.nnz_up[r0 + i];
    __syncthreads();

    constexpr int UNR = 8;
    for (int s = xcd; s < p.nslab; s += 8) {
        const int64_t dcol = (int64_t)s * kSlab + lane;
        const bool okd = dcol < p.dim_dn;
        const int64_t d = okd ? dcol : p.dim_dn - 1;
        for (int q = wave; q < nr; q += kSlabThreads / 64) {
            const int64_t r = r0 + q;
            const int n = nn[q];
            const uint32_t *er = ent + (size_t)q * p.w_up;
            T acc = (T)0;
            for (int k0 = 0; k0 < n; k0 += UNR) {
                int64_t c[UNR];
                T cf[UNR];
#pragma unroll
                for (int u = 0; u < UNR; u++) {
                    const bool live = k0 + u < n;
                    const uint32_t e = er[live ? k0 + u : 0];
                    c[u] = live ? (int64_t)(e & (GT ? kGtRowMask : 0x7fffffffu)) : r;
                    const T ap = GT ? class_amp(am, (e >> 24) & 3u) : tp;
                    cf[u] = live ? ((e >> 31) ? ap : -ap) : (T)0;
                }
                T v[UNR];
#pragma unroll
                for (int u = 0; u < UNR; u++)
                    v[u] = x[c[u] * ldx + d];
#pragma unroll
                for (int u = 0; u < UNR; u++)
                    acc = fma(cf[u], v[u], acc);
            }
            if (okd) {
                T *yp = y + r * ldy + d;
                const T prev = __builtin_nontemporal_load(yp);
                if (MODE == HV_STORE) {
                    __builtin_nontemporal_store(prev + acc, yp);
                } else if (MODE == HV_LANCZOS) {
                    const T q2 = prev + a_s * acc;
                    __builtin_nontemporal_store(q2, yp);
                    acc0 += (double)q2 * (double)x[r * ldx + d];
                } else {
                    const double z = (double)prev + (double)acc;  // H x - alpha x
                    const double xv = (double)x[r * ldx + d];
                    acc0 += z * z;
                    acc1 += xv * (z + alpha * xv);  // x . H x
                }
            }
        }
    }
    if (MODE != HV_STORE) {
        const double s0 = block_sum2(acc0, red);
        if (threadIdx.x == 0)
            partials[blockIdx.x] = s0;
        if (MODE == HV_RESIDUAL) {
            const double s1 = block_sum2(acc1, red);
            if (threadIdx.x == 0)
                partials[gridDim.x + blockIdx.x] = s1;
        }
    }
}


struct BlockArgs {
    const uint32_t *__restrict__ ent;    // per row: block-local internal hops, then external rows
    const uint16_t *__restrict__ nint;
    const uint16_t *__restrict__ next;
    const int32_t *__restrict__ bstart;
    int64_t dim_up, dim_dn;
    int w_up, nblocks, nslab;
    int contig;  // rows not on 128 bytes: each XCD takes a contiguous range of slabs
    double t;
    double amp[4];
};

// Blocked slab pass.  Workgroup b works on slab s and row block k, with
// xcd = b mod 8, s = (b / 8 / nblocks) * 8 + xcd, k = (b / 8) mod nblocks: the
// dispatcher starts workgroups in index order, so each XCD moves through its
// slabs about one at a time and the rows that other blocks' hops re-read are
// still in that XCD's L2.  A slab is 128 bytes of every row (one cache line).
// The workgroup stages its block's slab segment in LDS; hops that stay inside
// the block read LDS, the others read global memory.  Eight lanes cover one
// 128-byte row segment with 16-byte accesses, so a wave updates eight rows.
template <typename T, int MODE, bool GT>
__global__ __launch_bounds__(1024) void hv_blocks_kernel(BlockArgs p, const T *__restrict__ x, int64_t ldx,
                                                         T *__restrict__ y, int64_t ldy, double alpha,
                                                         const double *__restrict__ coef,
                                                         double *__restrict__ partials)
{
    constexpr int EPL = 16 / (int)sizeof(T);  // elements per lane
    constexpr int SL = 8 * EPL;               // slab width in elements
    typedef __attribute__((ext_vector_type(EPL))) T vec;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    vec *xs = reinterpret_cast<vec *>(smem_raw);  // [row in block][8]
    // 16-byte load of row elements d..d+EPL-1; past the last column the
    // elements are read one by one (and read as zero), so no access leaves the row
    auto load_row = [&](const T *row, int64_t d) -> vec {
        if (d + EPL <= p.dim_dn)
            return *reinterpret_cast<const vec *>(row + d);
        vec v;
#pragma unroll
        for (int e = 0; e < EPL; e++)
            v[e] = d + e < p.dim_dn ? row[d + e] : (T)0;
        return v;
    };
    __shared__ double red[16];
    if (MODE == HV_LANCZOS)
        alpha = coef[0];
    else if (MODE == HV_FUSED)
        alpha = coef[1];
    const T a_s = (T)alpha, tp = (T)p.t;
    const T am[4] = {(T)p.amp[0], (T)p.amp[1], (T)p.amp[2], (T)p.amp[3]};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwave = blockDim.x >> 6;
    const int xcd = blockIdx.x & 7;
    const int local = blockIdx.x >> 3;
    // slab-major per XCD: XCD k takes slabs k, k + 8, ... (rows on 128 bytes),
    // or the k-th contiguous range of slabs, so that the cache lines two
    // neighbouring slabs share stay in one L2 (rows not on 128 bytes)
    const int s = p.contig ? xcd * ((p.nslab + 7) / 8) + local / p.nblocks : (local / p.nblocks) * 8 + xcd;
    const int blk = local % p.nblocks;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (s < p.nslab) {
        const int64_t b0 = p.bstart[blk];
        const int bs = p.bstart[blk + 1] - (int)b0;
        const int64_t d0 = (int64_t)s * SL;
        // the block's slab segment: eight loads in flight per thread before
        // the first LDS write
        for (int i0 = 0; i0 < bs * 8; i0 += 8 * (int)blockDim.x) {
            vec v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                v[u] = i < bs * 8 ? load_row(x + (b0 + (i >> 3)) * ldx, d0 + (i & 7) * EPL) : (vec)(T)0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i < bs * 8)
                    xs[i] = v[u];
            }
        }
        __syncthreads();
        const int sub = lane >> 3, q = lane & 7;
        const int64_t d = d0 + q * EPL;
        for (int rb = wave * 8; rb < bs; rb += nwave * 8) {
            const int rl = min(rb + sub, bs - 1);
            const bool okr = rb + sub < bs;
            const int64_t r = b0 + rl;
            const uint32_t *__restrict__ er = p.ent + r * p.w_up;
            const int ni = p.nint[r], ne = p.next[r];
            int nim = ni, nem = ne;
            for (int o = 8; o < 64; o <<= 1) {
                nim = max(nim, __shfl_xor(nim, o, 64));
                nem = max(nem, __shfl_xor(nem, o, 64));
            }
            vec acc = (vec)(T)0;
            for (int k0 = 0; k0 < nim; k0 += 8) {
                int li[8];
                T cf[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const bool live = k0 + u < ni;
                    const uint32_t e = er[live ? k0 + u : 0];
                    li[u] = live ? (int)(e & (GT ? kGtRowMask : 0x7fffffffu)) : rl;
                    const T ap = GT ? class_amp(am, (e >> 24) & 3u) : tp;
                    cf[u] = live ? ((e >> 31) ? ap : -ap) : (T)0;
                }
                vec v[8];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    v[u] = xs[li[u] * 8 + q];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    acc += cf[u] * v[u];
            }
            for (int k0 = 0; k0 < nem; k0 += 8) {
                int64_t off[8];
                T cf[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const bool live = k0 + u < ne;
                    const uint32_t e = er[live ? ni + k0 + u : 0];
                    off[u] = (live ? (int64_t)(e & (GT ? kGtRowMask : 0x7fffffffu)) : r) * ldx;
                    const T ap = GT ? class_amp(am, (e >> 24) & 3u) : tp;
                    cf[u] = live ? ((e >> 31) ? ap : -ap) : (T)0;
                }
                vec v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    // slots past this row's external count issue no load
                    v[u] = (vec)(T)0;
                    if (k0 + u < ne)
                        v[u] = load_row(x + off[u], d);
                }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    acc += cf[u] * v[u];
            }
            if (okr && d < p.dim_dn) {
                T *yp = y + r * ldy + d;
                const vec xv = xs[rl * 8 + q];
                const bool whole = d + EPL <= p.dim_dn;
                vec prev;
                if (whole) {
                    prev = __builtin_nontemporal_load(reinterpret_cast<const vec *>(yp));
                } else {
#pragma unroll
                    for (int e = 0; e < EPL; e++)
                        prev[e] = d + e < p.dim_dn ? yp[e] : (T)0;
                }
                vec out;
                if (MODE == HV_STORE)
                    out = prev + acc;
                else if (MODE == HV_LANCZOS || MODE == HV_FUSED)
                    out = prev + a_s * acc;
                else
                    out = prev + acc;  // H x - alpha x
#pragma unroll
                for (int e = 0; e < EPL; e++) {
                    if (d + e < p.dim_dn) {
                        if (MODE == HV_LANCZOS) {
                            acc0 += (double)out[e] * (double)xv[e];
                        } else if (MODE == HV_FUSED) {
                            acc0 += (double)out[e] * (double)xv[e];
                            acc1 += (double)out[e] * (double)out[e];
                            acc2 += (double)xv[e] * (double)xv[e];
                        } else if (MODE == HV_RESIDUAL) {
                            acc0 += (double)out[e] * (double)out[e];
                            acc1 += (double)xv[e] * ((double)out[e] + alpha * (double)xv[e]);
                        }
                    }
                }
                if (MODE != HV_RESIDUAL) {
                    if (whole) {
                        __builtin_nontemporal_store(out, reinterpret_cast<vec *>(yp));
                    } else {
#pragma unroll
                        for (int e = 0; e < EPL; e++)
                            if (d + e < p.dim_dn)
                                yp[e] = out[e];
                    }
                }
            }
        }
    }
    if (MODE != HV_STORE) {
        const double s0 = block_sum2(acc0, red);
        if (threadIdx.x == 0)
            partials[blockIdx.x] = s0;
        if (MODE == HV_RESIDUAL || MODE == HV_FUSED) {
            const double s1 = block_sum2(acc1, red);
            if (threadIdx.x == 0)
                partials[gridDim.x + blockIdx.x] = s1;
        }
        if (MODE == HV_FUSED) {
            const double s2 = block_sum2(acc2, red);
            if (threadIdx.x == 0)
                partials[2 * gridDim.x + blockIdx.x] = s2;
        }
    }
}

struct LineArgs {
    const uint4 *__restrict__ line;    // per row: 32 slots = 8 x uint4
    const uint32_t *__restrict__ cnt;  // per row: internal, external hops, their maxima over the row's group of eight (bytes 0..3)
    const int32_t *__restrict__ bstart;
    int64_t dim_up, dim_dn;
    int nblocks, nslab;
    int contig;  // rows not on 128 bytes: each XCD takes a contiguous range of slabs
    double t;
    double amp[4];
    void *yo;      // where the result goes (y itself, or rows at stride ldyo)
    int64_t ldyo;
    int yoal;      // alignment of the result rows: 16 or 8 bytes (vector stores), else 0
    HvDefl defl;   // HV_FUSED_DEFL: the lower vectors psi_l . y and psi_l . x are summed against
    int64_t pair;  // 0, or the element offset of a second vector pair (x, y, result): workgroups
                   // from gpair on take it, and the partial sums cover both
    int gpair;
};

// Blocked slab pass, line layout (rows of at most 64 hops).  Same workgroup
// numbering and LDS staging as hv_blocks_kernel, plus a zero row after the
// block that padding hops point at.  A row's entries are one 128-byte line
// (internal hops from the front, external from the back): each of the eight
// lanes of a row group loads its own 16 bytes of it and a hop's entry reaches
// the other lanes by a permute within the group, so the line costs one load
// instead of eight.  The next row group's line, hop counts (one word, which
// also carries the group's largest counts) and running output are loaded one
// step ahead, which leaves the external rows as the only memory round trip of
// a step.  A hop adds its row with one FMA by +-1 (the factor's high word is
// the entry's sign bit or-ed into that of 1.0); -t (and alpha) multiply the
// sum once.  External rows are read four at a time, from 32-bit byte offsets
// where the vector allows (X32).  Padded lines (IPAD) let the internal slots
// be read without a per-slot test.  Workgroups whose slab lies inside the
// rows test no bounds; the slab at the rows' ends tests each lane.
// W = 32: one 128-byte line per row; W = 64 (rows of 33 to 64 hops): two lines,
// lane q of a row group holding slots 4q..4q+3 of each.
template <typename T, int MODE, bool GT, int W, bool IPAD, bool X32>
__global__ __launch_bounds__(1024) void hv_lines_kernel(LineArgs p, const T *__restrict__ x, int64_t ldx,
                                                        T *__restrict__ y, int64_t ldy, double alpha,
                                                        const double *__restrict__ coef,
                                                        double *__restrict__ partials)
{
    constexpr int EPL = 16 / (int)sizeof(T);  // elements per lane
    constexpr int SL = 8 * EPL;               // slab width in elements
    constexpr int XB = 4;                     // external rows in flight per lane
    typedef __attribute__((ext_vector_type(EPL))) T vec;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    vec *xs = reinterpret_cast<vec *>(smem_raw);  // [row in block][8], row bs = 0
    auto load_row = [&](const T *row, int64_t d) -> vec {
        if (d + EPL <= p.dim_dn)
            return *reinterpret_cast<const vec *>(row + d);
        vec v;
#pragma unroll
        for (int e = 0; e < EPL; e++)
            v[e] = d + e < p.dim_dn ? row[d + e] : (T)0;
        return v;
    };
    constexpr bool FUSED = MODE == HV_FUSED || MODE == HV_FUSED_DEFL;
    constexpr int ND = MODE == HV_FUSED_DEFL ? kFusedDefl : 0;  // slots for lower vectors
    if (MODE == HV_LANCZOS)
        alpha = coef[0];
    else if (FUSED)
        alpha = coef[1];
    // y += scale * sum_k (+-x_k): -t, times alpha in the Lanczos modes
    const double mt = GT ? -1.0 : -p.t;
    const T scale = (MODE == HV_LANCZOS || FUSED) ? (T)(alpha * mt) : (T)mt;
    // deflated step: shares of psi_l . y (du) and psi_l . x (dx)
    double du[ND > 0 ? ND : 1] = {}, dx[ND > 0 ? ND : 1] = {};
    const T am[4] = {(T)p.amp[0], (T)p.amp[1], (T)p.amp[2], (T)p.amp[3]};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwave = blockDim.x >> 6;
    int bid = (int)blockIdx.x;
    if (p.pair && bid >= p.gpair) {
        // the second vector pair (the imaginary halves of a complex vector)
        bid -= p.gpair;
        x += p.pair;
        y += p.pair;
        p.yo = static_cast<T *>(p.yo) + p.pair;
    }
    const int xcd = bid & 7;
    const int local = bid >> 3;
    // slab-major per XCD: XCD k takes slabs k, k + 8, ... (rows on 128 bytes),
    // or the k-th contiguous range of slabs, so that the cache lines two
    // neighbouring slabs share stay in one L2 (rows not on 128 bytes)
    const int s = p.contig ? xcd * ((p.nslab + 7) / 8) + local / p.nblocks : (local / p.nblocks) * 8 + xcd;
    const int blk = local % p.nblocks;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (s < p.nslab) {
        const int64_t b0 = p.bstart[blk];
        const int bs = p.bstart[blk + 1] - (int)b0;
        const int64_t d0 = (int64_t)s * SL;
        for (int i0 = 0; i0 < bs * 8; i0 += 8 * (int)blockDim.x) {
            vec v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                v[u] = i < bs * 8 ? load_row(x + (b0 + (i >> 3)) * ldx, d0 + (i & 7) * EPL) : (vec)(T)0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i < bs * 8)
                    xs[i] = v[u];
            }
        }
        if (threadIdx.x < 8)
            xs[bs * 8 + threadIdx.x] = (vec)(T)0;
        __syncthreads();
        const int sub = lane >> 3, q = lane & 7;
        const int64_t d = d0 + q * EPL;
        const bool dok = d < p.dim_dn, whole = d + EPL <= p.dim_dn;
        const int gbase = lane & ~7;
        const unsigned char *__restrict__ xb = reinterpret_cast<const unsigned char *>(x);
        const uint32_t rowb = (uint32_t)(ldx * (int64_t)sizeof(T)), colb = (uint32_t)(d * (int64_t)sizeof(T));
        // FULL: the slab lies inside the rows, so every lane's vector is whole
        // (rows start on 16 bytes) and no access needs a bounds test; the slab
        // holding the rows' ends tests each lane and never touches padding
        auto run = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            // running output of row r (zero past the last column)
            auto load_prev = [&](int64_t r) -> vec {
                const T *yp = y + r * ldy + d;
                if (FULL || whole)
                    return __builtin_nontemporal_load(reinterpret_cast<const vec *>(yp));
                vec v = (vec)(T)0;
                if (dok) {
#pragma unroll
                    for (int e = 0; e < EPL; e++)
                        v[e] = d + e < p.dim_dn ? yp[e] : (T)0;
                }
                return v;
            };
            // external row of entry e at this lane's columns: with X32 a 32-bit
            // byte offset from x (row and row stride below 2^24, the vector below
            // 4 GB) by one 24-bit multiply-add, which ignores the entry's sign
            // and class bits
            auto load_ext = [&](uint32_t e) -> vec {
                if (FULL && X32)
                    return *reinterpret_cast<const vec *>(xb + (__umul24(e, rowb) + colb));
                const T *row = x + (int64_t)(e & (GT ? kGtRowMask : 0x7fffffffu)) * ldx;
                if (FULL)
                    return *reinterpret_cast<const vec *>(row + d);
                return load_row(row, d);
            };
            // Lane q of a row group holds slots 4q..4q+3 of the row's line; entry
            // k reaches every lane of the group by a permute within the group.
            constexpr int NL = W / 32;  // 128-byte lines per row
            uint4 Em[NL];
#pragma unroll
            for (int h = 0; h < NL; h++)
                Em[h] = make_uint4(0u, 0u, 0u, 0u);
            uint32_t C = 0;
            vec prev = (vec)(T)0;
            int rb = wave * 8;
            if (rb < bs) {
                const int64_t r = b0 + min(rb + sub, bs - 1);
#pragma unroll
                for (int h = 0; h < NL; h++)
                    Em[h] = p.line[(r * NL + h) * 8 + q];
                C = p.cnt[r];
                if (rb + sub < bs)
                    prev = load_prev(r);
            }
            for (; rb < bs; rb += nwave * 8) {
                const int rl = min(rb + sub, bs - 1);
                const bool okr = rb + sub < bs;
                const int64_t r = b0 + rl;
                T *yp = static_cast<T *>(p.yo) + r * p.ldyo + d;
                // the lower vectors at this row's elements, loaded while the hops
                // are summed; the loads are unconditional (clamped in-bounds
                // indices, unused values weighted 0), so that waiting for them
                // never waits for the loads issued for the next row group
                double pv[ND > 0 ? ND : 1][EPL];
                if (ND > 0) {
#pragma unroll
                    for (int l = 0; l < ND; l++) {
                        const int lc = l < p.defl.nd ? l : 0;
                        const double *pr = p.defl.psi + (int64_t)lc * p.defl.pdim + r * p.dim_dn;
#pragma unroll
                        for (int e = 0; e < EPL; e++) {
                            const bool use = l < p.defl.nd && okr && (FULL || d + e < p.dim_dn);
                            const int64_t de = (FULL || d + e < p.dim_dn) ? d + e : p.dim_dn - 1;
                            pv[l][e] = pr[de] * (use ? 1.0 : 0.0);
                        }
                    }
                }
                const int ni = (int)(C & 0xffu), ne = (int)((C >> 8) & 0xffu);
                // the largest counts of the eight rows (the same in every lane)
                const int nim = __builtin_amdgcn_readfirstlane((int)((C >> 16) & 0xffu));
                const int nem = __builtin_amdgcn_readfirstlane((int)(C >> 24));
                // the next row group's entries, counts and running output, a
                // step ahead.  The loads are unconditional (past the block they
                // read its last row, unused), so the wait counters stay exact
                // and using this step's data never waits for them.
                uint4 En[NL];
                const int rbn = rb + nwave * 8;
                const int64_t rn = b0 + min(rbn + sub, bs - 1);
#pragma unroll
                for (int h = 0; h < NL; h++)
                    En[h] = p.line[(rn * NL + h) * 8 + q];
                const uint32_t Cn = p.cnt[rn];
                const vec prevn = load_prev(rn);
                auto entry = [&](int k) -> uint32_t {
                    const uint4 &E = Em[k >> 5];
                    const uint32_t c = (k & 3) == 0 ? E.x : (k & 3) == 1 ? E.y : (k & 3) == 2 ? E.z : E.w;
                    return (uint32_t)__builtin_amdgcn_ds_bpermute((gbase + ((k & 31) >> 2)) << 2, (int)c);
                };
                vec acc = (vec)(T)0;
                // internal hops, eight slots at a time.  Slot k past the row's
                // count reads the zero row: with padded lines (IPAD) the line
                // itself holds it up to the largest count of the group, so
                // only the group's last, partial chunk selects
                auto internal = [&](int k0, auto sel_tag) {
                    constexpr bool SEL = decltype(sel_tag)::value;
                    const int lim = IPAD ? nim : ni;
                    vec v[8];
                    uint32_t ev[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        ev[u] = entry(k0 + u);
                        const int li =
                            (!SEL || k0 + u < lim) ? (int)(ev[u] & (GT ? kGtRowMask : 0x7fffffffu)) : bs;
                        v[u] = xs[li * 8 + q];
                    }
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const T f = signed_factor<T, GT>(am, ev[u]);
#pragma unroll
                        for (int c = 0; c < EPL; c++)
                            acc[c] = fma(f, v[u][c], acc[c]);
                    }
                };
#pragma unroll
                for (int k0 = 0; k0 < W; k0 += 8) {
                    if (k0 < nim) {
                        if (IPAD && k0 + 8 <= nim)
                            internal(k0, std::false_type{});
                        else
                            internal(k0, std::true_type{});
                    }
                }
#pragma unroll
                for (int k0 = 0; k0 < W; k0 += XB) {
                    if (k0 < nem) {
                        vec v[XB];
                        uint32_t ev[XB];
#pragma unroll
                        for (int u = 0; u < XB; u++) {
                            ev[u] = entry(W - 1 - (k0 + u));
                            // slots past this row's external count issue no load
                            v[u] = (vec)(T)0;
                            if (k0 + u < ne)
                                v[u] = load_ext(ev[u]);
                        }
#pragma unroll
                        for (int u = 0; u < XB; u++) {
                            // and add nothing (factor 0)
                            const T f = k0 + u < ne ? signed_factor<T, GT>(am, ev[u]) : (T)0;
#pragma unroll
                            for (int c = 0; c < EPL; c++)
                                acc[c] = fma(f, v[u][c], acc[c]);
                        }
                    }
                }
                if (okr && (FULL || dok)) {
                    const vec xv = xs[rl * 8 + q];
                    const vec out = prev + scale * acc;  // in the residual mode prev = row pass of H x - alpha x
#pragma unroll
                    for (int e = 0; e < EPL; e++) {
                        if (FULL || d + e < p.dim_dn) {
                            if (MODE == HV_LANCZOS) {
                                acc0 += (double)out[e] * (double)xv[e];
                            } else if (FUSED) {
                                acc0 += (double)out[e] * (double)xv[e];
                                acc1 += (double)out[e] * (double)out[e];
                                acc2 += (double)xv[e] * (double)xv[e];
#pragma unroll
                                for (int l = 0; l < ND; l++) {
                                    du[l] += pv[l][e] * (double)out[e];
                                    dx[l] += pv[l][e] * (double)xv[e];
                                }
                            } else if (MODE == HV_RESIDUAL) {
                                acc0 += (double)out[e] * (double)out[e];
                                acc1 += (double)xv[e] * ((double)out[e] + alpha * (double)xv[e]);
                            }
                        }
                    }
                    if (MODE != HV_RESIDUAL) {
                        bool done = false;
                        if ((FULL || whole) && p.yoal == 16) {
                            __builtin_nontemporal_store(out, reinterpret_cast<vec *>(yp));
                            done = true;
                        }
                        if constexpr (EPL == 4) {
                            if (!done && (FULL || whole) && p.yoal == 8) {
                                // float rows on 8 bytes: two 8-byte stores
                                typedef __attribute__((ext_vector_type(2))) T vec2;
                                __builtin_nontemporal_store(vec2{out[0], out[1]}, reinterpret_cast<vec2 *>(yp));
                                __builtin_nontemporal_store(vec2{out[2], out[3]}, reinterpret_cast<vec2 *>(yp + 2));
                                done = true;
                            }
                        }
                        if (!done) {
#pragma unroll
                            for (int e = 0; e < EPL; e++)
                                if (d + e < p.dim_dn)
                                    yp[e] = out[e];
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < NL; h++)
                    Em[h] = En[h];
                C = Cn;
                prev = prevn;
            }
        };
        if (d0 + SL <= p.dim_dn)
            run(std::true_type{});
        else
            run(std::false_type{});
    }
    if (MODE != HV_STORE) {
        // all partial sums of the workgroup in one round: wave sums, one
        // barrier, then lane 0 of wave 0 adds the waves in a fixed order
        constexpr int NS = 3 + 2 * ND;
        __shared__ double red[NS][16];
        double sv[NS];
        sv[0] = wave_sum(acc0);
        sv[1] = (MODE == HV_RESIDUAL || FUSED) ? wave_sum(acc1) : 0.0;
        sv[2] = FUSED ? wave_sum(acc2) : 0.0;
#pragma unroll
        for (int l = 0; l < ND; l++) {
            sv[3 + 2 * l] = wave_sum(du[l]);
            sv[4 + 2 * l] = wave_sum(dx[l]);
        }
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < NS; k++)
                red[k][wave] = sv[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[NS];
#pragma unroll
            for (int k = 0; k < NS; k++)
                t[k] = 0.0;
            for (int w = 0; w < nwave; w++)
#pragma unroll
                for (int k = 0; k < NS; k++)
                    t[k] += red[k][w];
            partials[blockIdx.x] = t[0];
            if (MODE == HV_RESIDUAL || FUSED)
                partials[gridDim.x + blockIdx.x] = t[1];
            if (FUSED)
                partials[2 * gridDim.x + blockIdx.x] = t[2];
            // the deflated step's sums for the lower vectors it has
            for (int k = 3; k < 3 + 2 * p.defl.nd && k < NS; k++)
                partials[(int64_t)k * gridDim.x + blockIdx.x] = t[k];
        }
    }
}

template <typename T, int RPB>
size_t row_lds(int64_t ddn)
{
    return (size_t)RPB * (size_t)(ddn + 1) * sizeof(T);
}

}  // namespace

HvPlan make_hv_plan(const HvArgs &a, int elem_bytes)
{
    HvPlan pl;
    pl.elem_bytes = elem_bytes;
    const int64_t ddn = a.dim_dn;
    const size_t one_row = (size_t)(ddn + 1) * (size_t)elem_bytes;
    // per-bond amplitudes with more than four classes run the one-pass kernel:
    // the two-pass tables have room for two class bits
    pl.two_pass = one_row <= (size_t)kLdsBytes && (!a.tcls || a.ncls <= kTwoPassClasses);
    if (!pl.two_pass) {
        pl.ld = ddn;
        pl.nparts = hv_blocks(a, elem_bytes);
        return pl;
    }
    pl.ld = ((ddn + kSlab - 1) / kSlab) * kSlab;
    // rows per workgroup in the row pass: as many as fit in LDS, up to 3 (FP32) or 2 (FP64)
    int rpb = elem_bytes == 4 ? 3 : 2;
    while (rpb > 1 && one_row * (size_t)rpb > (size_t)kLdsBytes)
        rpb--;
    pl.rows_rpb = rpb;
    pl.rows_lds = one_row * (size_t)rpb;
    int64_t thr = ((ddn + 63) / 64) * 64;
    pl.rows_threads = (int)(thr < 1024 ? thr : 1024);
    int per_cu = 2048 / pl.rows_threads;
    int by_lds = (int)((size_t)kLdsBytes / pl.rows_lds);
    per_cu = by_lds < per_cu ? by_lds : per_cu;
    if (per_cu < 1)
        per_cu = 1;
    const int64_t groups = (a.dim_up + rpb - 1) / rpb;
    const int64_t cap = (int64_t)256 * per_cu;
    pl.rows_grid = (int)(groups < cap ? groups : cap);
    // slab pass: 8 XCDs x nw workgroups, each owning a block of rows
    int64_t nw = a.dim_up < 256 ? a.dim_up : 256;
    const int64_t wup = a.w_up > 0 ? a.w_up : 1;
    while (((a.dim_up + nw - 1) / nw) * (wup * 4 + 4) > 48 * 1024)
        nw *= 2;
    pl.slab_rw = (int)((a.dim_up + nw - 1) / nw);
    pl.slab_grid = (int)(8 * nw);
    pl.slab_lds = (size_t)pl.slab_rw * (size_t)(wup * 4 + 4);
    pl.nslab = (int)((ddn + kSlab - 1) / kSlab);
    pl.nparts = pl.slab_grid;
    // blocked slab pass: 128-byte slabs, one workgroup per (slab, row block)
    if (a.up_nblocks > 0 && a.up_max_block > 0) {
        const int sl = 128 / elem_bytes;
        pl.blk_nslab = (int)((ddn + sl - 1) / sl);
        const int64_t per_xcd = (pl.blk_nslab + 7) / 8;
        pl.blk_grid = (int)(8 * per_xcd * a.up_nblocks);
        // the line kernel stages a zero row after the block
        pl.blk_lds = (size_t)(a.up_max_block + (a.up_line ? 1 : 0)) * 128;
        const int64_t thr = ((int64_t)a.up_max_block * 8 + 63) / 64 * 64;
        pl.blk_threads = (int)(thr < 1024 ? (thr < 256 ? 256 : thr) : 1024);
        pl.nparts = std::max(pl.nparts, pl.blk_grid);
    }
    return pl;
}

template <typename T, int RPB>
static void launch_rows_rpb(const RowArgs &ra, bool g16, bool gt, const HvPlan &pl, const T *x, int64_t ldx, T *y,
                            int64_t ldy, int mode, double alpha, const double *coef, hipStream_t s)
{
    const size_t lds = row_lds<T, RPB>(ra.dim_dn);
    auto go = [&](auto kern) {
        HUB_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(pl.rows_grid), dim3(pl.rows_threads), lds, s, ra, x, ldx, y, ldy, alpha, 0.0,
                           coef);
        HUB_HIP(hipGetLastError());
    };
    // a column's groups fit the four registers loaded a column ahead
    const bool pf = ra.gmax <= 4;
    auto pick = [&](auto mc, auto g16c, auto gtc) {
        constexpr int M = decltype(mc)::value;
        constexpr bool G16 = decltype(g16c)::value, GT = decltype(gtc)::value;
        if constexpr (M == HV_FUSED_DEFL && GT)
            fail(HUBBARD_EDEVICE, "fused deflated step: per-bond amplitudes unsupported");
        else if (pf)
            go(hv_rows_kernel<T, RPB, M, G16, GT, true>);
        else
            go(hv_rows_kernel<T, RPB, M, G16, GT, false>);
    };
    using F = std::false_type;
    using Tr = std::true_type;
    auto by_mode = [&](auto g16c, auto gtc) {
        if (mode == HV_STORE)
            pick(std::integral_constant<int, HV_STORE>(), g16c, gtc);
        else if (mode == HV_LANCZOS)
            pick(std::integral_constant<int, HV_LANCZOS>(), g16c, gtc);
        else if (mode == HV_FUSED)
            pick(std::integral_constant<int, HV_FUSED>(), g16c, gtc);
        else if (mode == HV_FUSED_DEFL)
            pick(std::integral_constant<int, HV_FUSED_DEFL>(), g16c, gtc);
        else
            pick(std::integral_constant<int, HV_RESIDUAL>(), g16c, gtc);
    };
    // per-bond amplitudes use the 32-bit groups (the class sits above the offset)
    if (gt)
        by_mode(F(), Tr());
    else if (g16)
        by_mode(Tr(), F());
    else
        by_mode(F(), F());
}

// The FP64 row pass takes handles of one amplitude whose rows need the whole
// LDS (one row per workgroup) and fit kRow64Max elements.
static bool row64_ok(const HvArgs &a, const HvPlan &pl)
{
    // rows of up to 13 elements per thread are staged through registers
    return a.tcls == nullptr && a.dn_pidx != nullptr && pl.rows_rpb == 1 && a.w_dn <= 32 &&
           a.dim_dn <= 13 * kRowThreads;
}

// The FP64 row pass of hv_rows64_kernel: CH staging units per thread (16-byte
// pairs when x and y rows start on 16 bytes, else single elements); group
// slots for the table's largest counts (three groups of + hops and four of -
// hops cover the square lattices, eight of each any row of up to 32 hops).
template <int MODE, bool VEC, int CH>
static void launch_rows64_groups(const Row64Args &ra, int np, int nn, const HvPlan &pl, const double *x, int64_t ldx,
                                 double *y, int64_t ldy, double alpha, const double *coef, hipStream_t s)
{
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(pl.rows_grid), dim3(kRowThreads), 0, s, ra, x, ldx, y, ldy, alpha, 0.0, coef);
        HUB_HIP(hipGetLastError());
    };
    if (np <= 3 && nn <= 4)
        go(hv_rows64_kernel<MODE, VEC, CH, 3, 4>);
    else
        go(hv_rows64_kernel<MODE, VEC, CH, 4, 8>);
}

template <int MODE>
static void launch_rows64_mode(const Row64Args &ra, int np, int nn, const HvPlan &pl, const double *x, int64_t ldx,
                               double *y, int64_t ldy, double alpha, const double *coef, hipStream_t s)
{
    const bool vec = ((uintptr_t)x % 16 == 0) && ((uintptr_t)y % 16 == 0) && ldx % 2 == 0 && ldy % 2 == 0;
    const int64_t units = vec ? ra.dim_dn / 2 : ra.dim_dn;
    const int need = (int)((units + kRowThreads - 1) / kRowThreads);
    if (need > (vec ? 7 : 13))
        fail(HUBBARD_EDEVICE, "row too long for the FP64 row pass");
    if (np > 4 || nn > 8)
        fail(HUBBARD_EDEVICE, "too many hops per column for the FP64 row pass");
    if (vec)
        launch_rows64_groups<MODE, true, 7>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
    else
        launch_rows64_groups<MODE, false, 13>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
}

static void launch_rows64(const HvArgs &a, const HvPlan &pl, const double *x, int64_t ldx, double *y, int64_t ldy,
                          int mode, double alpha, const double *coef, hipStream_t s, double *xc, int64_t ldc,
                          const HvDefl &defl, double *yo, int64_t ldyo)
{
    Row64Args ra;
    ra.xc = xc;
    ra.ldc = ldc;
    ra.defl = defl;
    ra.yo = yo;
    ra.ldyo = ldyo;
    ra.pidx = a.dn_pidx;
    ra.nidx = a.dn_nidx;
    ra.pn = a.dn_pn;
    ra.states_up = a.states_up;
    ra.states_dn = a.states_dn;
    ra.dim_up = a.dim_up;
    ra.dim_dn = (int)a.dim_dn;
    ra.t = a.t;
    ra.U = a.U;
    const int np = a.dn_np, nn = a.dn_nn;
    if (mode == HV_STORE)
        launch_rows64_mode<HV_STORE>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
    else if (mode == HV_LANCZOS)
        launch_rows64_mode<HV_LANCZOS>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
    else if (mode == HV_FUSED)
        launch_rows64_mode<HV_FUSED>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
    else if (mode == HV_FUSED_DEFL)
        launch_rows64_mode<HV_FUSED_DEFL>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
    else
        launch_rows64_mode<HV_RESIDUAL>(ra, np, nn, pl, x, ldx, y, ldy, alpha, coef, s);
}

// The FP32 row pass on row pairs (hv_rows32x2_kernel): the same tables and
// conditions as the FP64 row pass (one amplitude, 16-bit indices, at most 32
// hops per column), any mode but the deflated step; one workgroup per CU.
static bool rows32x2_ok(const HvArgs &a, int mode)
{
    return a.tcls == nullptr && a.dn_pidx != nullptr && a.w_dn <= 32 && a.dim_dn <= 13 * kRowThreads &&
           mode != HV_FUSED_DEFL;
}

template <int MODE, bool VEC, int CH>
static void launch_rows32x2_groups(const Row32Args &ra, int np, int nn, const float *x, int64_t ldx, float *y,
                                   int64_t ldy, double alpha, const double *coef, hipStream_t s)
{
    const int64_t npair = (ra.dim_up + 1) / 2;
    const int grid = (int)(npair < 256 ? npair : 256);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kRowThreads), 0, s, ra, x, ldx, y, ldy, alpha, 0.0, coef);
        HUB_HIP(hipGetLastError());
    };
    if (np <= 3 && nn <= 4)
        go(hv_rows32x2_kernel<MODE, VEC, CH, 3, 4>);
    else
        go(hv_rows32x2_kernel<MODE, VEC, CH, 4, 8>);
}

template <int MODE>
static void launch_rows32x2_mode(const Row32Args &ra, int np, int nn, const float *x, int64_t ldx, float *y,
                                 int64_t ldy, double alpha, const double *coef, hipStream_t s)
{
    // 8-byte units where every row starts on 8 bytes
    bool vec = ((uintptr_t)x % 8 == 0) && ((uintptr_t)y % 8 == 0) && ldx % 2 == 0 && ldy % 2 == 0;
    if (ra.xc)
        vec = vec && (uintptr_t)ra.xc % 8 == 0 && ra.ldc % 2 == 0;
    const int64_t units = vec ? ra.dim_dn / 2 : ra.dim_dn;
    const int need = (int)((units + kRowThreads - 1) / kRowThreads);
    if (need > (vec ? 7 : 13))
        fail(HUBBARD_EDEVICE, "row too long for the FP32 row-pair pass");
    if (np > 4 || nn > 8)
        fail(HUBBARD_EDEVICE, "too many hops per column for the FP32 row-pair pass");
    if (vec)
        launch_rows32x2_groups<MODE, true, 7>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
    else
        launch_rows32x2_groups<MODE, false, 13>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
}

static void launch_rows32x2(const HvArgs &a, const float *x, int64_t ldx, float *y, int64_t ldy, int mode,
                            double alpha, const double *coef, hipStream_t s, float *xc, int64_t ldc, float *yo,
                            int64_t ldyo)
{
    Row32Args ra;
    ra.pidx = a.dn_pidx;
    ra.nidx = a.dn_nidx;
    ra.pn = a.dn_pn;
    ra.states_up = a.states_up;
    ra.states_dn = a.states_dn;
    ra.dim_up = a.dim_up;
    ra.dim_dn = (int)a.dim_dn;
    ra.t = a.t;
    ra.U = a.U;
    ra.xc = xc;
    ra.ldc = ldc;
    ra.yo = yo;
    ra.ldyo = ldyo;
    const int np = a.dn_np, nn = a.dn_nn;
    if (mode == HV_STORE)
        launch_rows32x2_mode<HV_STORE>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
    else if (mode == HV_LANCZOS)
        launch_rows32x2_mode<HV_LANCZOS>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
    else if (mode == HV_FUSED)
        launch_rows32x2_mode<HV_FUSED>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
    else
        launch_rows32x2_mode<HV_RESIDUAL>(ra, np, nn, x, ldx, y, ldy, alpha, coef, s);
}

template <typename T>
int launch_hv2(const HvArgs &a, const HvPlan &pl, const T *x, int64_t ldx, T *y, int64_t ldy, T *scratch,
               int64_t lds_, int mode, double alpha, const double *coef, double *partials, hipStream_t s, T *xpad,
               T *ypad, const HvDefl *defl, T *yout, int64_t pair)
{
    if (!pl.two_pass) {
        // rows too wide for LDS: the one-pass kernel (dense rows only)
        if (mode == HV_RESIDUAL)
            launch_hv<T>(a, x, nullptr, HV_RESIDUAL, alpha, coef, partials, pl.nparts, s);
        else
            launch_hv<T>(a, x, y, mode, alpha, coef, partials, pl.nparts, s);
        return pl.nparts;
    }
    RowArgs ra;
    const bool gt = a.tcls != nullptr;
    const bool g16 = !gt && a.dn_groups16 != nullptr;
    for (int c = 0; c < 4; c++)
        ra.amp[c] = a.amp4[c];
    ra.groups = g16 ? a.dn_groups16 : (sizeof(T) == 8 ? a.dn_groups64 : a.dn_groups32);
    ra.nq = g16 ? a.dn_nq8 : a.dn_nq;
    ra.states_up = a.states_up;
    ra.states_dn = a.states_dn;
    ra.dim_up = a.dim_up;
    ra.dim_dn = a.dim_dn;
    ra.ngroups = a.dn_ngroups;
    ra.gmax = g16 ? std::max((a.w_dn + 7) / 8, 1) : std::max(a.dn_ngroups, 1);
    ra.t = a.t;
    ra.U = a.U;
    T *yr = mode == HV_RESIDUAL ? scratch : y;
    int64_t ldyr = mode == HV_RESIDUAL ? lds_ : ldy;
    T *yo = y;  // where the up-spin pass writes the result
    int64_t ldyo = ldy;
    // Rows not on 128 bytes (a caller's dense vector) with padded work rows
    // given: the row pass writes its result to the padded rows and copies each
    // staged row of x beside it, so the up-spin pass runs on cache-line slabs
    // and writes the sum straight to y.
    const int64_t slw = 128 / (int64_t)sizeof(T), v16 = 16 / (int64_t)sizeof(T);
    const bool dense = ldx % slw != 0 || ldyr % slw != 0;
    const bool repad = pl.blk_grid > 0 && a.up_line && dense && xpad &&
                       (mode == HV_STORE ? ypad != nullptr : mode == HV_RESIDUAL);
    ra.xc = repad ? xpad : nullptr;
    ra.ldc = pl.ld;
    const HvDefl dfl = defl ? *defl : HvDefl();
    if (mode == HV_FUSED_DEFL && (gt || !a.up_line || !(dfl.nd >= 1 && dfl.nd <= kFusedDefl) || !dfl.psi || !dfl.g))
        fail(HUBBARD_EDEVICE, "fused deflated step: unsupported plan or deflation data");
    ra.defl = dfl;
    const bool fusedm = mode == HV_FUSED || mode == HV_FUSED_DEFL;
    if ((yout || pair) && !(fusedm && !repad && a.up_line))
        fail(HUBBARD_EDEVICE, "a separate result and vector pairs need a fused step on the line layout");
    ra.yo = yout;
    ra.ldyo = ldy;
    if (repad && mode == HV_STORE) {
        yr = ypad;
        ldyr = pl.ld;
    }
    // the row pass, once per vector pair
    for (int half = 0; half < (pair ? 2 : 1); half++) {
        const int64_t o = half ? pair : 0;
        RowArgs rh = ra;
        if (yout)
            rh.yo = yout + o;
        if (sizeof(T) == 8 && row64_ok(a, pl))
            launch_rows64(a, pl, reinterpret_cast<const double *>(x + o), ldx, reinterpret_cast<double *>(yr + o), ldyr,
                          mode, alpha, coef, s, reinterpret_cast<double *>(ra.xc), ra.ldc, dfl,
                          reinterpret_cast<double *>(rh.yo), ldy);
        else if (sizeof(T) == 4 && rows32x2_ok(a, mode))
            launch_rows32x2(a, reinterpret_cast<const float *>(x + o), ldx, reinterpret_cast<float *>(yr + o), ldyr,
                            mode, alpha, coef, s, reinterpret_cast<float *>(ra.xc), ra.ldc,
                            reinterpret_cast<float *>(rh.yo), ldy);
        else if (pl.rows_rpb == 3)
            launch_rows_rpb<T, 3>(rh, g16, gt, pl, x + o, ldx, yr + o, ldyr, mode, alpha, coef, s);
        else if (pl.rows_rpb == 2)
            launch_rows_rpb<T, 2>(rh, g16, gt, pl, x + o, ldx, yr + o, ldyr, mode, alpha, coef, s);
        else
            launch_rows_rpb<T, 1>(rh, g16, gt, pl, x + o, ldx, yr + o, ldyr, mode, alpha, coef, s);
    }
    if (yout) {
        // the up-spin pass adds to the result rows
        yr = yout;
        yo = yout;
    }

    if (repad) {
        x = xpad;
        ldx = pl.ld;
    }
    // the blocked passes load 16 bytes per lane: rows must start on 16 bytes
    // (on 128 bytes each row segment is one cache line)
    const bool on16 = ldx % v16 == 0 && ldyr % v16 == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)yr % 16 == 0;
    const int contig = (ldx % slw != 0 || ldyr % slw != 0 || (mode != HV_RESIDUAL && ldyo % slw != 0)) ? 1 : 0;
    if (pl.blk_grid > 0 && on16) {
        BlockArgs ba;
        ba.ent = a.up_blk;
        ba.nint = a.up_nint;
        ba.next = a.up_next;
        ba.bstart = a.up_bstart;
        ba.dim_up = a.dim_up;
        ba.dim_dn = a.dim_dn;
        ba.w_up = a.w_up > 0 ? a.w_up : 1;
        ba.nblocks = a.up_nblocks;
        ba.nslab = pl.blk_nslab;
        ba.contig = contig;
        ba.t = a.t;
        for (int c = 0; c < 4; c++)
            ba.amp[c] = a.amp4[c];
        auto gob = [&](auto kern) {
            if (pl.blk_lds > 64 * 1024)
                HUB_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)pl.blk_lds));
            hipLaunchKernelGGL(kern, dim3(pl.blk_grid), dim3(pl.blk_threads), pl.blk_lds, s, ba, x, ldx, yr, ldyr,
                               alpha, coef, partials);
            HUB_HIP(hipGetLastError());
        };
        if (a.up_line) {
            LineArgs la;
            la.line = reinterpret_cast<const uint4 *>(a.up_line);
            la.cnt = a.up_cnt;
            la.bstart = a.up_bstart;
            la.dim_up = a.dim_up;
            la.dim_dn = a.dim_dn;
            la.nblocks = a.up_nblocks;
            la.nslab = pl.blk_nslab;
            la.contig = contig;
            la.t = a.t;
            la.yo = yo;
            la.ldyo = ldyo;
            la.defl = dfl;
            la.pair = pair;
            la.gpair = pl.blk_grid;
            la.yoal = ((uintptr_t)yo % 16 == 0 && ldyo % v16 == 0)                         ? 16
                      : ((uintptr_t)yo % 8 == 0 && (ldyo * (int64_t)sizeof(T)) % 8 == 0) ? 8
                                                                                         : 0;
            const bool w64 = a.up_line_w == 64;
            for (int c = 0; c < 4; c++)
                la.amp[c] = a.amp4[c];
            auto gol = [&](auto kern) {
                if (pl.blk_lds > 64 * 1024)
                    HUB_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)pl.blk_lds));
                hipLaunchKernelGGL(kern, dim3(pl.blk_grid * (pair ? 2 : 1)), dim3(pl.blk_threads), pl.blk_lds, s, la,
                                   x, ldx, yr, ldyr, alpha, coef, partials);
                HUB_HIP(hipGetLastError());
            };
            // 32-bit external offsets: rows and row stride below 2^24, x below 4 GB
            const int64_t rowb = ldx * (int64_t)sizeof(T);
            const bool x32 = a.dim_up < (1 << 24) && rowb < (1 << 24) && a.dim_up * rowb < ((int64_t)1 << 32);
            const bool ipad = a.up_line_ipad != 0;
            auto pick = [&](auto mode_tag) {
                constexpr int M = decltype(mode_tag)::value;
                if constexpr (M == HV_FUSED_DEFL) {
                    // one amplitude only (checked above)
                    if (!w64)
                        (ipad && x32) ? gol(hv_lines_kernel<T, M, false, 32, true, true>)
                                      : gol(hv_lines_kernel<T, M, false, 32, false, false>);
                    else
                        (ipad && x32) ? gol(hv_lines_kernel<T, M, false, 64, true, true>)
                                      : gol(hv_lines_kernel<T, M, false, 64, false, false>);
                } else if (gt)
                    w64 ? gol(hv_lines_kernel<T, M, true, 64, false, false>)
                        : gol(hv_lines_kernel<T, M, true, 32, false, false>);
                else if (!w64)
                    (ipad && x32) ? gol(hv_lines_kernel<T, M, false, 32, true, true>)
                                  : gol(hv_lines_kernel<T, M, false, 32, false, false>);
                else if (x32)
                    ipad ? gol(hv_lines_kernel<T, M, false, 64, true, true>)
                         : gol(hv_lines_kernel<T, M, false, 64, false, true>);
                else
                    gol(hv_lines_kernel<T, M, false, 64, false, false>);
            };
            if (mode == HV_STORE)
                pick(std::integral_constant<int, HV_STORE>{});
            else if (mode == HV_LANCZOS)
                pick(std::integral_constant<int, HV_LANCZOS>{});
            else if (mode == HV_FUSED)
                pick(std::integral_constant<int, HV_FUSED>{});
            else if (mode == HV_FUSED_DEFL)
                pick(std::integral_constant<int, HV_FUSED_DEFL>{});
            else
                pick(std::integral_constant<int, HV_RESIDUAL>{});
            return pl.blk_grid * (pair ? 2 : 1);
        }
        if (mode == HV_STORE)
            gt ? gob(hv_blocks_kernel<T, HV_STORE, true>) : gob(hv_blocks_kernel<T, HV_STORE, false>);
        else if (mode == HV_LANCZOS)
            gt ? gob(hv_blocks_kernel<T, HV_LANCZOS, true>) : gob(hv_blocks_kernel<T, HV_LANCZOS, false>);
        else if (mode == HV_FUSED)
            gt ? gob(hv_blocks_kernel<T, HV_FUSED, true>) : gob(hv_blocks_kernel<T, HV_FUSED, false>);
        else
            gt ? gob(hv_blocks_kernel<T, HV_RESIDUAL, true>) : gob(hv_blocks_kernel<T, HV_RESIDUAL, false>);
        return pl.blk_grid;
    }
    if (mode == HV_FUSED || mode == HV_FUSED_DEFL)
        fail(HUBBARD_EDEVICE, "fused Lanczos step needs rows aligned to 16 bytes");

    SlabArgs sa;
    sa.up_rows = a.up_rows;
    sa.nnz_up = a.nnz_up;
    sa.dim_up = a.dim_up;
    sa.dim_dn = a.dim_dn;
    sa.w_up = a.w_up > 0 ? a.w_up : 1;
    sa.rows_per_wg = pl.slab_rw;
    sa.nslab = pl.nslab;
    sa.t = a.t;
    for (int c = 0; c < 4; c++)
        sa.amp[c] = a.amp4[c];
    auto go = [&](auto kern) {
        if (pl.slab_lds > 64 * 1024)
            HUB_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)pl.slab_lds));
        hipLaunchKernelGGL(kern, dim3(pl.slab_grid), dim3(kSlabThreads), pl.slab_lds, s, sa, x, ldx, yr, ldyr, alpha,
                           coef, partials);
        HUB_HIP(hipGetLastError());
    };
    if (mode == HV_STORE)
        gt ? go(hv_slabs_kernel<T, HV_STORE, true>) : go(hv_slabs_kernel<T, HV_STORE, false>);
    else if (mode == HV_LANCZOS)
        gt ? go(hv_slabs_kernel<T, HV_LANCZOS, true>) : go(hv_slabs_kernel<T, HV_LANCZOS, false>);
    else
        gt ? go(hv_slabs_kernel<T, HV_RESIDUAL, true>) : go(hv_slabs_kernel<T, HV_RESIDUAL, false>);
    return pl.slab_grid;
}

template int launch_hv2<double>(const HvArgs &, const HvPlan &, const double *, int64_t, double *, int64_t, double *,
                                int64_t, int, double, const double *, double *, hipStream_t, double *, double *,
                                const HvDefl *, double *, int64_t);
template int launch_hv2<float>(const HvArgs &, const HvPlan &, const float *, int64_t, float *, int64_t, float *,
                               int64_t, int, double, const double *, double *, hipStream_t, float *, float *,
                               const HvDefl *, float *, int64_t);

}  // namespace hub
