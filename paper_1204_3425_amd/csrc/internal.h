// Internal declarations of the Hubbard library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hubbard.h"

namespace hub {

// Error raised inside the library; converted to a return code at the ABI.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HUB_HIP(call) ::hub::hip_check((call), #call)

// One spin's basis and hopping table as built on the host.
struct SpinTable {
    int n = 0;                      // electrons of this spin
    int64_t dim = 0;                // C(sites, n)
    int32_t width = 0;              // ELL width = max entries of a row
    int64_t nnz = 0;
    std::vector<uint32_t> states;   // ascending configuration words
    std::vector<int32_t> col;       // column-major ELL: entry k of row r at k*dim + r
    std::vector<int8_t> sgn;        // +1 / -1, padding 0
    std::vector<uint16_t> row_nnz;  // entries used in each row
    std::vector<uint16_t> bond;     // column-major like col: the bond (edge index) of each entry
};

// Packed device form of a hopping entry: bits 0..30 column, bit 31 set when
// the element is +t (sgn = -1).
inline uint32_t pack_entry(int32_t col, int8_t sgn) { return (uint32_t)col | (sgn < 0 ? 0x80000000u : 0u); }
// With per-bond amplitudes (columns below 2^24): bits 24..30 hold the
// amplitude class, the element is -tcls[class] * sgn.
inline uint32_t pack_entry_class(int32_t col, int8_t sgn, int cls)
{
    return (uint32_t)col | ((uint32_t)cls << 24) | (sgn < 0 ? 0x80000000u : 0u);
}
constexpr uint32_t kClassColMask = 0x00FFFFFFu;
constexpr int kMaxAmpClasses = 127;
// per-bond handles with at most this many classes also get the two-pass tables
// (two class bits in the row-pass groups and the up-spin entries)
constexpr int kTwoPassClasses = 4;
// longest row the FP64 row pass stages in LDS (plus one zero slot: 160 KB)
constexpr int kRow64Max = 20000;

struct DeviceTables {
    uint32_t *states_up = nullptr, *states_dn = nullptr;
    uint32_t *up_rows = nullptr;   // row-major: entry k of row r at r*w_up + k (row entries are wave-uniform)
    uint32_t *dn_cols = nullptr;   // column-major: entry k of row d at k*dim_dn + d (coalesced across lanes)
    uint16_t *nnz_up = nullptr, *nnz_dn = nullptr;
    // down table for the row pass: groups of four entries holding the byte
    // offset of the source element in a staged row (FP64 and FP32 layouts),
    // sign in bit 31, padding pointing at the zero slot after the row
    uint32_t *dn_groups64 = nullptr, *dn_groups32 = nullptr;
    uint8_t *dn_nq = nullptr;      // groups needed by the 64 columns of a wave
    int dn_ngroups = 0;
    // the same table at half the size, for rows of at most 32767 elements:
    // groups of eight 16-bit entries (element index | sign<<15)
    uint16_t *dn_groups16 = nullptr;
    uint8_t *dn_nq8 = nullptr;     // groups of eight needed by the 64 columns of a wave
    // FP64 row pass (one amplitude, rows of at most kRow64Max elements): per
    // column the hops of sign + in groups of eight 16-bit element indices and
    // those of sign - in groups of four, each in ascending column order
    // (padding: the zero slot at index dim_dn), and per 64 columns the two
    // group counts (one byte each); dn_np, dn_nn: the largest counts
    uint16_t *dn_pidx = nullptr, *dn_nidx = nullptr;
    uint8_t *dn_pn = nullptr;
    int dn_np = 0, dn_nn = 0;
    // up table for the blocked slab pass: rows are grouped in blocks of equal
    // occupation of the top sites; per row the hops that stay in the block come
    // first (block-local row | sign<<31), then the others (row | sign<<31)
    uint32_t *up_blk = nullptr;
    uint16_t *up_nint = nullptr, *up_next = nullptr;
    int32_t *up_bstart = nullptr;  // nblocks + 1 row offsets
    int up_nblocks = 0, up_max_block = 0;
    // the same entries with one 32-slot line per row (two, 64 slots, for rows
    // of 33 to 64 hops, or where 32 slots leave no room for the padding):
    // internal hops from the front, external from the back; per row one word
    // with the internal and external counts and their largest values over the
    // row's group of eight (bytes 0..3).  Padded lines (up_line_ipad): the
    // slots past a row's internal count, up to the largest count of its group,
    // hold the block's zero row
    uint32_t *up_line = nullptr, *up_cnt = nullptr;
    size_t bytes = 0;
    double *tcls = nullptr;  // amplitude of each class (per-bond amplitudes only)
    int up_line_w = 32;      // slots per row of up_line (32 or 64)
    int up_line_ipad = 0;
};

}  // namespace hub

struct hubbard {
    int sites = 0, n_up = 0, n_dn = 0;
    double t = 0, U = 0;
    std::vector<int32_t> edges;  // 2 per bond
    hub::SpinTable up, dn;
    int64_t dim = 0;
    hub::DeviceTables dev;
    std::vector<double> tcls;      // per-bond amplitudes: distinct values (empty: one amplitude t)
    std::vector<uint8_t> bond_cls; // class of each bond
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = HUBBARD_FP64;
    uint64_t seed = 12043425ull;
    // device bytes a solve with psi may hold for its resident Lanczos basis
    size_t basis_limit = SIZE_MAX;
    // padded work rows for hubbard_apply on rows not on 128 bytes (two vectors
    // at the library's row stride, allocated on first use), and the event of
    // their last use, so that a call on another stream waits for it
    void *apply_work = nullptr;
    size_t apply_work_bytes = 0;
    hipEvent_t apply_ev = nullptr;
};

namespace hub {

// capi.cpp: the single-instance Lanczos driver (throws hub::Error)
void validate_opts(const hubbard_opts &o);
int lanczos_impl(hubbard *h, const hubbard_opts &o, hubbard_result *res);

// builder.cpp
void build_spin_table(int sites, const std::vector<int32_t> &edges, int n, SpinTable &out);
uint64_t binomial(int n, int k);

// tridiag.cpp: symmetric tridiagonal T with diagonal d[0..m-1] and
// off-diagonal e[i] between rows i and i+1 (i < m-1).
double tridiag_lowest(const double *d, const double *e, int m);
void tridiag_lowest_vector(const double *d, const double *e, int m, double lam, double *y);
// c = exp(-i tau T) e_1 (real and imaginary parts, m each); e holds the m-1 off-diagonals
void tridiag_expm_e1(const double *d, const double *e, int m, double tau, double *c_re, double *c_im);

// kernels.hip: launchers (all asynchronous on `s`).
struct HvArgs {
    // per-bond amplitudes: the distinct values, indexed by the class bits of
    // up_rows / dn_cols entries (NULL: every hop has amplitude t)
    const double *tcls = nullptr;
    int ncls = 0;
    double amp4[4] = {0.0, 0.0, 0.0, 0.0};  // the classes, for the two-pass kernels (ncls <= kTwoPassClasses)
    int up_line_w = 32;  // slots per row of up_line: 32 (one 128-byte line) or 64 (two)
    int up_line_ipad = 0;  // internal slots padded with the zero row up to the group's largest count
    const uint32_t *states_up, *states_dn, *up_rows, *dn_cols;
    const uint16_t *nnz_up, *nnz_dn;
    const uint4 *dn_groups64, *dn_groups32;
    const uint8_t *dn_nq;
    int dn_ngroups;
    const uint4 *dn_groups16;  // null when rows exceed 32767 elements
    const uint8_t *dn_nq8;
    const uint4 *dn_pidx = nullptr;       // FP64 row pass: + hops, eight per group (null: not built)
    const uint2 *dn_nidx = nullptr;       // - hops, four per group
    const uint8_t *dn_pn = nullptr;       // group counts per 64 columns
    int dn_np = 0, dn_nn = 0;             // their largest values
    const uint32_t *up_blk;
    const uint16_t *up_nint, *up_next;
    const int32_t *up_bstart;
    int up_nblocks, up_max_block;
    const uint32_t *up_line, *up_cnt;  // null when a row has more than 64 hops
    int64_t dim_up, dim_dn;
    int32_t w_up, w_dn;
    double t, U;
};

// Launch shape of the two-pass H.v for one element size (hv.hip).
struct HvPlan {
    int elem_bytes = 8;
    bool two_pass = false;  // false: rows too wide for LDS, one-pass kernel
    int64_t ld = 0;         // row stride of internal vectors (elements)
    int rows_rpb = 1, rows_threads = 64, rows_grid = 1;
    size_t rows_lds = 0;
    int slab_rw = 1, slab_grid = 8, nslab = 1;
    size_t slab_lds = 0;
    int blk_grid = 0, blk_nslab = 0, blk_threads = 1024;  // blocked slab pass (0: not available)
    size_t blk_lds = 0;
    int nparts = 1;         // largest number of partial sums any launch writes
};
enum HvMode { HV_STORE = 0, HV_LANCZOS = 1, HV_RESIDUAL = 2, HV_FUSED = 3, HV_FUSED_DEFL = 4 };
enum RedMode { RED_PLAIN = 0, RED_DOT = 1, RED_NORM = 2, RED_FUSED = 3, RED_START = 4, RED_FIX = 5 };
// Lower states a fused deflated step projects out (more take the unfused step).
constexpr int kFusedDefl = 2;
// Deflation data of HV_FUSED_DEFL: nd FP64 vectors in dense J order (vector l
// at psi + l * pdim) and their coefficients g (device, nd values).
struct HvDefl {
    const double *psi = nullptr;
    int nd = 0;
    int64_t pdim = 0;
    const double *g = nullptr;
};
// Fused Lanczos step: below this ratio b_{j+1}^2 / |q|^2 the expanded norm
// has lost too many digits and the step is finished by the explicit fix-up
// (device scalars S[kFixFlag], S[kFixScale]).
constexpr double kFixRatio = 1e-4;
constexpr int kFixFlag = 6, kFixScale = 7;

// HV_STORE:    y = H x
// HV_LANCZOS:  y = alpha H x + beta y (in place), alpha = coef[0], beta = coef[1];
//              partials[b] = block b's share of y.x
// HV_RESIDUAL: nothing stored; partials[b] = share of |Hx - alpha x|^2,
//              partials[nblocks + b] = share of x.Hx
// HV_FUSED:    (two-pass plans, padded rows) x <- x - c y is formed and written
//              back first, then y = alpha H x + beta y; coef = S (S[1] alpha,
//              S[2] beta, S[3] c); partials [3][n] = shares of y.x, y.y, x.x
// HV_FUSED_DEFL: as HV_FUSED with x <- x - c y - sum_l g_l psi_l (HvDefl,
//              nd <= kFusedDefl, line layout of the up-spin entries);
//              partials [3 + 2l][n] = shares of psi_l.y, [4 + 2l][n] of psi_l.x
template <typename T>
void launch_hv(const HvArgs &a, const T *x, T *y, int mode, double alpha, const double *coef, double *partials,
               int nblocks, hipStream_t s);
int hv_blocks(const HvArgs &a, int elem_bytes);

HvPlan make_hv_plan(const HvArgs &a, int elem_bytes);
// x, y (and scratch) are row-major dim_up x dim_dn with row strides ldx, ldy
// (lds_); scratch (the row-pass output) is used by HV_RESIDUAL only, where y
// is not written.  Partial sums: pl.nparts values (HV_RESIDUAL: twice that).
// Returns the number of partial sums written (HV_RESIDUAL: twice that many values).
// xpad, ypad: null, or dim_up x pl.ld work arrays.  When the rows of x or y do
// not start on 128 bytes, HV_STORE with both (HV_RESIDUAL with xpad) routes
// through them: the row pass writes its result to ypad (scratch) and a copy
// of x to xpad, and the up-spin pass runs on those and writes y.
// yout (fused modes, line layout): the result goes to yout (stride ldy) and y
// is only read (the beta and c terms).  pair > 0: the same step on a second
// vector pair at element offset pair from x, y and yout (the imaginary halves
// of complex vectors); the partial sums cover both pairs.
template <typename T>
int launch_hv2(const HvArgs &a, const HvPlan &pl, const T *x, int64_t ldx, T *y, int64_t ldy, T *scratch,
               int64_t lds_, int mode, double alpha, const double *coef, double *partials, hipStream_t s,
               T *xpad = nullptr, T *ypad = nullptr, const HvDefl *defl = nullptr, T *yout = nullptr,
               int64_t pair = 0);

template <typename T>
void launch_axpy_norm(T *w, const T *v, const double *coef, int64_t n, double *partials, int nblocks, hipStream_t s);
// the fix-up of a flagged fused step (a no-op when S[kFixFlag] is clear)
template <typename T>
void launch_fused_fix(T *w, const T *v, const double *S, int64_t n, double *partials, int nblocks, hipStream_t s);
// the same for a fused deflated step: w <- w - S[3] v - sum_l S[8 + l] psi_l,
// rows at stride ld (returns the number of partial sums)
template <typename T>
int launch_fused_fix_defl(T *w, const T *v, const double *S, const double *psi, int nd, int64_t pdim, int64_t dim_up,
                          int64_t dim_dn, int64_t ld, double *partials, hipStream_t s);
void launch_start_raw(uint64_t seed, double *f, int64_t n, hipStream_t s);
void launch_start_norm2(const double *given, uint64_t seed, int64_t n, double *partials, int nblocks, hipStream_t s);
// out[r*ld + d] = (T)(c f[r*dim_dn + d]) and 0 in the row padding; zero (if
// not NULL) is cleared including its padding
template <typename T>
void launch_start_fill(const double *given, uint64_t seed, double c, T *out, T *zero, int64_t dim_up, int64_t dim_dn,
                       int64_t ld, hipStream_t s);
// psi[r*dim_dn + d] (+)= y_j * coef[0] * v[r*ld + d]
template <typename T>
void launch_psi_acc(double *psi, const T *v, double yj, const double *coef, int64_t dim_up, int64_t dim_dn, int64_t ld,
                    bool first, hipStream_t s);
void launch_psi_stats(const double *psi, const double *given, uint64_t seed, int64_t n, double *partials, int nblocks,
                      hipStream_t s);
// psi[r*dim_dn + d] = sum_{j < m} y[j] * scale[j] * vecs[j][r*ld + d] (the resident Lanczos vectors)
template <typename T>
void launch_psi_combine(double *psi, const T *const *vecs, const double *y, const double *scale, int m, int64_t dim_up,
                        int64_t dim_dn, int64_t ld, hipStream_t s);
void launch_scale(double *v, double c, int64_t n, hipStream_t s);
void launch_reduce(const double *partials, int n, int stride, int count, double *out, hipStream_t s);
// observables.hip: unnormalised sums UU, DD, C (NS x NS each, NS = obs_ns_max)
// and the norm of psi^2 into out[3 * NS * NS + 1]; part holds
// obs_partial_count blocks of that size (the workgroups' partials and the
// group sums of the reduction).  max_blocks bounds the accumulating workgroups.
constexpr int kObsDefaultBlocks = 2048;
int obs_ns_max(int sites);
int obs_partial_count(int ns, int64_t dim_up, int64_t dim_dn, int max_blocks = kObsDefaultBlocks);
void launch_observables(const double *psi, const uint32_t *states_up, const uint32_t *states_dn, int ns,
                        int64_t dim_up, int64_t dim_dn, double *part, double *out, int max_blocks, hipStream_t s);
// The allocation-free form: a static device array of kObsScratchBytes per
// device (its address taken once per device), and the largest workgroup count
// whose partial sums fit it.
constexpr size_t kObsScratchBytes = (size_t)16 << 20;
constexpr int kObsMaxDevices = 64;
double *obs_scratch(int device);
int obs_noalloc_blocks(int ns, int64_t dim_up, int64_t dim_dn);

// propagate.hip: the Krylov propagation step (see the file's header for the
// slot layout and the device scalars sc[4j..4j+3] = {s_j, 0, a_j, b_{j+1}})
enum PropMode { PROP_START = 0, PROP_DOT = 1, PROP_NORM = 2 };
int launch_prop_load(const double *re, const double *im, double *slot, int64_t npad, int64_t dim_up, int64_t dim_dn,
                     int64_t ld, double *partials, hipStream_t s);
int launch_prop_update(double *y, const double *w, const double *wp, const double *sc, int j, int64_t n,
                       double *partials, hipStream_t s);
int launch_prop_combine(double *basis, int nv, int64_t slot_stride, int64_t npad, const double *gam, double *re,
                        double *im, int64_t dim_up, int64_t dim_dn, int64_t ld, double *partials, hipStream_t s);
void launch_prop_reduce(const double *partials, int n, int mode, double *sc, int j, hipStream_t s);

// Most lower eigenvectors one deflated Lanczos run projects out.
constexpr int kMaxDeflate = 15;
// number of partial sums the two deflation kernels write per vector
int defl_blocks(int64_t dim_up);
template <typename T>
int launch_defl_dots(T *q, const T *v, const double *coef, const double *psi, int nd, int64_t dim, int64_t dim_up,
                     int64_t dim_dn, int64_t ld, double *partials, hipStream_t s);
template <typename T>
int launch_defl_update(T *q, const double *psi, const double *D, int nd, int64_t dim, int64_t dim_up, int64_t dim_dn,
                       int64_t ld, double *partials, hipStream_t s);
// nd: lower vectors of a fused deflated step (RED_FUSED)
void launch_reduce_step(const double *partials, int n, int mode, double *S, double *hist, int j, hipStream_t s,
                        int nd = 0);
void launch_init_scalars(double *S, hipStream_t s);
int stream_blocks(int64_t n);

}  // namespace hub
