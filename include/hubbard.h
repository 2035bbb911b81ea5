/*
 * hubbard.h -- C ABI of the MI355X Hubbard exact-diagonalisation library.
 *
 * The library computes the lowest eigenvalue (and optionally the eigenvector)
 * of the Hubbard Hamiltonian
 *     H = -t sum_<ij> sum_sigma (c+_{i sigma} c_{j sigma} + h.c.) + U sum_i n_{i up} n_{i dn}
 * in one sector of fixed N_up and N_dn (Siro & Harju, arXiv:1204.3425,
 * Sec. 1, eq. H, and Sec. 2.1), with the Lanczos iteration of Sec. 2.2
 * (Alg. 1) running on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every call:
 *   - Sites are numbered 0..sites-1; bit i of a configuration word is site i
 *     (Sec. 2.1, eq. binaryrep).
 *   - Basis order: configurations of each spin in ascending integer order;
 *     J = i_up * dim_dn + i_dn (Sec. 2.1, eq. J-formula).  Every vector
 *     crossing this ABI is a contiguous array of dim elements in J order.
 *   - A bond (i, j) is undirected; the hermitian conjugate hop is implied
 *     (eq. H).  The matrix element of one hop is -t * sgn, sgn = (-1)^n, n the
 *     number of same-spin electrons on sites strictly between i and j
 *     (Sec. 2.1, the sign paragraph).
 *   - Device pointers are HIP device memory on the current device of the
 *     calling thread.  Host pointers are ordinary memory.  The caller owns every
 *     buffer it passes; the handle owns its basis and tables.
 *   - Return codes: 0 = success, > 0 = warning with results written,
 *     < 0 = error with nothing written.  hubbard_last_error() gives a message
 *     for the most recent failure on the calling thread.  No C++ exception
 *     crosses this boundary.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef HUBBARD_H
#define HUBBARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hubbard *hubbard_h;

enum {
    HUBBARD_OK = 0,
    HUBBARD_ENOCONV = 1,  /* max_iter reached before the energy test passed */
    HUBBARD_EINVAL = -1,  /* invalid argument */
    HUBBARD_ERANGE = -2,  /* sector too large for the index types */
    HUBBARD_ENOMEM = -3,  /* device or host allocation failed */
    HUBBARD_EDEVICE = -4, /* a HIP call failed */
    HUBBARD_EBUSY = -5    /* resource in use (server queue full) */
};

enum {
    HUBBARD_FP64 = 0,  /* vectors, H.v and reductions in FP64 */
    HUBBARD_MIXED = 1  /* vectors and H.v in FP32 (FP32 accumulation); alpha/beta
                          reductions, the tridiagonal solve and the residual in FP64 */
};

enum { HUBBARD_SPIN_UP = 0, HUBBARD_SPIN_DN = 1 };

/* Why a Lanczos run stopped. */
enum {
    HUBBARD_STOP_MAXITER = 0,   /* max_iter steps done */
    HUBBARD_STOP_CONVERGED = 1, /* |E_j - E_{j-1}| <= tol * max(1, |E_j|) (Sec. 2.2) */
    HUBBARD_STOP_BREAKDOWN = 2, /* b_{j+1} vanished: invariant subspace (Alg. 1) */
    HUBBARD_STOP_EXHAUSTED = 3  /* j reached dim */
};

typedef struct {
    int32_t sites, n_up, n_dn, n_edges;
    double t, U;
    int64_t dim_up, dim_dn, dim; /* C(sites, N_up), C(sites, N_dn), their product (Sec. 2.1) */
    int32_t w_up, w_dn;          /* ELL widths = max entries per row (Sec. 4.2, Fig. ELL) */
    int64_t nnz_up, nnz_dn;      /* stored hopping entries per spin */
    size_t device_bytes;         /* device memory held by the handle (tables + states) */
    size_t vector_bytes;         /* device memory one Lanczos run allocates (work vectors) */
    int64_t ld_pref;             /* row stride (elements) of the library's own vectors */
} hubbard_info_t;

typedef struct {
    double tol;          /* energy test of Sec. 2.2; tol < 0 runs exactly max_iter steps */
    int32_t max_iter;    /* >= 1 */
    int32_t precision;   /* HUBBARD_FP64 or HUBBARD_MIXED */
    uint64_t seed;       /* start vector f1[J] = 2u-1, u from SplitMix64 counter J+1, normalised */
    const double *start; /* optional device FP64 start vector (dim, unit norm, J order); overrides seed */
    double *psi;         /* optional device FP64 output: ground-state vector, unit norm, <psi,f1> > 0 */
    double *a_out;       /* optional host array[max_iter]: a_j, j = 1..n_iter (Alg. 1) */
    double *b_out;       /* optional host array[max_iter]: b_{j+1}, j = 1..n_iter */
    double *e_out;       /* optional host array[max_iter]: lowest eigenvalue of T_j */
} hubbard_opts;

typedef struct {
    double e0;          /* lowest eigenvalue of T_m (Sec. 2.2, eq. Tmatrix) */
    double residual;    /* FP64 ||H psi - e0 psi|| when psi was requested, else -1 */
    double rayleigh;    /* FP64 <psi|H|psi> when psi was requested, else NaN */
    double err_est;     /* residual / max(1, |e0|) when psi was requested; otherwise the Lanczos
                           estimate b_{m+1} |y_m| / max(1, |e0|) of that residual (y: eigenvector of T_m) */
    double seconds;     /* wall time of the whole call */
    double seconds_per_iter; /* mean wall time of one Lanczos step (first pass) */
    int32_t n_iter;     /* m = number of a_j computed */
    int32_t stop;       /* HUBBARD_STOP_* */
    int32_t status;     /* HUBBARD_OK or HUBBARD_ENOCONV, or an error code */
    int32_t precision;
    int32_t psi_resident; /* 1: psi was combined from the Lanczos vectors kept on the device;
                             0: from the replayed recurrence (or psi not requested) */
} hubbard_result;

/* Builds the basis of each spin (ascending configuration words, combinatorial
 * rank; Sec. 2.1) and the signed ELL hopping tables (Sec. 4.2, eq.
 * H-Kroneckersum and Fig. ELL), uploads them to the current device and
 * returns a handle.
 *   sites: 1..32.  edges: host array of 2*n_edges int32 site indices, each pair
 *   (i, j) with 0 <= i, j < sites, i != j, no unordered pair repeated.
 *   n_up, n_dn: 0..sites.  t, U: finite.
 * Errors: EINVAL (bad argument), ERANGE (dim >= 2^40: one vector would not
 * fit a device), ENOMEM, EDEVICE.  On a machine with no HIP device the handle
 * holds the host tables only: hubbard_info and the export calls work, and every
 * device call returns EDEVICE. */
int hubbard_build(int sites, const int32_t *edges, int n_edges, int n_up, int n_dn, double t, double U,
                  hubbard_h *out);

/* As hubbard_build with one hopping amplitude per bond: the hop over edge k
 * has the element -t[k] * sgn (eq. H with t_ij in place of t; Sec. 2.1 notes
 * that the construction holds for any lattice).  t: host array of n_edges
 * finite values (NULL only when n_edges = 0).  If all t[k] are equal the
 * handle is exactly the hubbard_build one.  Otherwise the amplitudes are
 * grouped into classes of equal value (at most 127) whose index each table
 * entry carries.  With at most four classes the two-pass H.v kernels run (the
 * class takes two bits of their entries); with more, the one-pass kernel runs
 * every call and hubbard_apply_ld takes only dense rows (ld = dim_dn, which
 * hubbard_info then reports as ld_pref).  Such a handle runs unbatched in
 * hubbard_lanczos_batch and reports t = NaN in hubbard_info.
 * Errors: as hubbard_build; EINVAL also for more than 127 distinct
 * amplitudes or a non-finite one; ERANGE also when non-uniform amplitudes meet
 * a spin dimension of 2^24 or more (the column must fit 24 bits beside the
 * class). */
int hubbard_build_bonds(int sites, const int32_t *edges, const double *t, int n_edges, int n_up, int n_dn, double U,
                        hubbard_h *out);

/* Releases the handle and its device memory.  NULL is accepted. */
int hubbard_free(hubbard_h h);

/* Stream for every later call on this handle (a hipStream_t; NULL = the null
 * stream).  The caller keeps the stream alive while the handle uses it. */
int hubbard_set_stream(hubbard_h h, void *hip_stream);

/* Arithmetic of hubbard_apply and hubbard_lanczos: HUBBARD_FP64 (default) or
 * HUBBARD_MIXED. */
int hubbard_set_precision(hubbard_h h, int precision);

/* Device bytes that a solve with psi requested may hold for its resident
 * Lanczos basis (default: no limit beyond the free memory less 2 GiB).  While
 * the basis fits, every Lanczos vector is kept in a slot of its own as the
 * first pass runs (on large sectors formed there by the step itself, elsewhere
 * copied) and psi = sum_j y_j f_j is one pass over them (Sec. 2.2 obtains psi
 * from the same sum); otherwise, or with 0, the slots are freed and the
 * recurrence is replayed to accumulate psi, as without the basis.  Both give
 * psi to rounding; hubbard_result.psi_resident tells which ran.  Slots are
 * allocated 32 vectors at a time. */
int hubbard_set_basis_limit(hubbard_h h, size_t bytes);

/* Seed of the start vector used by hubbard_lanczos (default 12043425). */
int hubbard_set_seed(hubbard_h h, uint64_t seed);

/* y = H x (Sec. 4.3: H_up (x) I, I (x) H_dn and the interaction term; two
 * passes over the rows of the dim_up x dim_dn view, the down-spin hops and the
 * interaction from rows staged in LDS, then the up-spin hops as row
 * combinations).  x, y: device arrays of dim elements in J order, double under
 * HUBBARD_FP64 and float under HUBBARD_MIXED; y is overwritten and must not
 * overlap x.  Asynchronous on the handle's stream.  When the rows of x or y do
 * not start on 128 bytes (dim_dn not a multiple of 16 doubles or 32 floats)
 * and the up-spin rows have at most 64 hops, the product routes through two work vectors at the stride ld_pref that the
 * handle allocates on the first such call (2 * dim_up * ld_pref elements of the
 * current precision, kept until hubbard_free; ENOMEM if they do not fit): the
 * row pass writes its result and a copy of x there, and the up-spin pass reads
 * them and writes y.  Calls share these vectors: a call on another stream
 * waits for the previous one. */
int hubbard_apply(hubbard_h h, const void *x, void *y);

/* y = H x as hubbard_apply, with x and y stored as dim_up rows of dim_dn
 * elements at row strides ldx and ldy (elements, >= dim_dn; the subvectors of
 * Sec. 4.3, Fig. slots).  Padding elements are neither read nor written.
 * hubbard_info gives the stride the library uses for its own vectors
 * (ld_pref, a multiple of 64 elements): strides that are a multiple of 128
 * bytes (and buffers aligned to 128 bytes) select the blocked up-spin pass,
 * which works on one cache line of every row at a time; other strides route
 * through the handle's work vectors as in hubbard_apply (up-spin rows of more
 * than 64 hops take a slower pass instead).  Where the one-pass kernel runs (rows too wide for LDS, or a
 * handle with more than four distinct per-bond amplitudes) ld_pref is dim_dn
 * and only dense rows (ldx = ldy = dim_dn) are accepted: other strides return
 * EINVAL. */
int hubbard_apply_ld(hubbard_h h, const void *x, int64_t ldx, void *y, int64_t ldy);

/* Lanczos ground state (Sec. 2.2, Alg. 1, two-vector form): iterates until
 * the energy test passes with tol (> 0), b_{j+1} vanishes, or max_iter (>= 1)
 * steps.  Writes the lowest Ritz value to *E0 (host).  psi: NULL, or a device
 * FP64 array of dim elements receiving the ground-state vector, combined from
 * the Lanczos vectors kept on the device (or accumulated by a replayed pass
 * when they do not fit; hubbard_set_basis_limit).  Synchronous.  Returns OK,
 * or ENOCONV when max_iter was hit first (E0 still written). */
int hubbard_lanczos(hubbard_h h, double tol, int max_iter, double *E0, double *psi);

/* As hubbard_lanczos with every option and the full result record. */
int hubbard_lanczos_ex(hubbard_h h, const hubbard_opts *opts, hubbard_result *res);

/* The k lowest eigenvalues of the sector, repeated by multiplicity, and their
 * eigenvectors (Sec. 2.2: the ground state and the lowest excited states),
 * found one after another: state i is the ground state of P H P with
 * P = 1 - sum_{l<i} psi_l psi_l^T, run as Alg. 1 with every new Lanczos vector
 * projected through P (the start vector too); psi_i is then formed from its
 * Lanczos vectors as for hubbard_lanczos, projected once more, normalised and signed
 * so that <psi_i, f1^(i)> > 0.  State i starts from its own vector f1^(i): the
 * seeded vector of hubbard_start_raw with seed opts->seed + i (state 0 from
 * opts->start when that is given).  Separate starts are what lets a degenerate
 * level come out once per eigenvector (in no particular order within the
 * level): one start vector shared by all states would have, inside the level,
 * only the component that the level's first state takes away.
 *   k: 1..16, at most dim.
 *   opts: tol, max_iter and precision as for hubbard_lanczos_ex, applied to
 *     every state (the energy test of Sec. 2.2 per state); seed and start as
 *     above; opts->psi and the history arrays must be NULL.
 *   E: host array[k] receiving E_0 <= E_1 <= ... (lowest Ritz value of each
 *     deflated run; ties and near-ties may come out in either order).
 *   psi: NULL, or a device FP64 array of k * dim elements receiving psi_i at
 *     psi + i * dim (J order).  With NULL the library allocates k * dim
 *     doubles for the duration of the call.
 *   res: NULL, or a host array[k] of results; res[i].residual is the FP64
 *     |H psi_i - E_i psi_i| of the full H (not of P H P).
 * The error of E_i is of the order of tol plus the squared eigenvector errors
 * of the lower states, so ask for tol well below the accuracy wanted for the
 * upper states.  A deflated step costs one H.v and two passes over the i lower
 * vectors; the large-sector fused step is used for state 0 only.
 * Errors: EINVAL (bad k or opts, or a start vector inside the span of the lower
 * states), ENOMEM, EDEVICE.  Synchronous.  Returns the most severe per-state
 * status (OK or ENOCONV). */
int hubbard_lowest_states(hubbard_h h, int k, const hubbard_opts *opts, double *E, double *psi,
                          hubbard_result *res);

/* Site occupations of a state and their correlations, <psi|O|psi> / <psi|psi>
 * for the number operators n_{i sigma} of eq. H (Sec. 1), which are diagonal in
 * the configuration basis (Sec. 2.1: bit i of a spin's word is n_i of that
 * spin).  One pass over psi on the device; the sums are FP64 and reduced in a
 * fixed order.
 *   psi: device FP64 array of dim elements (J order), any non-zero norm.
 *   dens: NULL or host array[2 * sites]: <n_{i up}> at i, <n_{i dn}> at sites + i.
 *   corr: NULL or host array[3 * sites * sites], row-major blocks:
 *     <n_{i up} n_{j up}> at i * sites + j, <n_{i dn} n_{j dn}> at
 *     sites^2 + i * sites + j, <n_{i up} n_{j dn}> at 2 sites^2 + i * sites + j;
 *     the diagonal of the last block is the double occupancy of each site.
 *   docc: NULL or host scalar: D = <sum_i n_{i up} n_{i dn}>, so that the
 *     interaction energy of eq. H is U * D (and, for a ground state,
 *     D = dE0/dU).
 * Errors: EINVAL (psi NULL, or zero or non-finite norm), ENOMEM, EDEVICE.
 * Synchronous on the handle's stream. */
int hubbard_observables(hubbard_h h, const double *psi, double *dens, double *corr, double *docc);

/* hubbard_observables for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and errors, with no hipMalloc,
 * hipFree or other allocating call.  The partial sums live in a static device
 * array of 16 MiB per device, held from the first call on that device until
 * the process ends; lattices whose partial sums would not fit it (none for the
 * workgroup counts used here) return ERANGE.  With more than 16 sites the
 * accumulation runs on fewer workgroups than hubbard_observables uses, so the
 * sums are added in another order (equal within FP64 rounding); with at most
 * 16 sites they are bitwise equal.  Every call on a device shares that
 * device's array: calls that overlap on one device (two streams, two host
 * threads) race and must be serialised by the caller.  Synchronous on the
 * handle's stream. */
int hubbard_observables_noalloc(hubbard_h h, const double *psi, double *dens, double *corr, double *docc);

/* Result of hubbard_propagate. */
typedef struct {
    double err_est;          /* sum over the steps of |psi| b_{m+1} |(exp(-i T_m dt) e_1)_m|: the Lanczos
                                estimate of each step's error (0 for a step that ended in an invariant subspace) */
    double norm;             /* |psi| after the last step (the start norm, up to that error) */
    double seconds;          /* wall time of the call */
    int32_t n_steps;
    int32_t krylov_dim_max;  /* largest Krylov dimension a step used (smaller after an invariant subspace) */
} hubbard_prop_result;

/* Real-time evolution psi <- exp(-i H t) psi (H of eq. H; the H.v of Sec. 4.3
 * drives it as it drives the ground-state search) in n_steps equal steps of
 * dt = t / n_steps.  Each step runs the recurrence of Alg. 1 on the complex
 * vector for krylov_dim steps (H is real and symmetric, so the coefficients
 * are real), keeps the whole Krylov basis on the device, and forms
 * psi(t + dt) = |psi| V_m exp(-i T_m dt) e_1 from it; a vanishing b_{j+1}
 * (an invariant subspace) makes the step exact with the smaller basis.
 * Always FP64, whatever the handle's precision.
 *   psi_re, psi_im: device FP64 arrays of dim elements (J order), the real and
 *     imaginary parts, overwritten with the result; distinct, non-overlapping.
 *   t: finite (negative t runs backwards).  n_steps >= 1.  krylov_dim: 2..64.
 *   energy: NULL or host array[n_steps + 1] receiving <psi|H|psi>/<psi|psi> at
 *     t_k = k dt, k = 0..n_steps (conserved by the exact evolution).
 *   res: NULL or a host result record.
 * Device memory: (krylov_dim + 1) complex vectors in the padded row layout
 * (16 (krylov_dim + 1) dim_up ld_pref bytes) for the duration of the call.
 * Errors: EINVAL (bad argument, or psi of zero norm), ENOMEM, EDEVICE.
 * Synchronous on the handle's stream. */
int hubbard_propagate(hubbard_h h, double *psi_re, double *psi_im, double t, int n_steps, int krylov_dim,
                      double *energy, hubbard_prop_result *res);

/* Sizes of the handle's sector and tables. */
int hubbard_info(hubbard_h h, hubbard_info_t *info);

/* Host copy of one spin's basis: dim_sigma configuration words, ascending. */
int hubbard_export_basis(hubbard_h h, int spin, uint32_t *states);

/* Host copy of one spin's ELL hopping table in the column-major layout of
 * Fig. ELL: entry k of row r at k * dim_sigma + r, for k < w_sigma.  col: the
 * column (rank of the hopped configuration); sgn: +1 or -1 (matrix element
 * -t * sgn); padding has col 0 and sgn 0.  Entries of a row ascend by column. */
int hubbard_export_table(hubbard_h h, int spin, int32_t *col, int8_t *sgn);

/* f[J] = 2u - 1 for J < dim, u = (SplitMix64(seed + (J+1) * 0x9E3779B97F4A7C15) >> 11) * 2^-53
 * (Steele, Lea & Flood 2014): the un-normalised start vector of Alg. 1.
 * f: device FP64 array.  Asynchronous on `hip_stream`. */
int hubbard_start_raw(uint64_t seed, int64_t dim, double *f, void *hip_stream);

/* Runs n independent Lanczos solves (one per handle, each with opts[i]) on the
 * current device, writing res[i].  Solves without a psi request whose rows fit
 * in 64 KB share their launches: every step of every such solve runs in the
 * same four kernel launches (Sec. 5 notes that small systems leave the GPU
 * idle), and the Ritz value E_j and the stop tests of hubbard_lanczos_ex are
 * evaluated on the device, so the host reads results a few steps behind.  The
 * others run one after another.  A batched result does not depend on which
 * other solves share the batch, and agrees with the same solve run alone
 * within rounding (the batched E_j comes from a multisection on the device,
 * the single-instance one from a bisection on the host).  res[i].err_est is
 * the Lanczos estimate b_{m+1} |y_m| / max(1, |E0|).  Synchronous; the stream
 * of hs[0] is used.  Returns the most severe per-solve status. */
int hubbard_lanczos_batch(hubbard_h *hs, int n, const hubbard_opts *opts, hubbard_result *res);

/* ---------------------------------------------------------------- serving
 * A server runs a continuous stream of independent ground-state requests on
 * the current device.  Requests are admitted first-fit in arrival order while
 * a slot is free and their device footprint (tables + work vectors, an upper
 * bound from the sector size) fits in the HBM budget; admitted requests have
 * their tables built on a host thread and then join the running work: small
 * sectors join a shared batch between Lanczos steps (every step of every
 * batched request runs in the same kernel launches), large ones run on a
 * second stream with the two-pass H.v, so both overlap on the device.  A
 * result does not depend on what else was running.  The caller polls
 * completions, which carry the result and the submit/admit/start/done times. */
typedef struct hubbard_server *hubbard_server_h;

typedef struct {
    int32_t sites;          /* as hubbard_build */
    const int32_t *edges;   /* 2*n_edges site indices; copied by submit */
    int32_t n_edges;
    int32_t n_up, n_dn;
    double t, U;
    double tol;             /* as hubbard_opts */
    int32_t max_iter;
    int32_t precision;
    uint64_t seed;
    uint64_t tag;           /* caller's value, returned in the completion */
} hubbard_request;

typedef struct {
    uint64_t id, tag;
    int32_t status;         /* OK / ENOCONV, or the error that ended the request (ENOMEM when it can never fit) */
    int32_t pad_;
    double t_submit, t_admit, t_start, t_done;  /* seconds since the server was created */
    hubbard_result result;  /* psi is never requested; err_est is the Lanczos residual estimate */
} hubbard_completion;

typedef struct {
    uint64_t budget, reserved, peak_reserved;   /* bytes */
    uint64_t submitted, admitted, completed, rejected, pending;
    int32_t max_active_batch, slots_used;
    uint64_t solo_runs;   /* requests run by the executor for large sectors (one at a time, own stream) */
} hubbard_server_stats_t;

/* Creates a server with an HBM budget (bytes, > 0) and a slot limit (>= 1). */
int hubbard_server_create(size_t hbm_budget, int max_slots, hubbard_server_h *out);
/* Queues one request and returns its id.  EINVAL for malformed requests; a
 * request whose footprint exceeds the whole budget completes at once with
 * status ENOMEM.  Thread-safe. */
int hubbard_server_submit(hubbard_server_h s, const hubbard_request *req, uint64_t *id);
/* Copies up to cap completions into out (host) and sets *n; waits up to
 * timeout_us when none is ready.  Thread-safe. */
int hubbard_server_poll(hubbard_server_h s, hubbard_completion *out, int cap, int *n, int timeout_us);
int hubbard_server_stats(hubbard_server_h s, hubbard_server_stats_t *stats);
/* Stops the server: running requests are abandoned, queued ones dropped. */
int hubbard_server_destroy(hubbard_server_h s);

/* The admission rule of the server, exposed for schedulers and tests: given
 * the footprints of n queued requests in arrival order, marks admit[k] = 1 for
 * each request taken first-fit while fewer than free_slots are taken and the
 * taken footprints fit in budget - used.  Returns the number taken. */
int hubbard_admission_plan(const uint64_t *footprints, int n, uint64_t budget, uint64_t used, int free_slots,
                           int32_t *admit);

/* Message for a return code, and the message of the calling thread's last
 * failure (empty when none). */
const char *hubbard_strerror(int code);
const char *hubbard_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HUBBARD_H */
