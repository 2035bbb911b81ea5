/*
 * hubbard_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential double-precision CPU implementation of what the
 * Hubbard exact-diagonalisation hot path computes, written from Siro & Harju,
 * "Exact diagonalization of the Hubbard model on graphics processing units"
 * (arXiv:1204.3425).  It is the checker the GPU library is compared against.
 * It shares no code, header, table or helper with the GPU library, and only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  Nothing here is blocked, fused or reordered for speed.
 *
 * What is computed, and the passage each part follows:
 *   - basis per spin: every Ns-bit word with N_sigma bits set, in ascending
 *     integer order, bit i = site i (Sec. 2.1, eq. binaryrep and the ordering
 *     paragraph after it);
 *   - position of a word in that list: binary search of the sorted list (a
 *     deliberately different route from any rank formula);
 *   - J = i_up * dim_dn + i_dn (Sec. 2.1, eq. J-formula);
 *   - hopping elements: for each edge {i,j} and direction, an electron of one
 *     spin moves from an occupied site to an empty one; the element is
 *     -t * (-1)^n with n the number of same-spin electrons on sites whose
 *     labels lie strictly between i and j (Sec. 2.1, the sign paragraph and
 *     eq. H); counted here by a per-site loop;
 *   - interaction: U times the number of doubly occupied sites, per-site loop
 *     (Sec. 2.1, eq. H; Alg. 4);
 *   - H.v: y[J] = diag[J] x[J] + sum over up hops + sum over down hops, a
 *     direct loop over (i_up, i_dn) (Sec. 4.3, the subvector view, eqs. for
 *     H_up (x) I and I (x) H_dn);
 *   - start vector: f1[J] = 2u - 1, u = (SplitMix64 output for counter J) / 2^64
 *     truncated to 53 bits, then normalised (Sec. 2.2: a random vector of
 *     norm 1; SplitMix64 is Steele, Lea & Flood, OOPSLA 2014);
 *   - Lanczos: Alg. 1 step by step in FP64, no re-orthogonalisation;
 *   - Ritz value: lowest eigenvalue of the tridiagonal T_j (Sec. 2.2, eq.
 *     Tmatrix) by Sturm-sequence bisection; convergence when the change from
 *     the previous iteration is at most tol * max(1, |E0|) (Sec. 2.2);
 *   - ground-state vector: eigenvector of T_m by inverse iteration, then the
 *     recurrence is replayed and psi = sum_j y_j f_j accumulated; residual
 *     ||H psi - E0 psi|| and the Rayleigh quotient <psi|H|psi> in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

/* ------------------------------------------------------------------ basis */

static int bits_set(uint32_t s, int ns)
{
    int c = 0;
    for (int k = 0; k < ns; k++)
        if ((s >> k) & 1u)
            c++;
    return c;
}

/* Every ns-bit word with n bits set, ascending.  Returns the count; writes at
 * most cap words when out is not NULL. */
int64_t orc_basis(int ns, int n, uint32_t *out, int64_t cap)
{
    int64_t count = 0;
    uint64_t end = (uint64_t)1 << ns;
    for (uint64_t s = 0; s < end; s++) {
        if (bits_set((uint32_t)s, ns) == n) {
            if (out && count < cap)
                out[count] = (uint32_t)s;
            count++;
        }
    }
    return count;
}

/* Position of word s in the ascending list, or -1 when absent. */
int64_t orc_position(const uint32_t *states, int64_t count, uint32_t s)
{
    int64_t lo = 0, hi = count - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (states[mid] == s)
            return mid;
        if (states[mid] < s)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* ----------------------------------------------------------- hopping rows */

/* One spin's hopping matrix as rows of (column, value), each row sorted by
 * column.  Row r lists <state_r | H_hop,sigma | state_c> for every c that one
 * hop of a sigma electron along an edge connects to state_r. */
typedef struct {
    int64_t dim;
    uint32_t *states;
    int64_t *row_start; /* dim + 1 */
    int32_t *col;
    double *val;
} spin_table;

static int count_between(uint32_t s, int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a, n = 0;
    for (int k = lo + 1; k < hi; k++)
        if ((s >> k) & 1u)
            n++;
    return n;
}

static int cmp_entry(const void *pa, const void *pb)
{
    const int64_t *a = (const int64_t *)pa, *b = (const int64_t *)pb;
    return (a[0] > b[0]) - (a[0] < b[0]);
}

static int build_spin_table(spin_table *tb, int ns, const int32_t *edges, const double *amp, int ne, int n)
{
    int64_t dim = orc_basis(ns, n, NULL, 0);
    tb->dim = dim;
    tb->states = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)dim);
    tb->row_start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(dim + 1));
    if (!tb->states || !tb->row_start)
        return -1;
    orc_basis(ns, n, tb->states, dim);

    /* first pass: entries per row, two directions per edge */
    int64_t total = 0;
    tb->row_start[0] = 0;
    for (int64_t r = 0; r < dim; r++) {
        uint32_t s = tb->states[r];
        for (int e = 0; e < ne; e++) {
            int i = edges[2 * e], j = edges[2 * e + 1];
            int oi = (s >> i) & 1u, oj = (s >> j) & 1u;
            if (oi != oj)
                total++; /* exactly one direction can hop */
        }
        tb->row_start[r + 1] = total;
    }
    tb->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    tb->val = (double *)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(ne > 0 ? 2 * ne : 1));
    if (!tb->col || !tb->val || !tmp)
        return -1;

    for (int64_t r = 0; r < dim; r++) {
        uint32_t s = tb->states[r];
        int m = 0;
        for (int e = 0; e < ne; e++) {
            int ends[2] = {edges[2 * e], edges[2 * e + 1]};
            for (int dir = 0; dir < 2; dir++) {
                int from = ends[dir], to = ends[1 - dir];
                if (((s >> from) & 1u) && !((s >> to) & 1u)) {
                    uint32_t s2 = s - (1u << from) + (1u << to);
                    int64_t c = orc_position(tb->states, dim, s2);
                    int nb = count_between(s, from, to);
                    double v = -amp[e] * ((nb % 2) ? -1.0 : 1.0);
                    tmp[2 * m] = c;
                    memcpy(&tmp[2 * m + 1], &v, sizeof(double));
                    m++;
                }
            }
        }
        qsort(tmp, (size_t)m, 2 * sizeof(int64_t), cmp_entry);
        int64_t base = tb->row_start[r];
        for (int k = 0; k < m; k++) {
            tb->col[base + k] = (int32_t)tmp[2 * k];
            memcpy(&tb->val[base + k], &tmp[2 * k + 1], sizeof(double));
        }
    }
    free(tmp);
    return 0;
}

static void free_spin_table(spin_table *tb)
{
    free(tb->states);
    free(tb->row_start);
    free(tb->col);
    free(tb->val);
    memset(tb, 0, sizeof(*tb));
}

/* ------------------------------------------------------------------ model */

typedef struct {
    int ns;
    double t, U;
    spin_table up, dn;
    int64_t dim;
} orc_model;

/* The model with one hopping amplitude per bond: the hop over edge e has the
 * element -amp[e] * (-1)^n (eq. H with t_ij for t; Sec. 2.1 notes that the
 * construction holds for any lattice).  amp[e] = t for every e is the model of
 * eq. H itself. */
orc_model *orc_model_new_bonds(int ns, const int32_t *edges, const double *amp, int ne, int n_up, int n_dn, double U)
{
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    if (!m)
        return NULL;
    m->ns = ns;
    m->t = ne > 0 ? amp[0] : 0.0;
    m->U = U;
    if (build_spin_table(&m->up, ns, edges, amp, ne, n_up) || build_spin_table(&m->dn, ns, edges, amp, ne, n_dn)) {
        free_spin_table(&m->up);
        free_spin_table(&m->dn);
        free(m);
        return NULL;
    }
    m->dim = m->up.dim * m->dn.dim;
    return m;
}

orc_model *orc_model_new(int ns, const int32_t *edges, int ne, int n_up, int n_dn, double t, double U)
{
    double *amp = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
    if (!amp)
        return NULL;
    for (int e = 0; e < ne; e++)
        amp[e] = t;
    orc_model *m = orc_model_new_bonds(ns, edges, amp, ne, n_up, n_dn, U);
    free(amp);
    return m;
}

void orc_model_free(orc_model *m)
{
    if (!m)
        return;
    free_spin_table(&m->up);
    free_spin_table(&m->dn);
    free(m);
}

int64_t orc_dim(const orc_model *m, int spin)
{
    if (spin == 0)
        return m->up.dim;
    if (spin == 1)
        return m->dn.dim;
    return m->dim;
}

int64_t orc_nnz(const orc_model *m, int spin)
{
    const spin_table *tb = spin == 0 ? &m->up : &m->dn;
    return tb->row_start[tb->dim];
}

/* Copy out one spin's states and hopping rows (row_start has dim+1 entries). */
void orc_export(const orc_model *m, int spin, uint32_t *states, int64_t *row_start, int32_t *col, double *val)
{
    const spin_table *tb = spin == 0 ? &m->up : &m->dn;
    if (states)
        memcpy(states, tb->states, sizeof(uint32_t) * (size_t)tb->dim);
    if (row_start)
        memcpy(row_start, tb->row_start, sizeof(int64_t) * (size_t)(tb->dim + 1));
    int64_t nnz = tb->row_start[tb->dim];
    if (col)
        memcpy(col, tb->col, sizeof(int32_t) * (size_t)nnz);
    if (val)
        memcpy(val, tb->val, sizeof(double) * (size_t)nnz);
}

static double diag_element(const orc_model *m, uint32_t su, uint32_t sd)
{
    int doubles = 0;
    for (int k = 0; k < m->ns; k++)
        if (((su >> k) & 1u) && ((sd >> k) & 1u))
            doubles++;
    return m->U * doubles;
}

/* y[J] for one J = iu * dim_dn + id. */
static double apply_one(const orc_model *m, const double *x, int64_t iu, int64_t id)
{
    int64_t ddn = m->dn.dim;
    int64_t J = iu * ddn + id;
    double y = diag_element(m, m->up.states[iu], m->dn.states[id]) * x[J];
    for (int64_t k = m->up.row_start[iu]; k < m->up.row_start[iu + 1]; k++)
        y += m->up.val[k] * x[(int64_t)m->up.col[k] * ddn + id];
    for (int64_t k = m->dn.row_start[id]; k < m->dn.row_start[id + 1]; k++)
        y += m->dn.val[k] * x[iu * ddn + m->dn.col[k]];
    return y;
}

/* y = H x over the whole sector. */
void orc_apply(const orc_model *m, const double *x, double *y)
{
    for (int64_t iu = 0; iu < m->up.dim; iu++)
        for (int64_t id = 0; id < m->dn.dim; id++)
            y[iu * m->dn.dim + id] = apply_one(m, x, iu, id);
}

/* y[k] = (H x)[rows[k]] for a list of basis indices J. */
void orc_apply_rows(const orc_model *m, const double *x, const int64_t *rows, int64_t nrows, double *y)
{
    for (int64_t k = 0; k < nrows; k++)
        y[k] = apply_one(m, x, rows[k] / m->dn.dim, rows[k] % m->dn.dim);
}

/* The diagonal of H (interaction term only). */
void orc_diagonal(const orc_model *m, double *d)
{
    for (int64_t iu = 0; iu < m->up.dim; iu++)
        for (int64_t id = 0; id < m->dn.dim; id++)
            d[iu * m->dn.dim + id] = diag_element(m, m->up.states[iu], m->dn.states[id]);
}

/* ------------------------------------------------------------ start vector */

/* SplitMix64 (Steele, Lea & Flood 2014): the state advances by the golden
 * gamma 0x9E3779B97F4A7C15 and each output is the state passed through the
 * published finaliser.  Output number k (k = 1, 2, ...) of the stream that
 * starts at `seed` is therefore the finaliser of seed + k * gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* f[J] = 2u - 1 with u = (output J+1 >> 11) * 2^-53, not normalised. */
void orc_start_raw(uint64_t seed, int64_t dim, double *f)
{
    for (int64_t J = 0; J < dim; J++) {
        double u = (double)(orc_splitmix64(seed, (uint64_t)J + 1) >> 11) * (1.0 / 9007199254740992.0);
        f[J] = 2.0 * u - 1.0;
    }
}

/* ------------------------------------------------------------- tridiagonal */

/* Number of eigenvalues of the symmetric tridiagonal matrix (diagonal a[0..m-1],
 * off-diagonal b[1..m-1] between rows i-1 and i) that are smaller than x:
 * the count of negative pivots of T - x I (Sturm sequence). */
static int sturm_count(const double *a, const double *b, int m, double x)
{
    const double pivmin = DBL_MIN * 4.0;
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; i++) {
        double sub = (i == 0) ? 0.0 : (b[i] * b[i]) / d;
        d = (a[i] - x) - sub;
        if (fabs(d) < pivmin)
            d = -pivmin;
        if (d < 0.0)
            cnt++;
    }
    return cnt;
}

/* Lowest eigenvalue of T by bisection until no double lies strictly between
 * the two bounds. */
double orc_tridiag_min(const double *a, const double *b, int m)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; i++) {
        double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < m ? fabs(b[i + 1]) : 0.0);
        if (a[i] - r < lo)
            lo = a[i] - r;
        if (a[i] + r > hi)
            hi = a[i] + r;
    }
    double w = hi - lo;
    lo -= 1e-300 + 2.0 * DBL_EPSILON * fabs(lo) + DBL_EPSILON * w;
    hi += 1e-300 + 2.0 * DBL_EPSILON * fabs(hi) + DBL_EPSILON * w;
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        if (sturm_count(a, b, m, mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

/* Solve (T - lam I) z = rhs by Gaussian elimination with partial pivoting on
 * the tridiagonal band (a zero pivot is replaced by a tiny one, as is usual
 * for inverse iteration).  rhs is overwritten by z. */
static void tridiag_shift_solve(const double *a, const double *b, int m, double lam, double *rhs)
{
    double *dl = (double *)malloc(sizeof(double) * (size_t)m * 4);
    double *d = dl + m, *du = dl + 2 * m, *du2 = dl + 3 * m;
    double scale = 0.0;
    for (int i = 0; i < m; i++)
        scale = fmax(scale, fabs(a[i] - lam) + (i > 0 ? fabs(b[i]) : 0.0));
    double tiny = DBL_EPSILON * (scale > 0 ? scale : 1.0);
    for (int i = 0; i < m; i++) {
        d[i] = a[i] - lam;
        dl[i] = (i + 1 < m) ? b[i + 1] : 0.0; /* sub-diagonal entry (i+1, i) */
        du[i] = (i + 1 < m) ? b[i + 1] : 0.0; /* super-diagonal entry (i, i+1) */
        du2[i] = 0.0;
    }
    /* forward elimination */
    for (int i = 0; i + 1 < m; i++) {
        if (fabs(d[i]) >= fabs(dl[i])) {
            if (d[i] == 0.0)
                d[i] = tiny;
            double f = dl[i] / d[i];
            d[i + 1] -= f * du[i];
            rhs[i + 1] -= f * rhs[i];
            dl[i] = 0.0;
        } else {
            /* swap rows i and i+1 */
            double f = d[i] / dl[i];
            d[i] = dl[i];
            double t1 = d[i + 1];
            d[i + 1] = du[i] - f * t1;
            double t2 = (i + 2 < m) ? du[i + 1] : 0.0;
            du2[i] = t2;
            if (i + 2 < m)
                du[i + 1] = -f * t2;
            du[i] = t1;
            double r = rhs[i];
            rhs[i] = rhs[i + 1];
            rhs[i + 1] = r - f * rhs[i + 1];
        }
    }
    if (d[m - 1] == 0.0)
        d[m - 1] = tiny;
    /* back substitution */
    for (int i = m - 1; i >= 0; i--) {
        double s = rhs[i];
        if (i + 1 < m)
            s -= du[i] * rhs[i + 1];
        if (i + 2 < m)
            s -= du2[i] * rhs[i + 2];
        rhs[i] = s / d[i];
    }
    free(dl);
}

/* Unit eigenvector of T for eigenvalue lam by inverse iteration, with the sign
 * chosen so that its first component is positive. */
void orc_tridiag_vec(const double *a, const double *b, int m, double lam, double *y)
{
    for (int i = 0; i < m; i++)
        y[i] = 1.0;
    for (int it = 0; it < 4; it++) {
        tridiag_shift_solve(a, b, m, lam, y);
        /* scale by the largest entry first: near an eigenvalue the solve
         * returns entries close to overflow */
        double big = 0.0;
        for (int i = 0; i < m; i++)
            big = fmax(big, fabs(y[i]));
        for (int i = 0; i < m; i++)
            y[i] /= big;
        double nrm = 0.0;
        for (int i = 0; i < m; i++)
            nrm += y[i] * y[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; i++)
            y[i] /= nrm;
    }
    if (y[0] < 0.0)
        for (int i = 0; i < m; i++)
            y[i] = -y[i];
}

/* ----------------------------------------------------------------- Lanczos */

static double dot(const double *u, const double *v, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++)
        s += u[i] * v[i];
    return s;
}

typedef struct {
    int n_iter;       /* m: number of a_j produced */
    int converged;    /* 1: energy change within tol; 2: breakdown; 3: Krylov space exhausted; 0: max_iter */
    double e0;        /* lowest eigenvalue of T_m */
    double residual;  /* ||H psi - e0 psi||, when psi was requested */
    double rayleigh;  /* <psi|H|psi>, when psi was requested */
} orc_result;

/* The tridiagonal T of eq. Tmatrix (Sec. 2.2) comes from the three-term
 * relation that orthonormal Krylov vectors of a symmetric H obey,
 *     H f_j = b_j f_{j-1} + a_j f_j + b_{j+1} f_{j+1}   (f_0 = 0, b_1 = 0).
 * Given f_{j-1}, f_j and b_j, this finds the next coefficients: a_j is the
 * component along f_j of what H f_j leaves after its f_{j-1} part is taken
 * away, and b_{j+1} the length of the rest, which is left in r (it is
 * b_{j+1} f_{j+1}).  The paper's Alg. 1 is this relation run from a random
 * unit f_1 without re-orthogonalisation, as here. */
static void next_coefficients(const orc_model *m, const double *f_prev, const double *f, double b_j, double *r,
                              double *a_j, double *b_next)
{
    const int64_t n = m->dim;
    orc_apply(m, f, r);
    for (int64_t i = 0; i < n; i++)
        r[i] -= b_j * f_prev[i];
    const double a = dot(r, f, n);
    for (int64_t i = 0; i < n; i++)
        r[i] -= a * f[i];
    *a_j = a;
    *b_next = sqrt(dot(r, r, n));
}

/* Moves the pair of vectors one step on: f_{j-1} <- f_j, f_j <- r / b_{j+1}. */
static void shift_vectors(double *f_prev, double *f, const double *r, double b_next, int64_t n)
{
    for (int64_t i = 0; i < n; i++) {
        f_prev[i] = f[i];
        f[i] = r[i] / b_next;
    }
}

/* Lanczos from the unit start vector f1 (length dim): a[j-1] = a_j and
 * b[j-1] = b_{j+1} for j = 1..m; e_hist[j-1] = lowest eigenvalue of T_j.
 * Stops on the energy test of Sec. 2.2, on a vanishing b_{j+1}, when the
 * Krylov space is exhausted or at max_iter.  When psi is not NULL the
 * coefficients are produced a second time from f1 and psi = sum_j y_j f_j
 * is formed (y: the eigenvector of T_m for its lowest eigenvalue).
 * Returns 0, or -1 when memory runs out. */
int orc_lanczos(const orc_model *m, const double *f1, double tol, int max_iter,
                double *a, double *b, double *e_hist, double *psi, orc_result *res)
{
    int64_t n = m->dim;
    double *f_prev = (double *)calloc((size_t)n, sizeof(double));
    double *f_cur = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *boff = (double *)malloc(sizeof(double) * (size_t)(max_iter + 2)); /* boff[j] = b_j, boff[1] = 0 */
    if (!f_prev || !f_cur || !q || !boff) {
        free(f_prev); free(f_cur); free(q); free(boff);
        return -1;
    }
    memcpy(f_cur, f1, sizeof(double) * (size_t)n);
    memset(res, 0, sizeof(*res));
    boff[0] = 0.0;
    boff[1] = 0.0;
    double scale = 0.0, e_last = 0.0;
    int mm = 0;
    for (int j = 1; j <= max_iter; j++) {
        double aj, bj1;
        next_coefficients(m, f_prev, f_cur, boff[j], q, &aj, &bj1);
        a[j - 1] = aj;
        b[j - 1] = bj1;
        boff[j + 1] = bj1;
        mm = j;
        /* Ritz value of T_j (diagonal a_1..a_j, off-diagonal b_2..b_j) */
        double e = orc_tridiag_min(a, boff + 1, j);
        e_hist[j - 1] = e;
        /* a negative tol switches the energy test off (fixed iteration count) */
        if (tol >= 0.0 && j >= 2 && fabs(e - e_last) <= tol * fmax(1.0, fabs(e))) {
            res->converged = 1;
            break;
        }
        e_last = e;
        scale = fmax(scale, fabs(aj) + boff[j]);
        if (bj1 == 0.0 || bj1 <= 1e-12 * scale) {
            res->converged = 2;
            break;
        }
        if ((int64_t)j >= n) {
            res->converged = 3;
            break;
        }
        shift_vectors(f_prev, f_cur, q, bj1, n);
    }
    res->n_iter = mm;
    res->e0 = e_hist[mm - 1];

    if (psi) {
        double *y = (double *)malloc(sizeof(double) * (size_t)mm);
        orc_tridiag_vec(a, boff + 1, mm, res->e0, y);
        /* the Krylov vectors again, in the same arithmetic, each added to
         * psi with its weight y_j */
        memset(f_prev, 0, sizeof(double) * (size_t)n);
        memcpy(f_cur, f1, sizeof(double) * (size_t)n);
        memset(psi, 0, sizeof(double) * (size_t)n);
        for (int j = 1; j <= mm; j++) {
            for (int64_t i = 0; i < n; i++)
                psi[i] += y[j - 1] * f_cur[i];
            if (j == mm)
                break;
            double aj, bj1;
            next_coefficients(m, f_prev, f_cur, boff[j], q, &aj, &bj1);
            shift_vectors(f_prev, f_cur, q, bj1, n);
        }
        double nrm = sqrt(dot(psi, psi, n));
        for (int64_t i = 0; i < n; i++)
            psi[i] /= nrm;
        if (dot(psi, f1, n) < 0.0)
            for (int64_t i = 0; i < n; i++)
                psi[i] = -psi[i];
        /* residual ||H psi - E0 psi|| and Rayleigh quotient <psi|H|psi> */
        orc_apply(m, psi, q);
        res->rayleigh = dot(psi, q, n);
        double r2 = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double d = q[i] - res->e0 * psi[i];
            r2 += d * d;
        }
        res->residual = sqrt(r2);
        free(y);
    }
    free(f_prev);
    free(f_cur);
    free(q);
    free(boff);
    return 0;
}
