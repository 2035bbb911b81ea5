// Lowest eigenpair of the Lanczos tridiagonal matrix T (Siro & Harju,
// Sec. 2.2, eq. Tmatrix: diagonal a_1..a_m, off-diagonal b_2..b_m).
//
// Eigenvalue: bisection on the inertia of T - x I.  The number of negative
// pivots of the LDL^T factorisation of T - x I equals the number of
// eigenvalues below x (Sylvester's law of inertia), so the lowest eigenvalue
// is the smallest x at which that count becomes 1.
// Eigenvector: inverse iteration with the shifted matrix factorised by
// Gaussian elimination with row interchanges.
#include <cfloat>
#include <cmath>
#include <vector>

#include "internal.h"

namespace hub {

static int negative_pivots(const double *d, const double *e, int m, double x)
{
    int neg = 0;
    double piv = d[0] - x;
    const double floor_piv = 1e-290;
    if (std::fabs(piv) < floor_piv)
        piv = -floor_piv;
    neg += piv < 0;
    for (int i = 1; i < m; i++) {
        piv = (d[i] - x) - e[i - 1] * (e[i - 1] / piv);
        if (std::fabs(piv) < floor_piv)
            piv = -floor_piv;
        neg += piv < 0;
    }
    return neg;
}

double tridiag_lowest(const double *d, const double *e, int m)
{
    // Gershgorin interval
    double lo = d[0], hi = d[0];
    for (int i = 0; i < m; i++) {
        double rad = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(e[i]) : 0.0);
        lo = std::fmin(lo, d[i] - rad);
        hi = std::fmax(hi, d[i] + rad);
    }
    double pad = DBL_EPSILON * (std::fabs(lo) + std::fabs(hi)) + 1e-290;
    lo -= pad;
    hi += pad;
    while (true) {
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi))
            break;
        if (negative_pivots(d, e, m, mid) > 0)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

void tridiag_lowest_vector(const double *d, const double *e, int m, double lam, double *y)
{
    if (m == 1) {
        y[0] = 1.0;
        return;
    }
    // LU with partial pivoting of the band of T - lam I: U has up to two
    // super-diagonals (u0 = diagonal, u1, u2), L multipliers l[i], swap[i].
    std::vector<double> u0(m), u1(m), u2(m), l(m);
    std::vector<char> swap(m, 0);
    double nrmT = 0.0;
    for (int i = 0; i < m; i++)
        nrmT = std::fmax(nrmT, std::fabs(d[i] - lam) + (i ? std::fabs(e[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(e[i]) : 0.0));
    const double tiny = DBL_EPSILON * (nrmT > 0 ? nrmT : 1.0);

    double cur0 = d[0] - lam, cur1 = e[0];  // current row's diagonal and super-diagonal
    for (int i = 0; i < m - 1; i++) {
        double below0 = e[i], below1 = d[i + 1] - lam, below2 = (i + 1 < m - 1) ? e[i + 1] : 0.0;
        if (std::fabs(cur0) >= std::fabs(below0)) {
            if (cur0 == 0.0)
                cur0 = tiny;
            double f = below0 / cur0;
            u0[i] = cur0;
            u1[i] = cur1;
            u2[i] = 0.0;
            l[i] = f;
            cur0 = below1 - f * cur1;
            cur1 = below2;
        } else {
            double f = cur0 / below0;
            swap[i] = 1;
            u0[i] = below0;
            u1[i] = below1;
            u2[i] = below2;
            l[i] = f;
            cur0 = cur1 - f * below1;
            cur1 = -f * below2;
        }
    }
    u0[m - 1] = (cur0 == 0.0) ? tiny : cur0;
    u1[m - 1] = u2[m - 1] = 0.0;

    std::vector<double> v(m, 1.0);
    for (int it = 0; it < 4; it++) {
        // forward: apply the row interchanges and multipliers
        for (int i = 0; i < m - 1; i++) {
            if (swap[i]) {
                double tmp = v[i];
                v[i] = v[i + 1];
                v[i + 1] = tmp - l[i] * v[i + 1];
            } else {
                v[i + 1] -= l[i] * v[i];
            }
        }
        // backward
        for (int i = m - 1; i >= 0; i--) {
            double s = v[i];
            if (i + 1 < m)
                s -= u1[i] * v[i + 1];
            if (i + 2 < m)
                s -= u2[i] * v[i + 2];
            v[i] = s / u0[i];
        }
        double mx = 0.0;
        for (int i = 0; i < m; i++)
            mx = std::fmax(mx, std::fabs(v[i]));
        double ss = 0.0;
        for (int i = 0; i < m; i++) {
            v[i] /= mx;
            ss += v[i] * v[i];
        }
        double inv = 1.0 / std::sqrt(ss);
        for (int i = 0; i < m; i++)
            v[i] *= inv;
    }
    double sg = v[0] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < m; i++)
        y[i] = sg * v[i];
}

}  // namespace hub
