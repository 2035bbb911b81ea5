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

namespace hub {

// c = exp(-i tau T) e_1 for the symmetric tridiagonal T (diagonal d[0..m-1],
// off-diagonal e[0..m-2]): T = Z diag(w) Z^T by cyclic Jacobi rotations on the
// dense m x m matrix (Golub and Van Loan, Matrix Computations, the cyclic
// Jacobi method), then c = Z diag(exp(-i tau w)) Z^T e_1.  m is small (the
// Krylov dimension of one propagation step), so O(m^3) per sweep is nothing.
void tridiag_expm_e1(const double *d, const double *e, int m, double tau, double *c_re, double *c_im)
{
    std::vector<double> A((size_t)m * m, 0.0), Z((size_t)m * m, 0.0);
    for (int i = 0; i < m; i++) {
        A[(size_t)i * m + i] = d[i];
        Z[(size_t)i * m + i] = 1.0;
        if (i + 1 < m) {
            A[(size_t)i * m + i + 1] = e[i];
            A[(size_t)(i + 1) * m + i] = e[i];
        }
    }
    double fro = 0.0;
    for (double v : A)
        fro += v * v;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0;
        for (int p = 0; p < m; p++)
            for (int q = p + 1; q < m; q++)
                off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
        if (off <= 1e-34 * fro || off == 0.0)
            break;
        for (int p = 0; p < m; p++)
            for (int q = p + 1; q < m; q++) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0)
                    continue;
                const double theta = (A[(size_t)q * m + q] - A[(size_t)p * m + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(1.0 + theta * theta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // A <- J^T A J with J the rotation in the (p, q) plane
                for (int k = 0; k < m; k++) {
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; k++) {
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; k++) {
                    const double zkp = Z[(size_t)k * m + p], zkq = Z[(size_t)k * m + q];
                    Z[(size_t)k * m + p] = c * zkp - s * zkq;
                    Z[(size_t)k * m + q] = s * zkp + c * zkq;
                }
            }
    }
    for (int i = 0; i < m; i++) {
        c_re[i] = 0.0;
        c_im[i] = 0.0;
    }
    for (int k = 0; k < m; k++) {
        const double w = A[(size_t)k * m + k];
        const double z0 = Z[k];  // Z[0][k]
        const double pr = std::cos(tau * w) * z0, pi = -std::sin(tau * w) * z0;
        for (int i = 0; i < m; i++) {
            c_re[i] += Z[(size_t)i * m + k] * pr;
            c_im[i] += Z[(size_t)i * m + k] * pi;
        }
    }
}

}  // namespace hub
