// Small dense FP64 linear algebra on the host (n <= a few hundred):
// Cholesky with dependent-pivot handling, triangular inverse and the
// one-sided Jacobi SVD (Hestenes), started from the eigenvectors of the
// Gram matrix.  Row-major storage.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "dense.h"

namespace rtt {

int cholesky_upper(const std::vector<double>& G, int n, double shift, double dead_tol, std::vector<double>& R,
                   std::vector<char>& dead)
{
    R.assign((size_t)n * n, 0.0);
    dead.assign(n, 0);
    double maxdiag = 0.0;
    for (int j = 0; j < n; ++j) maxdiag = std::max(maxdiag, G[(size_t)j * n + j]);
    int ndead = 0;
    for (int j = 0; j < n; ++j) {
        double d = G[(size_t)j * n + j] + shift;
        for (int k = 0; k < j; ++k) d -= R[(size_t)k * n + j] * R[(size_t)k * n + j];
        if (!(d > dead_tol * maxdiag) || maxdiag <= 0.0) {
            // dependent column: keep its projection coefficients R[k][j] (k < j),
            // zero diagonal, zero row (it spans no new direction)
            dead[j] = 1;
            ++ndead;
            R[(size_t)j * n + j] = 0.0;
            continue;
        }
        const double rjj = std::sqrt(d);
        R[(size_t)j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            double v = G[(size_t)j * n + i];
            for (int k = 0; k < j; ++k) v -= R[(size_t)k * n + j] * R[(size_t)k * n + i];
            R[(size_t)j * n + i] = v / rjj;
        }
    }
    return ndead;
}

void upper_inverse(const std::vector<double>& R, int n, const std::vector<char>& dead, std::vector<double>& Ri)
{
    Ri.assign((size_t)n * n, 0.0);
    // column by column back substitution: R * Ri[:, j] = e_j
    for (int j = 0; j < n; ++j) {
        if (dead[j]) continue;
        Ri[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
        for (int i = j - 1; i >= 0; --i) {
            if (dead[i]) continue;
            double v = 0.0;
            for (int k = i + 1; k <= j; ++k) v += R[(size_t)i * n + k] * Ri[(size_t)k * n + j];
            Ri[(size_t)i * n + j] = -v / R[(size_t)i * n + i];
        }
    }
}

void matmul(const std::vector<double>& A, const std::vector<double>& B, int n, std::vector<double>& C)
{
    C.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = A[(size_t)i * n + k];
            if (a == 0.0) continue;
            const double* b = &B[(size_t)k * n];
            double* c = &C[(size_t)i * n];
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
}

// Eigenvectors of a symmetric n x n matrix S (row-major, destroyed): Householder reduction to
// tridiagonal form T = Q^T S Q with Q accumulated, then implicit symmetric QR steps with the
// Wilkinson shift on T (Golub and Van Loan, Matrix Computations, Sec. 8.3), the Givens rotations
// applied to the columns of Q.  On return row j of Zt (n x n, row-major) is eigenvector j: Q is
// kept transposed so that every update runs along contiguous memory.  The eigenvalues are not
// needed by the caller.
static void sym_eigvectors(std::vector<double>& S, int n, std::vector<double>& Zt)
{
    std::vector<double>& Z = Zt;
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> d(n, 0.0), e(n, 0.0), v(n), p(n), w(n), q(n);
    auto A = [&](int i, int j) -> double& { return S[(size_t)i * n + j]; };
    // reduction: step k annihilates A[k+2:, k] with a reflector H = I - beta v v^T on rows k+1..
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;   // length of the active part
        double xn = 0.0;
        for (int i = 0; i < m; ++i) xn += A(k + 1 + i, k) * A(k + 1 + i, k);
        xn = std::sqrt(xn);
        const double x0 = A(k + 1, k);
        double beta = 0.0, alpha = x0;
        if (xn > 0.0) {
            alpha = x0 >= 0.0 ? -xn : xn;   // A[k+1,k] after the reflection
            // v = x - alpha e1 scaled so v[0] = 1
            const double v0 = x0 - alpha;
            v[0] = 1.0;
            for (int i = 1; i < m; ++i) v[i] = A(k + 1 + i, k) / v0;
            double vv = 0.0;
            for (int i = 0; i < m; ++i) vv += v[i] * v[i];
            beta = 2.0 / vv;
        }
        d[k] = A(k, k);
        e[k] = alpha;
        if (beta == 0.0) continue;
        // A22 <- H A22 H = A22 - v w^T - w v^T with p = beta A22 v, w = p - (beta/2)(p^T v) v
        double pv = 0.0;
        for (int i = 0; i < m; ++i) {
            double t = 0.0;
            for (int j = 0; j < m; ++j) t += A(k + 1 + i, k + 1 + j) * v[j];
            p[i] = beta * t;
            pv += p[i] * v[i];
        }
        for (int i = 0; i < m; ++i) w[i] = p[i] - 0.5 * beta * pv * v[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) A(k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
        // Q <- Q H on columns k+1.. (rows k+1.. of Qt)
        for (int r = 0; r < n; ++r) q[r] = 0.0;
        for (int j = 0; j < m; ++j) {
            const double* zj = &Z[(size_t)(k + 1 + j) * n];
            for (int r = 0; r < n; ++r) q[r] += zj[r] * v[j];
        }
        for (int j = 0; j < m; ++j) {
            double* zj = &Z[(size_t)(k + 1 + j) * n];
            const double bv = beta * v[j];
            for (int r = 0; r < n; ++r) zj[r] -= q[r] * bv;
        }
    }
    if (n >= 2) {
        d[n - 2] = A(n - 2, n - 2);
        e[n - 2] = A(n - 1, n - 2);
    }
    d[n - 1] = A(n - 1, n - 1);
    e[n - 1] = 0.0;
    // implicit QR on the tridiagonal (d, e): e[i] couples i and i+1
    const double eps = 2.3e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0 && guard < 64 * n) {
        // deflate converged off-diagonals at the bottom
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        ++guard;
        // Wilkinson shift from the trailing 2 x 2 block of [lo, hi]
        const double dd = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation in the plane (k, k+1) that zeroes z against x
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            const double a = d[k], b = e[k], d2 = d[k + 1];
            d[k] = c * c * a + 2.0 * c * sn * b + sn * sn * d2;
            d[k + 1] = sn * sn * a - 2.0 * c * sn * b + c * c * d2;
            e[k] = c * sn * (d2 - a) + (c * c - sn * sn) * b;
            if (k + 1 < hi) {
                z = sn * e[k + 1];   // bulge at (k+2, k)
                e[k + 1] *= c;
                x = e[k];
            }
            double* zk = &Z[(size_t)k * n];
            double* zk1 = &Z[(size_t)(k + 1) * n];
            for (int r2 = 0; r2 < n; ++r2) {
                const double u0 = zk[r2], u1 = zk1[r2];
                zk[r2] = c * u0 + sn * u1;
                zk1[r2] = -sn * u0 + c * u1;
            }
        }
    }
}

void jacobi_svd(const std::vector<double>& M, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& W)
{
    // work on columns: a[j] = column j of the working matrix (contiguous), v[j] = column j of W.
    // The sweeps start from M Z, Z the eigenvectors of M^T M: its columns are already nearly
    // orthogonal, so the one-sided Jacobi that follows (and sets the accuracy) needs few sweeps.
    std::vector<double> a((size_t)n * n, 0.0), v((size_t)n * n, 0.0);
    {
        std::vector<double> G((size_t)n * n, 0.0), Z;
        for (int k = 0; k < n; ++k) {
            const double* mk = &M[(size_t)k * n];
            for (int i = 0; i < n; ++i) {
                const double mi = mk[i];
                if (mi == 0.0) continue;
                double* gi = &G[(size_t)i * n];
                for (int j = 0; j < n; ++j) gi[j] += mi * mk[j];
            }
        }
        sym_eigvectors(G, n, Z);   // row j of Z: eigenvector j
        v = Z;
        for (int i = 0; i < n; ++i) {
            const double* mi = &M[(size_t)i * n];
            for (int j = 0; j < n; ++j) {
                const double* zj = &v[(size_t)j * n];
                double t = 0.0;
                for (int k = 0; k < n; ++k) t += mi[k] * zj[k];
                a[(size_t)j * n + i] = t;
            }
        }
    }
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += a[(size_t)j * n + i] * a[(size_t)j * n + i];
        nrm[j] = t;
    }
    const double eps = 1e-15;
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rot = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double* ap = &a[(size_t)p * n];
                double* aq = &a[(size_t)q * n];
                double g = 0.0;
                for (int i = 0; i < n; ++i) g += ap[i] * aq[i];
                const double al = nrm[p], be = nrm[q];
                if (std::fabs(g) <= eps * std::sqrt(al * be) || g == 0.0) continue;
                ++rot;
                const double zeta = (be - al) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                double np = 0.0, nq = 0.0;
                for (int i = 0; i < n; ++i) {
                    const double x = ap[i], y = aq[i];
                    const double xn = c * x - sn * y, yn = sn * x + c * y;
                    ap[i] = xn;
                    aq[i] = yn;
                    np += xn * xn;
                    nq += yn * yn;
                }
                nrm[p] = np;
                nrm[q] = nq;
                double* vp = &v[(size_t)p * n];
                double* vq = &v[(size_t)q * n];
                for (int i = 0; i < n; ++i) {
                    const double x = vp[i], y = vq[i];
                    vp[i] = c * x - sn * y;
                    vq[i] = sn * x + c * y;
                }
            }
        }
        if (rot == 0) break;
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::vector<double> sv(n);
    for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += a[(size_t)j * n + i] * a[(size_t)j * n + i];
        sv[j] = std::sqrt(t);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sv[x] > sv[y]; });
    U.assign((size_t)n * n, 0.0);
    W.assign((size_t)n * n, 0.0);
    s.assign(n, 0.0);
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        s[jj] = sv[j];
        for (int i = 0; i < n; ++i) {
            U[(size_t)i * n + jj] = sv[j] > 0.0 ? a[(size_t)j * n + i] / sv[j] : 0.0;
            W[(size_t)i * n + jj] = v[(size_t)j * n + i];
        }
    }
}

}  // namespace rtt
