// Small dense FP64 linear algebra on the host (n <= a few hundred):
// Cholesky with dependent-pivot handling, triangular inverse and the
// one-sided Jacobi SVD (Hestenes).  Row-major storage.
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

void jacobi_svd(const std::vector<double>& M, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& W)
{
    // work on columns: a[j] = column j of M (contiguous), v[j] = column j of W
    std::vector<double> a((size_t)n * n), v((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)j * n + i] = M[(size_t)i * n + j];
    for (int j = 0; j < n; ++j) v[(size_t)j * n + j] = 1.0;
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
