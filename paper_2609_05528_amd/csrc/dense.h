// Dense building blocks of the spectral drivers (device kernels in dense.hip,
// small FP64 factorisations on the host in smallla.cpp).
#pragma once

#include <functional>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "rtt_internal.h"

namespace rtt {

// Named, grow-only device scratch buffers owned by one driver call.
struct Workspace {
    std::map<std::string, std::pair<void*, size_t>> bufs;
    void* get(const char* name, size_t bytes);
    void release();
    ~Workspace();
};

// G (device, FP64, M x N row-major) = A B^T with A: M rows, B: N rows of length L.
int gram(Workspace& ws, const float* A, int64_t lda, const float* B, int64_t ldb, int M, int N, int64_t L,
         double* G_dev, hipStream_t s);
// Out[m][l] = beta*Out[m][l] + sum_k C[k][m] Y[k][l]; C device FP32 K x M row-major.  upper: the
// caller guarantees C[k][m] = 0 for k > m (e.g. an upper triangular R^-1), and those terms are skipped.
int combine(const float* C, int K, int M, const float* Y, int64_t ldy, float* Out, int64_t ldo, int64_t L,
            float beta, hipStream_t s, bool upper = false);
// out[v] = <a_v, b_v> in FP64 for nvec vectors of length n.
int dots(Workspace& ws, const float* a, int64_t lda, const float* b, int64_t ldb, int64_t n, int nvec,
         double* out_dev, hipStream_t s);
// out[v*G + g] = <a_v, b_v> over segment g (device table seg[2g] = offset, seg[2g+1] = length,
// max_len >= every length), FP64, deterministic.
int dots_seg(Workspace& ws, const float* a, int64_t lda, const float* b, int64_t ldb, const int64_t* seg_dev,
             int G, int64_t max_len, int nvec, double* out_dev, hipStream_t s);
// p[0..n) = v with a kernel (safe inside captured graphs, unlike memset nodes).
int fill(float* p, int64_t n, float v, hipStream_t s);
// C[set][i][r] = Cd[set][i][r] / sigma[set*k + i]^2 if sigma >= sigma_min and > 0, else 0 (FP64 in, FP32 out).
int scale_inv_sq(const double* Cd, const double* sigma_dev, int sets, int t, int k, int nrhs, double sigma_min,
                 float* C, hipStream_t s);
// N(0,1) FP32 draws from Philox-4x32-10 counters (seeded).
int normal_fill(float* out, int64_t n, uint64_t seed, hipStream_t s);
// y[i] += sigma * (the same draws)
int normal_add(float* y, int64_t n, uint64_t seed, float sigma, hipStream_t s);

// host FP64 small dense linear algebra (column-major n x n unless stated)
// Cholesky G = R^T R of a symmetric n x n (row-major) matrix; pivots below
// dead_tol * max diag mark dependent columns (reported in dead[]): their
// diagonal and row of R are zero and their projection coefficients R[k][j]
// (k < j) are kept.  shift is added to the diagonal.  Returns the number of
// dependent columns.
int cholesky_upper(const std::vector<double>& G, int n, double shift, double dead_tol, std::vector<double>& R,
                   std::vector<char>& dead);
// Inverse of R on the independent columns: dependent rows/columns of the result are zero.
void upper_inverse(const std::vector<double>& R, int n, const std::vector<char>& dead, std::vector<double>& Rinv);
// One-sided Jacobi SVD of an n x n row-major matrix M = U diag(s) W^T, s descending.
void jacobi_svd(const std::vector<double>& M, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& W);
// f(0) .. f(n - 1), each once, on the host thread pool (at most 16 threads); returns when all have
// finished.  Calls made from inside f run serially in their thread.
void host_for(int n, const std::function<void(int)>& f);
// C = A B for n x n row-major matrices.
void matmul(const std::vector<double>& A, const std::vector<double>& B, int n, std::vector<double>& C);
// C = A B for upper triangular A and B (n x n row-major); the strictly lower part of C is zero.
void matmul_upper(const std::vector<double>& A, const std::vector<double>& B, int n, std::vector<double>& C);

}  // namespace rtt
