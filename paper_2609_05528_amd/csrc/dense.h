// Dense building blocks of the spectral drivers (device kernels in dense.hip and cholqr.hip; the
// small FP64 SVDs on the host in smallla.cpp).
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

// G (device, FP64, M x N row-major) = A B^T with A: M rows, B: N rows of length L.  run_if (device,
// optional): the kernels do nothing when *run_if == 0 (a pass decided on the device).
int gram(Workspace& ws, const float* A, int64_t lda, const float* B, int64_t ldb, int M, int N, int64_t L,
         double* G_dev, hipStream_t s, const int* run_if = nullptr);
// Out[m][l] = beta*Out[m][l] + sum_k C[k][m] Y[k][l]; C device FP32 K x M row-major.  upper: the
// caller guarantees C[k][m] = 0 for k > m (e.g. an upper triangular R^-1), and those terms are skipped.
// run_if as for gram.
int combine(const float* C, int K, int M, const float* Y, int64_t ldy, float* Out, int64_t ldo, int64_t L,
            float beta, hipStream_t s, bool upper = false, const int* run_if = nullptr);

// Cholesky QR factors on the device (cholqr.hip), FP64, for ns independent lp x lp Gram matrices
// stored one after another (lp a multiple of 32, at most 512).  mode 0: first pass (pivots below
// 1e-5 max diag re-factor with a 1e-6 max diag shift and set st[q] = 1, else st[q] = 0); mode 1: a
// further pass; mode 2: the conditional pass, only for problems with st[q] != 0 (the others are
// left untouched).  dead_tol: pivots at or below dead_tol * max diag mark dependent columns
// (dead[q*lp + j] = 1; zero diagonal and row).  S is lp x lp scratch per problem.
int chol_factor(const double* G, int lp, int ns, int mode, double dead_tol, double* S, double* R, int* dead, int* st,
                hipStream_t s);
// Ri = R^-1 on the independent columns (dependent rows and columns zero), FP64 and FP32 copies.
int chol_inverse(const double* R, const int* dead, const int* st, int lp, int ns, int mode, double* Ri, float* Ri32,
                 hipStream_t s);
// C = A B for upper triangular A, B; in mode 2, C = B for problems with st[q] == 0.
int upper_product(const double* A, const double* B, const int* st, int lp, int ns, int mode, double* C, hipStream_t s);
// ns identity matrices lp x lp.
int identity_f64(double* R, int lp, int ns, hipStream_t s);
// dst = src over rows x len (row stride ld) when *run_if != 0.
int copy_rows_if(const int* run_if, const float* src, float* dst, int64_t ld, int rows, int64_t len, hipStream_t s);
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

// host FP64 small dense linear algebra (row-major n x n)
// One-sided Jacobi SVD of an n x n row-major matrix M = U diag(s) W^T, s descending.
void jacobi_svd(const std::vector<double>& M, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& W);
// f(0) .. f(n - 1), each once, on the host thread pool (at most 16 threads); returns when all have
// finished.  Calls made from inside f run serially in their thread.
void host_for(int n, const std::function<void(int)>& f);

}  // namespace rtt
