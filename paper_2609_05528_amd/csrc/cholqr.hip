// Cholesky QR factors on the device, FP64 (the orthonormalisation step of the randomized
// subspace iteration and of block Lanczos: Halko, Martinsson & Tropp 2011, Alg. 4.4 / 5.1;
// the singular values of Sec. 3.6 eq. (19) and Sec. 4.4 eq. (31)).  For ns independent
// problems at once, each an lp x lp Gram matrix G = Y Y^T (lp a multiple of 32, at most 512):
//
//   k_chol_factor   G = R^T R (R upper), one workgroup per problem: panels of 32 rows, each
//                   factored by all threads (one column per thread, in registers), the rows below
//                   it then updated from the panel kept in LDS.
//                   Every entry receives its terms in increasing row order (the order of the
//                   textbook column formula), product and difference rounded separately.  Pivots
//                   at or below dead_tol * max diag(G) mark dependent columns: zero diagonal and
//                   row, their projection coefficients R[k][j] (k < j) kept.  On a first pass a pivot below
//                   1e-5 max diag(G) (past the FP32 accuracy of the Gram matrix) re-factors
//                   G + 1e-6 max diag(G) I and flags one more pass (shifted CholQR3, Fukaya et
//                   al. 2020); the extra pass runs only where that flag is set.
//   k_chol_diag_inv / k_chol_offdiag_inv
//                   R^-1 on the independent columns (dependent rows and columns zero), blocked:
//                   the 32 x 32 diagonal blocks by back substitution, then block column J from
//                   X_IJ = -R_II^-1 sum_{K=I+1..J} R_IK X_KJ for I = J-1 .. 0; written in FP64 and
//                   in FP32 for the MFMA combine Q = Y R^-1.
//   k_upper_product C = A B for upper triangular A, B (the accumulated factor of a final basis).
//
// Everything is stream-ordered: no host synchronisation, no memset nodes, and the
// conditional pass is decided on the device.
#include <algorithm>

#include "dense.h"

namespace rtt {

namespace {

constexpr int CB = 32;           // panel rows / block size
constexpr int CQ_MAX = 512;      // largest lp
constexpr int PW = CQ_MAX - CB;  // columns right of a panel, at most

__device__ __forceinline__ double uniform_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Materialise the column held in registers at this point: without it the compiler may defer the
// right-looking updates of a fully unrolled factorisation into long chains that keep every step's
// operands alive (and spill them).
__device__ __forceinline__ void pin_column(double (&s)[CB])
{
#pragma unroll
    for (int i = 0; i < CB; ++i) asm volatile("" : "+v"(s[i]));
}

// max (op 0) or min (op 1) over the workgroup (at most 1024 threads); every thread gets the result
__device__ double block_reduce(double v, int op, double* red)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = op == 0 ? fmax(v, w) : fmin(v, w);
    }
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = op == 0 ? fmax(r, red[w]) : fmin(r, red[w]);
    return r;
}

// mode 0: first pass (may shift, sets st[q]); 1: plain pass; 2: the conditional pass (only where
// st[q] != 0).  S: scratch lp x lp per problem.  R: lp x lp per problem, written in full (zero
// below the diagonal).  dead: lp flags per problem.  512 threads.
__global__ __launch_bounds__(512) void k_chol_factor(const double* __restrict__ G, double* __restrict__ S,
                                                     double* __restrict__ R, int* __restrict__ dead,
                                                     int* __restrict__ st, int lp, int mode, double dead_tol)
{
#pragma clang fp contract(off)
    const int q = blockIdx.x;
    if (mode == 2 && st[q] == 0) return;
    const size_t lp2 = (size_t)lp * lp;
    G += q * lp2;
    S += q * lp2;
    R += q * lp2;
    dead += (size_t)q * lp;
    __shared__ double P[CB * PW];         // rows p0 .. p1 - 1 of R right of the panel: P[j][l - p1]
    __shared__ double rowbuf[CB + 1];     // row j of the diagonal block, and the pivot
    __shared__ double red[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nwaves = blockDim.x >> 6;

    double md = 0.0;
    for (int j = t; j < lp; j += blockDim.x) md = fmax(md, G[(size_t)j * lp + j]);
    const double maxdiag = uniform_f64(block_reduce(md, 0, red));
    const double tol = dead_tol * maxdiag;
    const bool all_dead = !(maxdiag > 0.0);

    double shift = 0.0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        // flat over the entries, unrolled so that a thread has eight loads of G in flight (one
        // load-store round trip per entry had left this copy latency-bound)
        const int n2 = lp * lp;
#pragma unroll 8
        for (int e = t; e < n2; e += (int)blockDim.x) {
            const double g = G[e];
            S[e] = e % (lp + 1) == 0 ? g + shift : g;
            R[e] = 0.0;
        }
        __syncthreads();
        for (int p0 = 0; p0 < lp; p0 += CB) {
            const int p1 = p0 + CB;
            // 1. the panel's rows p0 .. p1 - 1, right-looking, one column p0 + t per thread
            //    (columns left of the diagonal compute zeros): at step j the pivot comes from the
            //    thread of column p0 + j, every column forms its R[j][.], and the rows j+1 .. 31
            //    of each column are updated with the diagonal block's R[j][i] from LDS.  Two
            //    barriers per step.
            const int ncol = lp - p0;
            int tc = t;
            asm volatile("" : "+v"(tc));   // opaque per panel: keeps the per-step masks in the loop
            const bool act = tc < ncol;
            const int lcol = p0 + (act ? tc : 0);
            double s[CB];
#pragma unroll
            for (int i = 0; i < CB; ++i) s[i] = act ? S[(size_t)(p0 + i) * lp + lcol] : 0.0;
            int my_dead = 0;
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                if (tc == j) rowbuf[CB] = s[j];
                __syncthreads();
                const double d = rowbuf[CB];
                const bool dj = !(d > tol) || all_dead;
                const double rjj = sqrt(dj ? 1.0 : d);
                const double qv = s[j] / rjj;
                const double r = dj ? 0.0 : (tc == j ? rjj : (tc > j ? qv : 0.0));
                if (tc < CB) rowbuf[tc] = r;
                my_dead = tc == j ? (dj ? 1 : 0) : my_dead;
                __syncthreads();
#pragma unroll
                for (int i = j + 1; i < CB; ++i) s[i] -= rowbuf[i] * r;   // rows i > column: never read
                if (act) {
                    R[(size_t)(p0 + j) * lp + lcol] = r;
                    if (tc >= CB) P[j * PW + tc - CB] = r;
                }
                pin_column(s);
            }
            if (tc < CB) dead[p0 + tc] = my_dead;
            __syncthreads();
            // 2. rows below the panel: S[i][l] -= R[j][i] R[j][l] for the panel's rows j in
            //    increasing order, l >= i; an item is TR rows x 64 columns of one wave, and the
            //    wave loads its next item's entries while it computes the current one
            constexpr int TR = 4;
            const int nr = lp - p1;
            const int ngrp = (nr + 63) / 64, nrg = (nr + TR - 1) / TR;
            const int nitem = nrg * ngrp;
            // items of this wave that lie (partly) on or above the diagonal
            auto next_item = [&](int it) {
                for (; it < nitem; it += nwaves)
                    if (64 * (it % ngrp) + 63 >= TR * (it / ngrp)) break;
                return it;
            };
            int item = next_item(wave);
            double nxt[TR];
            auto load_item = [&](int it, double (&v)[TR]) {
                const int ii0 = TR * (it / ngrp), cc = 64 * (it % ngrp) + lane;
#pragma unroll
                for (int r = 0; r < TR; ++r) {
                    const bool ok = ii0 + r < nr && cc >= ii0 + r && cc < nr;
                    v[r] = ok ? S[(size_t)(p1 + ii0 + r) * lp + p1 + cc] : 0.0;
                }
            };
            if (item < nitem) load_item(item, nxt);
            while (item < nitem) {
                const int ii0 = TR * (item / ngrp), cc = 64 * (item % ngrp) + lane;
                double acc[TR];
#pragma unroll
                for (int r = 0; r < TR; ++r) acc[r] = nxt[r];
                const int following = next_item(item + nwaves);
                if (following < nitem) load_item(following, nxt);
                const int ccl = min(cc, nr - 1);
                int rr[TR];
#pragma unroll
                for (int r = 0; r < TR; ++r) rr[r] = min(ii0 + r, nr - 1);
#pragma unroll 4
                for (int j = 0; j < CB; ++j) {
                    const double pj = P[j * PW + ccl];
#pragma unroll
                    for (int r = 0; r < TR; ++r) acc[r] -= P[j * PW + rr[r]] * pj;
                }
#pragma unroll
                for (int r = 0; r < TR; ++r)
                    if (ii0 + r < nr && cc >= ii0 + r && cc < nr) S[(size_t)(p1 + ii0 + r) * lp + p1 + cc] = acc[r];
                item = following;
            }
            __syncthreads();
        }
        if (mode != 0 || attempt == 1) break;
        // first pass: the smallest independent pivot against the FP32 accuracy of the Gram matrix
        double mp = INFINITY;
        for (int j = t; j < lp; j += blockDim.x)
            if (!dead[j]) {
                const double r = R[(size_t)j * lp + j];
                mp = fmin(mp, r * r);
            }
        const double minpiv = block_reduce(mp, 1, red);
        const bool shifted = minpiv < 1e-5 * maxdiag;
        if (t == 0) st[q] = shifted ? 1 : 0;
        if (!shifted) break;
        shift = 1e-6 * maxdiag;
        __syncthreads();
    }
}

// The inverses of the 32 x 32 diagonal blocks of R (one wave per block; lane c solves column c
// by back substitution, sums in increasing k).  Ri and Ri32: lp x lp per problem.
__global__ __launch_bounds__(64) void k_chol_diag_inv(const double* __restrict__ R, const int* __restrict__ dead,
                                                      const int* __restrict__ st, int lp, int mode,
                                                      double* __restrict__ Ri, float* __restrict__ Ri32)
{
    const int q = blockIdx.y, b0 = blockIdx.x * CB;
    if (mode == 2 && st[q] == 0) return;
    const size_t lp2 = (size_t)lp * lp;
    R += q * lp2;
    Ri += q * lp2;
    Ri32 += q * lp2;
    dead += (size_t)q * lp;
    __shared__ double D[CB][CB + 1];
    __shared__ int dd[CB];
    const int c = threadIdx.x;
    for (int e = c; e < CB * CB; e += 64) D[e / CB][e % CB] = R[(size_t)(b0 + e / CB) * lp + b0 + e % CB];
    if (c < CB) dd[c] = dead[b0 + c];
    __syncthreads();
    if (c >= CB) return;
    const bool dc = dd[c] != 0;
    double x[CB];
#pragma unroll
    for (int i = CB - 1; i >= 0; --i) {
        double xi = 0.0;
        if (!dc && i == c) xi = 1.0 / D[c][c];
        if (!dc && i < c && !dd[i]) {
            double v = 0.0;
#pragma unroll
            for (int k = i + 1; k < CB; ++k)
                if (k <= c) v += D[i][k] * x[k];
            xi = v == 0.0 ? 0.0 : -v / D[i][i];
        }
        x[i] = xi;
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
        Ri[(size_t)(b0 + i) * lp + b0 + c] = x[i];
        Ri32[(size_t)(b0 + i) * lp + b0 + c] = (float)x[i];
    }
}

// Block column J of R^-1 above its diagonal block, and zeros below it.  One workgroup of 1024
// threads per (J, problem); thread (a, b) owns entry (a, b) of the 32 x 32 block being formed.  At
// step I every thread first loads its element of each 32 x 32 block R_IK (K = I+1 .. J) into
// registers -- one round trip for all of them -- and the blocks then pass through LDS one by one.
__global__ __launch_bounds__(1024) void k_chol_offdiag_inv(const double* __restrict__ R, const int* __restrict__ st,
                                                           int lp, int mode, double* __restrict__ Ri,
                                                           float* __restrict__ Ri32)
{
    const int q = blockIdx.y, J = blockIdx.x;
    if (mode == 2 && st[q] == 0) return;
    const size_t lp2 = (size_t)lp * lp;
    R += q * lp2;
    Ri += q * lp2;
    Ri32 += q * lp2;
    constexpr int KMAX = CQ_MAX / CB - 1;   // blocks right of a block row, at most
    __shared__ double X[CQ_MAX * CB];       // rows 0 .. (J + 1) * 32 - 1 of block column J
    __shared__ double T[CB][CB + 1];
    __shared__ double Rb[CB][CB + 1];       // one block R_IK
    const int t = threadIdx.x, a = t >> 5, b = t & 31;
    const int j = J * CB + b;
    // below the diagonal block: zero
    for (int i = (J + 1) * CB + a; i < lp; i += CB) {
        Ri[(size_t)i * lp + j] = 0.0;
        Ri32[(size_t)i * lp + j] = 0.f;
    }
    X[(J * CB + a) * CB + b] = Ri[(size_t)(J * CB + a) * lp + j];
    __syncthreads();
    for (int I = J - 1; I >= 0; --I) {
        // element (a, b) of R_IK for K = I+1 .. J
        double rk[KMAX];
#pragma unroll
        for (int K = 0; K < KMAX; ++K)
            if (K < J - I) rk[K] = R[(size_t)(I * CB + a) * lp + (I + 1 + K) * CB + b];
        // T = sum_{K = I+1 .. J} R_IK X_KJ, terms in increasing column order
        double acc = 0.0;
#pragma unroll
        for (int K = 0; K < KMAX; ++K) {
            if (K >= J - I) break;
            Rb[a][b] = rk[K];
            __syncthreads();
            const int k0 = (I + 1 + K) * CB;
#pragma unroll 8
            for (int u = 0; u < CB; ++u) acc += Rb[a][u] * X[(k0 + u) * CB + b];
            __syncthreads();
        }
        T[a][b] = acc;
        // row a of R_II^-1 (zero left of the diagonal)
        const double dv = Ri[(size_t)(I * CB + a) * lp + I * CB + b];
        Rb[a][b] = dv;
        __syncthreads();
        // X_IJ = -R_II^-1 T
        double x = 0.0;
#pragma unroll 8
        for (int c = 0; c < CB; ++c)
            if (c >= a) x += Rb[a][c] * T[c][b];
        x = -x;
        X[(I * CB + a) * CB + b] = x;
        Ri[(size_t)(I * CB + a) * lp + j] = x;
        Ri32[(size_t)(I * CB + a) * lp + j] = (float)x;
        __syncthreads();
    }
}

// C = A B (A, B upper triangular lp x lp; C upper, zero below the diagonal): C[i][j] = sum_{k=i..j}
// A[i][k] B[k][j] in increasing k.  Mode 2: C = B where st[q] == 0 (no conditional pass there).
// One workgroup per 32 x 32 tile (I, J) of C; thread (a, b) owns its entry.
__global__ __launch_bounds__(1024) void k_upper_product(const double* __restrict__ A, const double* __restrict__ B,
                                                        const int* __restrict__ st, int lp, int mode,
                                                        double* __restrict__ C)
{
    const int q = blockIdx.z, I = blockIdx.y, J = blockIdx.x;
    const size_t lp2 = (size_t)lp * lp;
    A += q * lp2;
    B += q * lp2;
    C += q * lp2;
    const int i = I * CB + (threadIdx.x >> 5), j = J * CB + (threadIdx.x & 31);
    double v = 0.0;
    if (mode == 2 && st[q] == 0) v = B[(size_t)i * lp + j];
    else if (I <= J) {
        const double* ai = &A[(size_t)i * lp];
        // batches of 8 loads ahead of their products (latency); terms past j are skipped
        for (int k0 = i; k0 <= j; k0 += 8) {
            double av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = min(k0 + u, j);
                av[u] = ai[k];
                bv[u] = B[(size_t)k * lp + j];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u <= j && av[u] != 0.0) v += av[u] * bv[u];
        }
    }
    C[(size_t)i * lp + j] = v;
}

__global__ void k_identity_f64(double* __restrict__ R, int lp, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t r = e % ((int64_t)lp * lp);
    R[e] = (r / lp == r % lp) ? 1.0 : 0.0;
}

// grid-stride over the rows (blockIdx.y) and columns: a small grid, so that the launch costs
// little when *run_if == 0
__global__ void k_copy_rows_if(const int* __restrict__ run_if, const float* __restrict__ src, float* __restrict__ dst,
                               int64_t ld, int rows, int64_t len)
{
    if (!*run_if) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y)
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < len; c += (int64_t)gridDim.x * blockDim.x)
            dst[r * ld + c] = src[r * ld + c];
}

}  // namespace

int chol_factor(const double* G, int lp, int ns, int mode, double dead_tol, double* S, double* R, int* dead, int* st,
                hipStream_t s)
{
    if (lp % CB || lp <= 0 || lp > CQ_MAX || ns <= 0) return fail(RTT_EINVAL, "chol_factor: bad size");
    // 512 threads: one per column right of a panel (at most 480), 256 registers each for the
    // panel column held in registers
    hipLaunchKernelGGL(k_chol_factor, dim3((unsigned)ns), dim3(512), 0, s, G, S, R, dead, st, lp, mode, dead_tol);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int chol_inverse(const double* R, const int* dead, const int* st, int lp, int ns, int mode, double* Ri, float* Ri32,
                 hipStream_t s)
{
    if (lp % CB || lp <= 0 || lp > CQ_MAX || ns <= 0) return fail(RTT_EINVAL, "chol_inverse: bad size");
    const dim3 grid((unsigned)(lp / CB), (unsigned)ns);
    hipLaunchKernelGGL(k_chol_diag_inv, grid, dim3(64), 0, s, R, dead, st, lp, mode, Ri, Ri32);
    hipLaunchKernelGGL(k_chol_offdiag_inv, grid, dim3(1024), 0, s, R, st, lp, mode, Ri, Ri32);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int upper_product(const double* A, const double* B, const int* st, int lp, int ns, int mode, double* C, hipStream_t s)
{
    if (lp % CB || lp <= 0 || lp > CQ_MAX || ns <= 0) return fail(RTT_EINVAL, "upper_product: bad size");
    hipLaunchKernelGGL(k_upper_product, dim3((unsigned)(lp / CB), (unsigned)(lp / CB), (unsigned)ns), dim3(1024), 0, s,
                       A, B, st, lp, mode, C);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int identity_f64(double* R, int lp, int ns, hipStream_t s)
{
    const int64_t n = (int64_t)lp * lp * ns;
    if (n <= 0) return RTT_OK;
    hipLaunchKernelGGL(k_identity_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R, lp, n);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int copy_rows_if(const int* run_if, const float* src, float* dst, int64_t ld, int rows, int64_t len, hipStream_t s)
{
    if (rows <= 0 || len <= 0) return RTT_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(64, (len + 255) / 256);
    const unsigned gy = (unsigned)std::min(rows, 64);
    hipLaunchKernelGGL(k_copy_rows_if, dim3(gx, gy), dim3(256), 0, s, run_if, src, dst, ld, rows, len);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

}  // namespace rtt
