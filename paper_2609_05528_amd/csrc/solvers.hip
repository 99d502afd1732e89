// Ridge (Tikhonov) estimator of Sec. 9: conjugate gradients on the normal
// equations (A^T A + lambda I) x = A^T y, one independent CG per right-hand
// side.  Every iteration is one block application of A and of A^T (all
// right-hand sides at once) plus FP64 dot products; the step lengths live in
// device memory, so the host only looks at the residuals every few iterations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.h"

namespace rtt {

__global__ void k_axpy_lambda(float* __restrict__ Ap, const float* __restrict__ p, int64_t n, float lam)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t off = (int64_t)blockIdx.y * n;
    if (i < n) Ap[off + i] += lam * p[off + i];
}

__global__ void k_cg_alpha(const double* rr, const double* pap, const int* done, double* alpha, int nrhs)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nrhs) return;
    alpha[v] = (done[v] || !(pap[v] > 0.0)) ? 0.0 : rr[v] / pap[v];
}

__global__ void k_cg_xr(float* __restrict__ x, float* __restrict__ r, const float* __restrict__ p,
                        const float* __restrict__ Ap, const double* __restrict__ alpha, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    const float a = (float)alpha[v];
    if (i < n && a != 0.f) {
        const int64_t o = (int64_t)v * n + i;
        x[o] += a * p[o];
        r[o] -= a * Ap[o];
    }
}

__global__ void k_cg_beta(double* rr, const double* rr_new, const double* bb, const double* pap, int* done,
                          double* beta, int nrhs, double tol2)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nrhs) return;
    if (done[v]) {
        beta[v] = 0.0;
        return;
    }
    beta[v] = rr[v] > 0.0 ? rr_new[v] / rr[v] : 0.0;
    rr[v] = rr_new[v];
    if (rr_new[v] <= tol2 * bb[v] || !(pap[v] > 0.0)) done[v] = 1;
}

__global__ void k_cg_p(float* __restrict__ p, const float* __restrict__ r, const double* __restrict__ beta,
                       const int* __restrict__ done, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (i < n && !done[v]) {
        const int64_t o = (int64_t)v * n + i;
        p[o] = r[o] + (float)beta[v] * p[o];
    }
}

}  // namespace rtt

using namespace rtt;

extern "C" int ridge_solve(const rtt_geometry* g, const float* y, int32_t nrhs, float lambda,
                           const rtt_cg_opts* opts, float* x, rtt_solve_info* info, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (nrhs < 0 || nrhs > 4096) return fail(RTT_EINVAL, "nrhs must be 0..4096");
    if (nrhs > 0 && (!y || !x)) return fail(RTT_EINVAL, "NULL data pointer");
    if (!(lambda >= 0.0f) || !std::isfinite(lambda)) return fail(RTT_EINVAL, "lambda must be finite and >= 0");
    const float tol = opts ? opts->tol : 1e-6f;
    const int maxit = opts ? opts->maxit : 1000;
    const uint32_t mask = opts ? opts->order_mask : 0u;
    if (!(tol > 0.0f) || maxit < 1) return fail(RTT_EINVAL, "need tol > 0 and maxit >= 1");
    if (info) *info = rtt_solve_info{0, 0, 0.f, 0};
    if (nrhs == 0) return RTT_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n_cols, m = g->n_rows;
    Workspace ws;
    float* r = (float*)ws.get("cg_r", sizeof(float) * (size_t)nrhs * n);
    float* p = (float*)ws.get("cg_p", sizeof(float) * (size_t)nrhs * n);
    float* Ap = (float*)ws.get("cg_ap", sizeof(float) * (size_t)nrhs * n);
    float* q = (float*)ws.get("cg_q", sizeof(float) * (size_t)nrhs * m);
    double* sc = (double*)ws.get("cg_scal", sizeof(double) * 7 * nrhs);
    int* done = (int*)ws.get("cg_done", sizeof(int) * nrhs);
    if (!r || !p || !Ap || !q || !sc || !done) return fail(RTT_ENOMEM, "ridge_solve workspace");
    double *rr = sc, *rr_new = sc + nrhs, *bb = sc + 2 * nrhs, *pap = sc + 3 * nrhs, *alpha = sc + 4 * nrhs,
           *beta = sc + 5 * nrhs;
    int rc;
    const dim3 vgrid((unsigned)((n + 255) / 256), (unsigned)nrhs);
    const dim3 sgrid((unsigned)((nrhs + 127) / 128));
    // x = 0, r = A^T y, p = r
    RTT_HIP(hipMemsetAsync(x, 0, sizeof(float) * (size_t)nrhs * n, s));
    RTT_HIP(hipMemsetAsync(done, 0, sizeof(int) * nrhs, s));
    if ((rc = apply_op(g, -1, true, y, r, nrhs, mask, s))) return rc;
    RTT_HIP(hipMemcpyAsync(p, r, sizeof(float) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, s));
    if ((rc = dots(ws, r, n, r, n, n, nrhs, rr, s))) return rc;
    RTT_HIP(hipMemcpyAsync(bb, rr, sizeof(double) * nrhs, hipMemcpyDeviceToDevice, s));
    const double tol2 = (double)tol * (double)tol;
    std::vector<double> h_rr(nrhs), h_bb(nrhs);
    std::vector<int> h_done(nrhs);
    RTT_HIP(hipMemcpyAsync(h_bb.data(), bb, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipStreamSynchronize(s));
    int it = 0, ndone = 0;
    for (int v = 0; v < nrhs; ++v)
        if (h_bb[v] == 0.0) ++ndone;   // y in the null space of A^T: x = 0 is exact
    if (ndone == nrhs) {
        if (info) *info = rtt_solve_info{0, nrhs, 0.f, 0};
        return RTT_OK;
    }
    const int check_every = 8;
    while (it < maxit) {
        if ((rc = apply_op(g, -1, false, p, q, nrhs, mask, s))) return rc;
        if ((rc = apply_op(g, -1, true, q, Ap, nrhs, mask, s))) return rc;
        if (lambda != 0.f) hipLaunchKernelGGL(k_axpy_lambda, vgrid, dim3(256), 0, s, Ap, p, n, lambda);
        if ((rc = dots(ws, p, n, Ap, n, n, nrhs, pap, s))) return rc;
        hipLaunchKernelGGL(k_cg_alpha, sgrid, dim3(128), 0, s, rr, pap, done, alpha, nrhs);
        hipLaunchKernelGGL(k_cg_xr, vgrid, dim3(256), 0, s, x, r, p, Ap, alpha, n);
        if ((rc = dots(ws, r, n, r, n, n, nrhs, rr_new, s))) return rc;
        hipLaunchKernelGGL(k_cg_beta, sgrid, dim3(128), 0, s, rr, rr_new, bb, pap, done, beta, nrhs, tol2);
        hipLaunchKernelGGL(k_cg_p, vgrid, dim3(256), 0, s, p, r, beta, done, n);
        RTT_HIP(hipGetLastError());
        ++it;
        if (it % check_every == 0 || it == maxit) {
            RTT_HIP(hipMemcpyAsync(h_done.data(), done, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
            RTT_HIP(hipStreamSynchronize(s));
            ndone = 0;
            for (int v = 0; v < nrhs; ++v) ndone += (h_done[v] || h_bb[v] == 0.0) ? 1 : 0;
            if (ndone == nrhs) break;
        }
    }
    RTT_HIP(hipMemcpyAsync(h_rr.data(), rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipMemcpyAsync(h_done.data(), done, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    ndone = 0;
    for (int v = 0; v < nrhs; ++v) {
        if (h_bb[v] > 0.0) worst = std::max(worst, std::sqrt(h_rr[v] / h_bb[v]));
        ndone += (h_done[v] || h_bb[v] == 0.0) ? 1 : 0;
    }
    if (info) *info = rtt_solve_info{it, ndone, (float)worst, 0};
    if (ndone < nrhs) return fail(RTT_ENOCONV, "ridge_solve: CG did not reach tol within maxit");
    return RTT_OK;
}
