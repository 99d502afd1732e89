// Ridge (Tikhonov) estimator of Sec. 9: conjugate gradients on the normal
// equations (A^T A + lambda I) x = A^T y.  For a handle with G geometries the
// normal equations are block diagonal, so every (right-hand side, geometry)
// pair runs its own CG with its own step lengths: the same iterates as G
// separate solves.  Every iteration is one block application of A and of A^T
// (all pairs at once) plus FP64 dot products per pair; step lengths live in
// device memory.  The blocking mode looks at the residuals every few
// iterations from the host; the stream-ordered mode runs a fixed number of
// iterations with no host synchronisation (pairs that have converged stop
// changing) so that a whole solve can be captured into a graph.
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

// scalar index of (right-hand side v, geometry g): v * G + g
__global__ void k_cg_alpha(const double* rr, const double* pap, const int* done, double* alpha, int npair)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= npair) return;
    alpha[v] = (done[v] || !(pap[v] > 0.0)) ? 0.0 : rr[v] / pap[v];
}

// grid (column blocks of the longest geometry, right-hand sides, geometries)
__global__ void k_cg_xr(float* __restrict__ x, float* __restrict__ r, const float* __restrict__ p,
                        const float* __restrict__ Ap, const double* __restrict__ alpha,
                        const int64_t* __restrict__ seg, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y, g = blockIdx.z, G = gridDim.z;
    if (i >= seg[2 * g + 1]) return;
    const float a = (float)alpha[(int64_t)v * G + g];
    if (a != 0.f) {
        const int64_t o = (int64_t)v * n + seg[2 * g] + i;
        x[o] += a * p[o];
        r[o] -= a * Ap[o];
    }
}

__global__ void k_cg_beta(double* rr, const double* rr_new, const double* bb, const double* pap, int* done,
                          double* beta, int npair, double tol2)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= npair) return;
    if (done[v]) {
        beta[v] = 0.0;
        return;
    }
    beta[v] = rr[v] > 0.0 ? rr_new[v] / rr[v] : 0.0;
    rr[v] = rr_new[v];
    if (rr_new[v] <= tol2 * bb[v] || !(pap[v] > 0.0)) done[v] = 1;
}

__global__ void k_cg_p(float* __restrict__ p, const float* __restrict__ r, const double* __restrict__ beta,
                       const int* __restrict__ done, const int64_t* __restrict__ seg, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y, g = blockIdx.z, G = gridDim.z;
    if (i >= seg[2 * g + 1]) return;
    const int64_t pi = (int64_t)v * G + g;
    if (!done[pi]) {
        const int64_t o = (int64_t)v * n + seg[2 * g] + i;
        p[o] = r[o] + (float)beta[pi] * p[o];
    }
}

// start: rr = bb = |A^T y|^2 per pair; a pair with bb = 0 (y orthogonal to the range) is done
__global__ void k_cg_init(double* rr, double* bb, int* done, int npair)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= npair) return;
    bb[v] = rr[v];
    done[v] = rr[v] > 0.0 ? 0 : 1;
}

__global__ void k_cg_resid(const double* rr, const double* bb, float* out, int npair)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= npair) return;
    out[v] = bb[v] > 0.0 ? (float)sqrt(rr[v] / bb[v]) : 0.f;
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
    const int32_t flags = opts ? opts->flags : 0;
    float* resid_dev = opts ? opts->resid_dev : nullptr;
    const bool async = (flags & RTT_SOLVE_ASYNC) != 0;
    if (!(tol > 0.0f) || maxit < 1) return fail(RTT_EINVAL, "need tol > 0 and maxit >= 1");
    if (flags & ~(RTT_SOLVE_ASYNC | RTT_SOLVE_NORMAL_RHS)) return fail(RTT_EINVAL, "unknown ridge_solve flags");
    const bool normal_rhs = (flags & RTT_SOLVE_NORMAL_RHS) != 0;
    if (info) *info = rtt_solve_info{0, 0, 0.f, 0};
    if (nrhs == 0) return RTT_OK;
    hipStream_t s = (hipStream_t)stream;
    const int G = (int)g->members.size();
    const int npair = nrhs * G;
    const int64_t n = g->n_cols, m = g->n_rows;
    int64_t max_cols = 0;
    for (const Member& mb : g->members) max_cols = std::max(max_cols, mb.n_cols);
    Workspace local;
    if (async && !g->solve_ws) g->solve_ws = new (std::nothrow) Workspace();
    Workspace& ws = async ? *g->solve_ws : local;
    if (async && !g->solve_ws) return fail(RTT_ENOMEM, "ridge_solve workspace");
    float* r = (float*)ws.get("cg_r", sizeof(float) * (size_t)nrhs * n);
    float* p = (float*)ws.get("cg_p", sizeof(float) * (size_t)nrhs * n);
    float* Ap = (float*)ws.get("cg_ap", sizeof(float) * (size_t)nrhs * n);
    float* q = (float*)ws.get("cg_q", sizeof(float) * (size_t)nrhs * m);
    double* sc = (double*)ws.get("cg_scal", sizeof(double) * 6 * npair);
    int* done = (int*)ws.get("cg_done", sizeof(int) * npair);
    if (!r || !p || !Ap || !q || !sc || !done) return fail(RTT_ENOMEM, "ridge_solve workspace");
    double *rr = sc, *rr_new = sc + npair, *bb = sc + 2 * npair, *pap = sc + 3 * npair, *alpha = sc + 4 * npair,
           *beta = sc + 5 * npair;
    const int64_t* seg = g->d_seg;   // column blocks
    int rc;
    const dim3 vgrid((unsigned)((n + 255) / 256), (unsigned)nrhs);
    const dim3 mgrid((unsigned)((max_cols + 255) / 256), (unsigned)nrhs, (unsigned)G);
    const dim3 sgrid((unsigned)((npair + 127) / 128));
    auto pair_dots = [&](const float* a, const float* b, double* out) {
        return dots_seg(ws, a, n, b, n, seg, G, max_cols, nrhs, out, s);
    };
    // x = 0, r = A^T y (or the given normal-equation right-hand side), p = r
    if ((rc = fill(x, (int64_t)nrhs * n, 0.f, s))) return rc;
    if (normal_rhs) {
        RTT_HIP(hipMemcpyAsync(r, y, sizeof(float) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, s));
    } else if ((rc = apply_op(g, -1, true, y, r, nrhs, mask, s))) {
        return rc;
    }
    RTT_HIP(hipMemcpyAsync(p, r, sizeof(float) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, s));
    if ((rc = pair_dots(r, r, rr))) return rc;
    hipLaunchKernelGGL(k_cg_init, sgrid, dim3(128), 0, s, rr, bb, done, npair);
    const double tol2 = (double)tol * (double)tol;
    std::vector<double> h_rr(npair), h_bb(npair);
    std::vector<int> h_done(npair);
    int it = 0;
    if (!async) {
        RTT_HIP(hipMemcpyAsync(h_done.data(), done, sizeof(int) * npair, hipMemcpyDeviceToHost, s));
        RTT_HIP(hipStreamSynchronize(s));
        if (std::all_of(h_done.begin(), h_done.end(), [](int d) { return d != 0; })) {
            if (info) *info = rtt_solve_info{0, npair, 0.f, 0};
            return RTT_OK;
        }
    }
    const int check_every = 8;
    while (it < maxit) {
        if ((rc = apply_op(g, -1, false, p, q, nrhs, mask, s))) return rc;
        if ((rc = apply_op(g, -1, true, q, Ap, nrhs, mask, s))) return rc;
        if (lambda != 0.f) hipLaunchKernelGGL(k_axpy_lambda, vgrid, dim3(256), 0, s, Ap, p, n, lambda);
        if ((rc = pair_dots(p, Ap, pap))) return rc;
        hipLaunchKernelGGL(k_cg_alpha, sgrid, dim3(128), 0, s, rr, pap, done, alpha, npair);
        hipLaunchKernelGGL(k_cg_xr, mgrid, dim3(256), 0, s, x, r, p, Ap, alpha, seg, n);
        if ((rc = pair_dots(r, r, rr_new))) return rc;
        hipLaunchKernelGGL(k_cg_beta, sgrid, dim3(128), 0, s, rr, rr_new, bb, pap, done, beta, npair, tol2);
        hipLaunchKernelGGL(k_cg_p, mgrid, dim3(256), 0, s, p, r, beta, done, seg, n);
        RTT_HIP(hipGetLastError());
        ++it;
        if (!async && (it % check_every == 0 || it == maxit)) {
            RTT_HIP(hipMemcpyAsync(h_done.data(), done, sizeof(int) * npair, hipMemcpyDeviceToHost, s));
            RTT_HIP(hipStreamSynchronize(s));
            if (std::all_of(h_done.begin(), h_done.end(), [](int d) { return d != 0; })) break;
        }
    }
    if (resid_dev) hipLaunchKernelGGL(k_cg_resid, sgrid, dim3(128), 0, s, rr, bb, resid_dev, npair);
    RTT_HIP(hipGetLastError());
    if (async) {
        if (info) *info = rtt_solve_info{it, -1, -1.f, 0};
        return RTT_OK;
    }
    RTT_HIP(hipMemcpyAsync(h_rr.data(), rr, sizeof(double) * npair, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipMemcpyAsync(h_bb.data(), bb, sizeof(double) * npair, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipMemcpyAsync(h_done.data(), done, sizeof(int) * npair, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    int ndone = 0;
    for (int v = 0; v < npair; ++v) {
        if (h_bb[v] > 0.0) worst = std::max(worst, std::sqrt(h_rr[v] / h_bb[v]));
        ndone += h_done[v] ? 1 : 0;
    }
    if (info) *info = rtt_solve_info{it, ndone, (float)worst, 0};
    if (ndone < npair) return fail(RTT_ENOCONV, "ridge_solve: CG did not reach tol within maxit");
    return RTT_OK;
}

extern "C" int noise_add(float* y, int64_t n, uint64_t seed, float sigma, void* stream)
{
    if (n < 0) return fail(RTT_EINVAL, "n must be >= 0");
    if (n > 0 && !y) return fail(RTT_EINVAL, "NULL data pointer");
    if (!std::isfinite(sigma)) return fail(RTT_EINVAL, "sigma must be finite");
    return normal_add(y, n, seed, sigma, (hipStream_t)stream);
}
