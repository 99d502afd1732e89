// Spectral drivers (Sec. 3.6 eq. (19), Sec. 4.4 eq. (31)) and the TSVD estimator (Sec. 9).
//
// rsvd, RTT_SVD_RSVD: randomized subspace iteration (Halko, Martinsson &
// Tropp, SIAM Rev. 2011, Alg. 4.4) with l = k + p test vectors and q power
// iterations, followed by their Alg. 5.1: B^T = A^T Q, B^T = Qb R, SVD of
// R^T = Ur S W^T, so B = Ur S (Qb W)^T.  Every block is orthonormalised by
// Cholesky QR: the Gram matrix comes from the FP32 MFMA kernel with FP64
// slice reduction, the Cholesky factor and its inverse are FP64 (host), the
// triangular apply is the MFMA combine kernel.  Two passes (CholQR2); when the
// first Gram matrix is too ill-conditioned for FP32 a diagonal shift is added
// in the first pass and a third pass follows (shifted CholQR3, Fukaya et al.
// 2020).  Columns that are numerically dependent are dropped (zeroed).
//
// rsvd, RTT_SVD_BLOCK_LANCZOS: block Golub-Kahan bidiagonalisation with the
// right (coefficient-space) basis stored and reorthogonalised twice against
// every previous block; the projected block-bidiagonal matrix is
// diagonalised by an FP64 one-sided Jacobi SVD and the Ritz vectors are
// formed on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "dense.h"

using namespace rtt;

struct rtt_svd {
    uint32_t magic = 0x53564431u;
    int k = 0;
    int member = -1;
    int64_t n_rows = 0, n_cols = 0;
    std::vector<double> sigma, resid;
    float* V = nullptr;
    float* U = nullptr;
    ~rtt_svd()
    {
        if (V) hipFree(V);
        if (U) hipFree(U);
    }
};

namespace {

struct Ctx {
    const rtt_geometry* g;
    int member;
    uint32_t mask;
    int64_t n_rows, n_cols;
    hipStream_t s;
    Workspace ws;
};

int pad32(int n) { return (n + 31) / 32 * 32; }

// download an FP64 device matrix after the stream's work is done
int download(Ctx& c, const double* d, std::vector<double>& h, size_t n)
{
    h.resize(n);
    RTT_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, c.s));
    RTT_HIP(hipStreamSynchronize(c.s));
    return RTT_OK;
}

// upload an FP64 host matrix (rows x cols, row-major) as FP32
int upload_f32(Ctx& c, const char* name, const std::vector<double>& h, size_t n, float** out)
{
    float* d = (float*)c.ws.get(name, n * sizeof(float));
    if (!d) return fail(RTT_ENOMEM, "upload buffer");
    // pinned staging through a host vector; small (<= 512 x 512)
    std::vector<float> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (float)h[i];
    RTT_HIP(hipMemcpyAsync(d, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, c.s));
    RTT_HIP(hipStreamSynchronize(c.s));
    *out = d;
    return RTT_OK;
}

// Orthonormalise the l (padded to lp) vectors of length n stored in *Y (row
// stride n), using *T as ping-pong storage; on return *Y holds Q.  R_total
// (lp x lp, row-major, upper) receives the accumulated triangular factor with
// Y = Q R_total on the retained columns.
int orth(Ctx& c, float** Y, float** T, int lp, int64_t n, std::vector<double>& R_total, int* n_dead)
{
    double* Gd = (double*)c.ws.get("orth_gram", sizeof(double) * lp * lp);
    if (!Gd) return fail(RTT_ENOMEM, "orth gram");
    R_total.assign((size_t)lp * lp, 0.0);
    for (int i = 0; i < lp; ++i) R_total[(size_t)i * lp + i] = 1.0;
    int passes = 2;
    std::vector<double> G, R, Ri, Rt;
    std::vector<char> dead;
    for (int pass = 0; pass < passes; ++pass) {
        int rc = gram(c.ws, *Y, n, *Y, n, lp, lp, n, Gd, c.s);
        if (rc) return rc;
        if ((rc = download(c, Gd, G, (size_t)lp * lp))) return rc;
        double maxdiag = 0.0;
        for (int i = 0; i < lp; ++i) maxdiag = std::max(maxdiag, G[(size_t)i * lp + i]);
        double shift = 0.0;
        const double dead_tol = pass == 0 ? 1e-12 : 1e-8;
        int nd = cholesky_upper(G, lp, 0.0, dead_tol, R, dead);
        if (pass == 0) {
            // a pivot below the FP32 Gram accuracy: shift the first pass and add a third one
            double minpiv = INFINITY;
            for (int i = 0; i < lp; ++i)
                if (!dead[i]) minpiv = std::min(minpiv, R[(size_t)i * lp + i] * R[(size_t)i * lp + i]);
            if (minpiv < 1e-5 * maxdiag) {
                shift = 1e-6 * maxdiag;
                nd = cholesky_upper(G, lp, shift, dead_tol, R, dead);
                passes = 3;
            }
        }
        if (n_dead) *n_dead = nd;
        upper_inverse(R, lp, dead, Ri);
        float* Cd = nullptr;
        if ((rc = upload_f32(c, "orth_rinv", Ri, (size_t)lp * lp, &Cd))) return rc;
        if ((rc = combine(Cd, lp, lp, *Y, n, *T, n, n, 0.f, c.s))) return rc;
        std::swap(*Y, *T);
        matmul(R, R_total, lp, Rt);
        R_total.swap(Rt);
    }
    return RTT_OK;
}

float* dev_alloc(Ctx& c, const char* name, size_t n)
{
    return (float*)c.ws.get(name, n * sizeof(float));
}

int apply(Ctx& c, bool adjoint, const float* in, float* out, int nvec)
{
    return apply_op(c.g, c.member, adjoint, in, out, nvec, c.mask, c.s);
}

int run_rsvd(Ctx& c, const rtt_svd_opts& o, const float* omega, rtt_svd* res)
{
    const int l = o.k + o.p, lp = pad32(l);
    const int64_t n = c.n_cols, m = c.n_rows;
    float* X = dev_alloc(c, "rs_x", (size_t)lp * n);
    float* X2 = dev_alloc(c, "rs_x2", (size_t)lp * n);
    float* Y = dev_alloc(c, "rs_y", (size_t)lp * m);
    float* Y2 = dev_alloc(c, "rs_y2", (size_t)lp * m);
    if (!X || !X2 || !Y || !Y2) return fail(RTT_ENOMEM, "rsvd block buffers");
    RTT_HIP(hipMemsetAsync(X, 0, sizeof(float) * lp * n, c.s));
    RTT_HIP(hipMemsetAsync(Y, 0, sizeof(float) * lp * m, c.s));
    RTT_HIP(hipMemsetAsync(X2, 0, sizeof(float) * lp * n, c.s));
    RTT_HIP(hipMemsetAsync(Y2, 0, sizeof(float) * lp * m, c.s));
    if (omega) RTT_HIP(hipMemcpyAsync(X, omega, sizeof(float) * l * n, hipMemcpyDeviceToDevice, c.s));
    else {
        int rc = normal_fill(X, (int64_t)l * n, o.seed, c.s);
        if (rc) return rc;
    }
    std::vector<double> R;
    int rc;
    // Y = A Omega; Q = orth(Y)
    if ((rc = apply(c, false, X, Y, l))) return rc;
    if ((rc = orth(c, &Y, &Y2, lp, m, R, nullptr))) return rc;
    for (int it = 0; it < o.q; ++it) {
        if ((rc = apply(c, true, Y, X, l))) return rc;
        if ((rc = orth(c, &X, &X2, lp, n, R, nullptr))) return rc;
        if ((rc = apply(c, false, X, Y, l))) return rc;
        if ((rc = orth(c, &Y, &Y2, lp, m, R, nullptr))) return rc;
    }
    // B^T = A^T Q = Qb R
    if ((rc = apply(c, true, Y, X, l))) return rc;
    if ((rc = orth(c, &X, &X2, lp, n, R, nullptr))) return rc;
    // SVD of R^T (l x l leading block)
    std::vector<double> Mt((size_t)l * l), Ur, s, W;
    for (int i = 0; i < l; ++i)
        for (int j = 0; j < l; ++j) Mt[(size_t)i * l + j] = R[(size_t)j * lp + i];
    jacobi_svd(Mt, l, Ur, s, W);
    const int k = o.k;
    res->k = k;
    res->sigma.assign(s.begin(), s.begin() + k);
    res->resid.assign(k, 0.0);
    // V = Qb W[:, :k] ; U = Q Ur[:, :k]
    std::vector<double> Wk((size_t)l * k), Uk((size_t)l * k);
    for (int i = 0; i < l; ++i)
        for (int j = 0; j < k; ++j) {
            Wk[(size_t)i * k + j] = W[(size_t)i * l + j];
            Uk[(size_t)i * k + j] = Ur[(size_t)i * l + j];
        }
    float* Cw = nullptr;
    if ((rc = upload_f32(c, "rs_w", Wk, Wk.size(), &Cw))) return rc;
    RTT_HIP(hipMalloc((void**)&res->V, sizeof(float) * (size_t)k * n));
    if ((rc = combine(Cw, l, k, X, n, res->V, n, n, 0.f, c.s))) return rc;
    if (o.keep_u) {
        float* Cu = nullptr;
        if ((rc = upload_f32(c, "rs_u", Uk, Uk.size(), &Cu))) return rc;
        RTT_HIP(hipMalloc((void**)&res->U, sizeof(float) * (size_t)k * m));
        if ((rc = combine(Cu, l, k, Y, m, res->U, m, m, 0.f, c.s))) return rc;
        // residuals || A v_i - sigma_i u_i ||
        float* AV = Y2;
        if ((rc = apply(c, false, res->V, AV, k))) return rc;
        double* d = (double*)c.ws.get("rs_dots", sizeof(double) * 3 * k);
        if (!d) return fail(RTT_ENOMEM, "dots");
        if ((rc = dots(c.ws, AV, m, AV, m, m, k, d, c.s))) return rc;
        if ((rc = dots(c.ws, AV, m, res->U, m, m, k, d + k, c.s))) return rc;
        if ((rc = dots(c.ws, res->U, m, res->U, m, m, k, d + 2 * k, c.s))) return rc;
        std::vector<double> h;
        if ((rc = download(c, d, h, 3 * (size_t)k))) return rc;
        for (int i = 0; i < k; ++i) {
            const double si = res->sigma[i];
            res->resid[i] = std::sqrt(std::max(0.0, h[i] - 2 * si * h[k + i] + si * si * h[2 * k + i]));
        }
    }
    RTT_HIP(hipStreamSynchronize(c.s));
    return RTT_OK;
}

int run_lanczos(Ctx& c, const rtt_svd_opts& o, const float* start, rtt_svd* res)
{
    const int b = o.block, steps = o.steps, mdim = b * steps;
    const int bp = pad32(b);
    const int64_t n = c.n_cols, m = c.n_rows;
    if (b % 32) return fail(RTT_EINVAL, "Lanczos block size must be a multiple of 32");
    float* Vall = dev_alloc(c, "lz_v", (size_t)mdim * n);
    float* Z = dev_alloc(c, "lz_z", (size_t)bp * n);
    float* Z2 = dev_alloc(c, "lz_z2", (size_t)bp * n);
    float* W = dev_alloc(c, "lz_w", (size_t)bp * m);
    float* W2 = dev_alloc(c, "lz_w2", (size_t)bp * m);
    float* Up = dev_alloc(c, "lz_up", (size_t)bp * m);
    double* Cd = (double*)c.ws.get("lz_coef", sizeof(double) * (size_t)mdim * bp);
    if (!Vall || !Z || !Z2 || !W || !W2 || !Up || !Cd) return fail(RTT_ENOMEM, "Lanczos buffers");
    int rc;
    if (start) RTT_HIP(hipMemcpyAsync(Z, start, sizeof(float) * b * n, hipMemcpyDeviceToDevice, c.s));
    else if ((rc = normal_fill(Z, (int64_t)b * n, o.seed, c.s))) return rc;
    std::vector<double> R, L, Rprev, T((size_t)mdim * mdim, 0.0), coef;
    if ((rc = orth(c, &Z, &Z2, b, n, R, nullptr))) return rc;
    RTT_HIP(hipMemcpyAsync(Vall, Z, sizeof(float) * b * n, hipMemcpyDeviceToDevice, c.s));
    bool have_prev = false;
    for (int j = 0; j < steps; ++j) {
        const float* Vj = Vall + (size_t)j * b * n;
        // W = A V_j - U_{j-1} R_{j-1}^T
        if ((rc = apply(c, false, Vj, W, b))) return rc;
        if (have_prev) {
            std::vector<double> C((size_t)b * b);
            for (int kk = 0; kk < b; ++kk)
                for (int mm = 0; mm < b; ++mm) C[(size_t)kk * b + mm] = -Rprev[(size_t)mm * b + kk];
            float* Cf = nullptr;
            if ((rc = upload_f32(c, "lz_c1", C, C.size(), &Cf))) return rc;
            if ((rc = combine(Cf, b, b, Up, m, W, m, m, 1.f, c.s))) return rc;
        }
        if ((rc = orth(c, &W, &W2, b, m, L, nullptr))) return rc;   // W now holds U_j
        for (int i = 0; i < b; ++i)
            for (int jj = 0; jj < b; ++jj) T[(size_t)(j * b + i) * mdim + j * b + jj] = L[(size_t)i * b + jj];
        // Z = A^T U_j - V_j L_j^T
        if ((rc = apply(c, true, W, Z, b))) return rc;
        {
            std::vector<double> C((size_t)b * b);
            for (int kk = 0; kk < b; ++kk)
                for (int mm = 0; mm < b; ++mm) C[(size_t)kk * b + mm] = -L[(size_t)mm * b + kk];
            float* Cf = nullptr;
            if ((rc = upload_f32(c, "lz_c2", C, C.size(), &Cf))) return rc;
            if ((rc = combine(Cf, b, b, Vj, n, Z, n, n, 1.f, c.s))) return rc;
        }
        // reorthogonalise twice against all stored right blocks
        const int nv = (j + 1) * b;
        for (int pass = 0; pass < 2; ++pass) {
            if ((rc = gram(c.ws, Vall, n, Z, n, nv, b, n, Cd, c.s))) return rc;
            if ((rc = download(c, Cd, coef, (size_t)nv * b))) return rc;
            for (auto& v : coef) v = -v;
            float* Cf = nullptr;
            if ((rc = upload_f32(c, "lz_c3", coef, coef.size(), &Cf))) return rc;
            if ((rc = combine(Cf, nv, b, Vall, n, Z, n, n, 1.f, c.s))) return rc;
        }
        if ((rc = orth(c, &Z, &Z2, b, n, R, nullptr))) return rc;   // Z = V_{j+1}, R_j
        if (j + 1 < steps) {
            for (int i = 0; i < b; ++i)
                for (int jj = 0; jj < b; ++jj)
                    T[(size_t)(j * b + i) * mdim + (j + 1) * b + jj] = R[(size_t)jj * b + i];
            RTT_HIP(hipMemcpyAsync(Vall + (size_t)(j + 1) * b * n, Z, sizeof(float) * b * n,
                                   hipMemcpyDeviceToDevice, c.s));
        }
        std::swap(Up, W);   // U_j becomes the previous left block
        Rprev = R;
        have_prev = true;
    }
    std::vector<double> P, s, Wt;
    jacobi_svd(T, mdim, P, s, Wt);
    const int k = std::min(o.k, mdim);
    res->k = k;
    res->sigma.assign(s.begin(), s.begin() + k);
    res->resid.assign(k, 0.0);
    for (int i = 0; i < k; ++i) {
        double acc = 0.0;
        for (int r = 0; r < b; ++r) {
            double v = 0.0;
            for (int t = 0; t < b; ++t) v += Rprev[(size_t)r * b + t] * P[(size_t)((steps - 1) * b + t) * mdim + i];
            acc += v * v;
        }
        res->resid[i] = std::sqrt(acc);
    }
    std::vector<double> Wk((size_t)mdim * k);
    for (int i = 0; i < mdim; ++i)
        for (int jj = 0; jj < k; ++jj) Wk[(size_t)i * k + jj] = Wt[(size_t)i * mdim + jj];
    float* Cw = nullptr;
    if ((rc = upload_f32(c, "lz_w", Wk, Wk.size(), &Cw))) return rc;
    RTT_HIP(hipMalloc((void**)&res->V, sizeof(float) * (size_t)k * n));
    if ((rc = combine(Cw, mdim, k, Vall, n, res->V, n, n, 0.f, c.s))) return rc;
    RTT_HIP(hipStreamSynchronize(c.s));
    return RTT_OK;
}

}  // namespace

extern "C" int rsvd(const rtt_geometry* g, const rtt_svd_opts* o, const float* omega, rtt_svd** out, void* stream)
{
    if (out) *out = nullptr;
    if (!out || !o) return fail(RTT_EINVAL, "rsvd: NULL opts or out");
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (o->geometry < -1 || o->geometry >= (int)g->members.size()) return fail(RTT_EINVAL, "rsvd: bad member index");
    Ctx c;
    c.g = g;
    c.member = o->geometry;
    c.mask = o->order_mask;
    c.n_rows = c.member < 0 ? g->n_rows : g->members[c.member].n_rows;
    c.n_cols = c.member < 0 ? g->n_cols : g->members[c.member].n_cols;
    c.s = (hipStream_t)stream;
    std::unique_ptr<rtt_svd> res(new rtt_svd());
    res->member = c.member;
    res->n_rows = c.n_rows;
    res->n_cols = c.n_cols;
    int rc;
    if (o->method == RTT_SVD_RSVD) {
        if (o->k < 1 || o->p < 0 || o->q < 0 || o->q > 64) return fail(RTT_EINVAL, "rsvd: need k >= 1, p >= 0, 0 <= q <= 64");
        if (o->k + o->p > 512) return fail(RTT_EINVAL, "rsvd: k + p must be <= 512");
        if ((int64_t)(o->k + o->p) > std::min(c.n_rows, c.n_cols))
            return fail(RTT_EINVAL, "rsvd: k + p exceeds the matrix dimensions");
        rc = run_rsvd(c, *o, omega, res.get());
    } else if (o->method == RTT_SVD_BLOCK_LANCZOS) {
        if (o->block < 32 || o->steps < 1 || (int64_t)o->block * o->steps > 1024 || o->k < 1)
            return fail(RTT_EINVAL, "lanczos: need block >= 32 (multiple of 32), steps >= 1, block*steps <= 1024");
        if ((int64_t)o->block * o->steps > std::min(c.n_rows, c.n_cols))
            return fail(RTT_EINVAL, "lanczos: block*steps exceeds the matrix dimensions");
        rc = run_lanczos(c, *o, omega, res.get());
    } else {
        return fail(RTT_EINVAL, "rsvd: unknown method");
    }
    if (rc) return rc;
    *out = res.release();
    return RTT_OK;
}

extern "C" int svd_free(rtt_svd* s)
{
    if (!s) return RTT_OK;
    if (s->magic != 0x53564431u) return fail(RTT_ESTATE, "not an svd handle");
    s->magic = 0;
    delete s;
    return RTT_OK;
}

extern "C" int svd_get(const rtt_svd* s, int32_t* k_out, double* sigma_host, const float** V_dev,
                       const float** U_dev, double* resid_host)
{
    if (!s || s->magic != 0x53564431u) return fail(RTT_EINVAL, "invalid svd handle");
    if (k_out) *k_out = s->k;
    if (sigma_host) std::memcpy(sigma_host, s->sigma.data(), sizeof(double) * s->k);
    if (resid_host) std::memcpy(resid_host, s->resid.data(), sizeof(double) * s->k);
    if (V_dev) *V_dev = s->V;
    if (U_dev) *U_dev = s->U;
    return RTT_OK;
}

extern "C" int tsvd_solve(const rtt_geometry* g, const rtt_svd* sv, const float* y, int32_t nrhs, int32_t t,
                          double sigma_min, float* x, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (!sv || sv->magic != 0x53564431u) return fail(RTT_EINVAL, "invalid svd handle");
    if (nrhs < 0 || nrhs > 4096) return fail(RTT_EINVAL, "nrhs must be 0..4096");
    if (nrhs > 0 && (!y || !x)) return fail(RTT_EINVAL, "NULL data pointer");
    if (nrhs == 0) return RTT_OK;
    int tt = t;
    if (tt <= 0) {
        tt = 0;
        while (tt < sv->k && sv->sigma[tt] >= sigma_min && sv->sigma[tt] > 0.0) ++tt;
    }
    if (tt > sv->k) return fail(RTT_EINVAL, "tsvd_solve: t exceeds the number of singular triplets");
    Ctx c;
    c.g = g;
    c.member = sv->member;
    c.mask = 0;
    c.n_rows = sv->n_rows;
    c.n_cols = sv->n_cols;
    c.s = (hipStream_t)stream;
    const int64_t n = c.n_cols;
    if (tt == 0) {
        RTT_HIP(hipMemsetAsync(x, 0, sizeof(float) * (size_t)nrhs * n, c.s));
        return RTT_OK;
    }
    int rc;
    // g = A^T y (into x), c = V_t g, c_i /= sigma_i^2, x = V_t^T c
    if ((rc = apply_op(g, c.member, true, y, x, nrhs, 0, c.s))) return rc;
    double* Cd = (double*)c.ws.get("ts_c", sizeof(double) * (size_t)tt * nrhs);
    if (!Cd) return fail(RTT_ENOMEM, "tsvd workspace");
    if ((rc = gram(c.ws, sv->V, n, x, n, tt, nrhs, n, Cd, c.s))) return rc;
    std::vector<double> coef;
    if ((rc = download(c, Cd, coef, (size_t)tt * nrhs))) return rc;
    for (int i = 0; i < tt; ++i)
        for (int r = 0; r < nrhs; ++r) coef[(size_t)i * nrhs + r] /= sv->sigma[i] * sv->sigma[i];
    float* Cf = nullptr;
    if ((rc = upload_f32(c, "ts_cf", coef, coef.size(), &Cf))) return rc;
    if ((rc = combine(Cf, tt, nrhs, sv->V, n, x, n, n, 0.f, c.s))) return rc;
    RTT_HIP(hipStreamSynchronize(c.s));
    return RTT_OK;
}
