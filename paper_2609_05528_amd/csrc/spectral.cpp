// Spectral drivers (Sec. 3.6 eq. (19), Sec. 4.4 eq. (31)) and the TSVD estimator (Sec. 9).
//
// rsvd, RTT_SVD_RSVD: randomized subspace iteration (Halko, Martinsson &
// Tropp, SIAM Rev. 2011, Alg. 4.4) with l = k + p test vectors and q power
// iterations, followed by their Alg. 5.1: B^T = A^T Q, B^T = Qb R, SVD of
// R^T = Ur S W^T, so B = Ur S (Qb W)^T.  Every block is orthonormalised by
// Cholesky QR: the Gram matrix comes from the FP32 MFMA kernel with FP64
// slice reduction, the Cholesky factor and its inverse are FP64 (device, one
// workgroup per factor), the triangular apply is the MFMA combine kernel.  Two passes (CholQR2) for the
// final bases Q and Qb; one for the intermediate bases of the power iterations,
// which only carry a span.  When the first Gram matrix is too ill-conditioned
// for FP32 a diagonal shift is added in the first pass and one more pass
// follows (shifted CholQR3, Fukaya et al. 2020).  Columns that are numerically
// dependent are dropped (zeroed).
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
    int member = -1;      // -1 whole operator, g >= 0 one member, RTT_EACH_GEOMETRY every member
    int sets = 1;         // independent factorisations held (G for RTT_EACH_GEOMETRY)
    int64_t n_rows = 0, n_cols = 0;
    std::vector<double> sigma, resid;   // [sets][k]
    bool has_resid = false;             // resid holds residuals (Lanczos; rSVD with keep_u)
    float* V = nullptr;
    float* U = nullptr;
    double* d_sigma = nullptr;          // device copy of sigma
    rtt::Workspace* ws = nullptr;       // grow-only scratch of tsvd_solve
    ~rtt_svd()
    {
        if (V) hipFree(V);
        if (U) hipFree(U);
        if (d_sigma) hipFree(d_sigma);
        delete ws;
    }
};

namespace {

// A block of rows (or columns) processed as one independent problem: [off, off + len) of
// vectors whose stride is the full length.
struct Seg {
    int64_t off, len;
};

struct Ctx {
    const rtt_geometry* g;
    int member;
    uint32_t mask;
    int64_t n_rows, n_cols;          // vector lengths (strides)
    std::vector<Seg> rseg, cseg;     // one problem: {0, n}; every member: the member blocks
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

// Orthonormalise, independently on every segment, the l (padded to lp) vectors stored in *Y
// (row stride n), using *T as ping-pong storage; on return *Y holds Q.  Every step is queued on the
// stream (no host synchronisation): the Gram matrices (MFMA, FP64 slice reduction), their FP64
// Cholesky factors and inverses (cholqr.hip), the MFMA combines Q = Y R^-1.  final_basis: two
// passes (CholQR2); otherwise one, as the basis only carries a span to the next product (the
// intermediate steps of subspace iteration).  A first pass whose Gram matrix had to be shifted adds
// one more pass on that segment, decided on the device: the extra pass is always queued and its
// kernels do nothing on segments that do not need it.  R_out (optional): receives a device pointer
// to the accumulated factors R_total (lp x lp, upper, one per segment) with Y = Q R_total on the
// retained columns; it stays valid until the next orth call on the same context.
int orth(Ctx& c, float** Y, float** T, int lp, int64_t n, const std::vector<Seg>& segs, bool final_basis,
         double** R_out = nullptr)
{
    const int base = final_basis ? 2 : 1;
    const int ns = (int)segs.size();
    const size_t lp2 = (size_t)lp * lp;
    double* Gd = (double*)c.ws.get("orth_gram", sizeof(double) * lp2 * ns);
    double* S = (double*)c.ws.get("orth_s", sizeof(double) * lp2 * ns);
    double* R = (double*)c.ws.get("orth_r", sizeof(double) * lp2 * ns);
    double* Ri = (double*)c.ws.get("orth_ri", sizeof(double) * lp2 * ns);
    float* Ri32 = (float*)c.ws.get("orth_ri32", sizeof(float) * lp2 * ns);
    int* dead = (int*)c.ws.get("orth_dead", sizeof(int) * (size_t)lp * ns);
    int* st = (int*)c.ws.get("orth_state", sizeof(int) * (size_t)ns);
    double* rt[2] = {nullptr, nullptr};
    if (R_out) {
        rt[0] = (double*)c.ws.get("orth_rt0", sizeof(double) * lp2 * ns);
        rt[1] = (double*)c.ws.get("orth_rt1", sizeof(double) * lp2 * ns);
    }
    if (!Gd || !S || !R || !Ri || !Ri32 || !dead || !st || (R_out && (!rt[0] || !rt[1])))
        return fail(RTT_ENOMEM, "orth workspace");
    int rc, cur = 0;
    if (R_out && (rc = identity_f64(rt[0], lp, ns, c.s))) return rc;
    auto pass = [&](int mode, double dead_tol) -> int {
        for (int q = 0; q < ns; ++q) {
            const Seg sg = segs[q];
            if ((rc = gram(c.ws, *Y + sg.off, n, *Y + sg.off, n, lp, lp, sg.len, Gd + q * lp2, c.s,
                           mode == 2 ? st + q : nullptr)))
                return rc;
        }
        if ((rc = chol_factor(Gd, lp, ns, mode, dead_tol, S, R, dead, st, c.s))) return rc;
        if ((rc = chol_inverse(R, dead, st, lp, ns, mode, Ri, Ri32, c.s))) return rc;
        if (R_out) {
            if ((rc = upper_product(R, rt[cur], st, lp, ns, mode, rt[1 - cur], c.s))) return rc;
            cur = 1 - cur;
        }
        for (int q = 0; q < ns; ++q) {
            const Seg sg = segs[q];
            if ((rc = combine(Ri32 + q * lp2, lp, lp, *Y + sg.off, n, *T + sg.off, n, sg.len, 0.f, c.s, true,
                              mode == 2 ? st + q : nullptr)))
                return rc;
        }
        if (mode != 2) {
            std::swap(*Y, *T);
            return RTT_OK;
        }
        // the conditional pass wrote its segments to *T: copy them back so that *Y holds every Q
        for (int q = 0; q < ns; ++q) {
            const Seg sg = segs[q];
            if ((rc = copy_rows_if(st + q, *T + sg.off, *Y + sg.off, n, lp, sg.len, c.s))) return rc;
        }
        return RTT_OK;
    };
    // dependent-pivot thresholds: 1e-12 of the largest diagonal in the first pass, 1e-8 after
    for (int p = 0; p < base; ++p)
        if ((rc = pass(p == 0 ? 0 : 1, p == 0 ? 1e-12 : 1e-8))) return rc;
    if ((rc = pass(2, 1e-8))) return rc;
    if (R_out) *R_out = rt[cur];
    return RTT_OK;
}

// orth, then the accumulated factor of the single segment on the host (lp x lp, row-major)
int orth_r(Ctx& c, float** Y, float** T, int lp, int64_t n, const std::vector<Seg>& segs, std::vector<double>& Rh)
{
    double* Rd = nullptr;
    int rc;
    if ((rc = orth(c, Y, T, lp, n, segs, true, &Rd))) return rc;
    return download(c, Rd, Rh, (size_t)lp * lp * segs.size());
}

float* dev_alloc(Ctx& c, const char* name, size_t n)
{
    return (float*)c.ws.get(name, n * sizeof(float));
}

int apply(Ctx& c, bool adjoint, const float* in, float* out, int nvec)
{
    return apply_op(c.g, c.member >= 0 ? c.member : -1, adjoint, in, out, nvec, c.mask, c.s);
}

int run_rsvd(Ctx& c, const rtt_svd_opts& o, const float* omega, rtt_svd* res)
{
    const int l = o.k + o.p, lp = pad32(l);
    const int64_t n = c.n_cols, m = c.n_rows;
    const int sets = (int)c.cseg.size();
    float* X = dev_alloc(c, "rs_x", (size_t)lp * n);
    float* X2 = dev_alloc(c, "rs_x2", (size_t)lp * n);
    float* Y = dev_alloc(c, "rs_y", (size_t)lp * m);
    float* Y2 = dev_alloc(c, "rs_y2", (size_t)lp * m);
    if (!X || !X2 || !Y || !Y2) return fail(RTT_ENOMEM, "rsvd block buffers");
    int rc;
    // Rows l .. lp of X and Y are padding that the Gram and combine kernels read: zero them.  Rows
    // below l are written by the test block and the products before they are read (all of a row of
    // X; of a row of Y only the entries of the selected orders, so with an order mask Y is zeroed
    // whole), and X2 / Y2 are written in full by the combine kernel before they are read.
    if (lp > l && (rc = fill(X + (size_t)l * n, (int64_t)(lp - l) * n, 0.f, c.s))) return rc;
    const int y_from = c.mask != 0 ? 0 : l;
    if (lp > y_from && (rc = fill(Y + (size_t)y_from * m, (int64_t)(lp - y_from) * m, 0.f, c.s))) return rc;
    if (omega) RTT_HIP(hipMemcpyAsync(X, omega, sizeof(float) * l * n, hipMemcpyDeviceToDevice, c.s));
    else if ((rc = normal_fill(X, (int64_t)l * n, o.seed, c.s))) return rc;
    // Y = A Omega; Q = orth(Y)
    if ((rc = apply(c, false, X, Y, l))) return rc;
    // the last basis of the range (Q) is final: U = Q Ur and B^T = A^T Q need it orthonormal
    if ((rc = orth(c, &Y, &Y2, lp, m, c.rseg, o.q == 0))) return rc;
    for (int it = 0; it < o.q; ++it) {
        if ((rc = apply(c, true, Y, X, l))) return rc;
        if ((rc = orth(c, &X, &X2, lp, n, c.cseg, false))) return rc;
        if ((rc = apply(c, false, X, Y, l))) return rc;
        if ((rc = orth(c, &Y, &Y2, lp, m, c.rseg, it == o.q - 1))) return rc;
    }
    // B^T = A^T Q = Qb R; R of every set comes to the host for the small SVDs (the one download)
    if ((rc = apply(c, true, Y, X, l))) return rc;
    std::vector<double> Rh;
    if ((rc = orth_r(c, &X, &X2, lp, n, c.cseg, Rh))) return rc;
    const size_t lp2 = (size_t)lp * lp;
    const int k = o.k;
    res->k = k;
    res->sets = sets;
    res->sigma.assign((size_t)sets * k, 0.0);
    res->resid.assign((size_t)sets * k, 0.0);
    RTT_HIP(hipMalloc((void**)&res->V, sizeof(float) * (size_t)k * n));
    if (o.keep_u) RTT_HIP(hipMalloc((void**)&res->U, sizeof(float) * (size_t)k * m));
    // SVD of R^T (l x l leading block) of every set, the sets on host threads
    std::vector<std::vector<double>> Urs(sets), svs(sets), Ws(sets);
    host_for(sets, [&](int q) {
        std::vector<double> Mt((size_t)l * l);
        for (int i = 0; i < l; ++i)
            for (int j = 0; j < l; ++j) Mt[(size_t)i * l + j] = Rh[q * lp2 + (size_t)j * lp + i];
        jacobi_svd(Mt, l, Urs[q], svs[q], Ws[q]);
    });
    for (int q = 0; q < sets; ++q) {
        const std::vector<double>&Ur = Urs[q], &sv = svs[q], &W = Ws[q];
        std::copy(sv.begin(), sv.begin() + k, res->sigma.begin() + (size_t)q * k);
        // V = Qb W[:, :k] ; U = Q Ur[:, :k]
        std::vector<double> Wk((size_t)l * k), Uk((size_t)l * k);
        for (int i = 0; i < l; ++i)
            for (int j = 0; j < k; ++j) {
                Wk[(size_t)i * k + j] = W[(size_t)i * l + j];
                Uk[(size_t)i * k + j] = Ur[(size_t)i * l + j];
            }
        float* Cw = nullptr;
        if ((rc = upload_f32(c, "rs_w", Wk, Wk.size(), &Cw))) return rc;
        const Seg cs = c.cseg[q], rs = c.rseg[q];
        if ((rc = combine(Cw, l, k, X + cs.off, n, res->V + cs.off, n, cs.len, 0.f, c.s))) return rc;
        if (o.keep_u) {
            float* Cu = nullptr;
            if ((rc = upload_f32(c, "rs_u", Uk, Uk.size(), &Cu))) return rc;
            if ((rc = combine(Cu, l, k, Y + rs.off, m, res->U + rs.off, m, rs.len, 0.f, c.s))) return rc;
        }
    }
    if (o.keep_u) {
        // residuals || A v_i - sigma_i u_i || per set
        float* AV = Y2;
        if ((rc = apply(c, false, res->V, AV, k))) return rc;
        const size_t nd = (size_t)k * sets;
        double* d = (double*)c.ws.get("rs_dots", sizeof(double) * 3 * nd);
        int64_t* segd = (int64_t*)c.ws.get("rs_seg", sizeof(int64_t) * 2 * sets);
        if (!d || !segd) return fail(RTT_ENOMEM, "dots");
        std::vector<int64_t> hs;
        int64_t maxlen = 0;
        for (const Seg& sg : c.rseg) {
            hs.insert(hs.end(), {sg.off, sg.len});
            maxlen = std::max(maxlen, sg.len);
        }
        RTT_HIP(hipMemcpyAsync(segd, hs.data(), hs.size() * sizeof(int64_t), hipMemcpyHostToDevice, c.s));
        if ((rc = dots_seg(c.ws, AV, m, AV, m, segd, sets, maxlen, k, d, c.s))) return rc;
        if ((rc = dots_seg(c.ws, AV, m, res->U, m, segd, sets, maxlen, k, d + nd, c.s))) return rc;
        if ((rc = dots_seg(c.ws, res->U, m, res->U, m, segd, sets, maxlen, k, d + 2 * nd, c.s))) return rc;
        std::vector<double> h;
        if ((rc = download(c, d, h, 3 * nd))) return rc;
        // dots_seg output index: vector i, set q -> i * sets + q
        for (int q = 0; q < sets; ++q)
            for (int i = 0; i < k; ++i) {
                const size_t e = (size_t)i * sets + q;
                const double si = res->sigma[(size_t)q * k + i];
                res->resid[(size_t)q * k + i] =
                    std::sqrt(std::max(0.0, h[e] - 2 * si * h[nd + e] + si * si * h[2 * nd + e]));
            }
        res->has_resid = true;
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
    const std::vector<Seg> cwhole{{0, n}}, rwhole{{0, m}};
    if ((rc = orth_r(c, &Z, &Z2, b, n, cwhole, R))) return rc;
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
        if ((rc = orth_r(c, &W, &W2, b, m, rwhole, L))) return rc;   // W now holds U_j
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
        if ((rc = orth_r(c, &Z, &Z2, b, n, cwhole, R))) return rc;   // Z = V_{j+1}, R_j
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
    res->has_resid = true;
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
    if (o->geometry < RTT_EACH_GEOMETRY || o->geometry >= (int)g->members.size())
        return fail(RTT_EINVAL, "rsvd: bad member index");
    Ctx c;
    c.g = g;
    c.member = o->geometry;
    c.mask = o->order_mask;
    c.n_rows = c.member < 0 ? g->n_rows : g->members[c.member].n_rows;
    c.n_cols = c.member < 0 ? g->n_cols : g->members[c.member].n_cols;
    if (c.member == RTT_EACH_GEOMETRY) {
        for (const Member& m : g->members) {
            c.rseg.push_back({m.row_offset, m.n_rows});
            c.cseg.push_back({m.col_offset, m.n_cols});
        }
    } else {
        c.rseg.push_back({0, c.n_rows});
        c.cseg.push_back({0, c.n_cols});
    }
    int64_t min_dim = INT64_MAX;
    for (size_t q = 0; q < c.rseg.size(); ++q) min_dim = std::min({min_dim, c.rseg[q].len, c.cseg[q].len});
    c.s = (hipStream_t)stream;
    std::unique_ptr<rtt_svd> res(new rtt_svd());
    res->member = c.member;
    res->n_rows = c.n_rows;
    res->n_cols = c.n_cols;
    int rc;
    if (o->method == RTT_SVD_RSVD) {
        if (o->k < 1 || o->p < 0 || o->q < 0 || o->q > 64) return fail(RTT_EINVAL, "rsvd: need k >= 1, p >= 0, 0 <= q <= 64");
        if (o->k + o->p > 512) return fail(RTT_EINVAL, "rsvd: k + p must be <= 512");
        if ((int64_t)(o->k + o->p) > min_dim)
            return fail(RTT_EINVAL, "rsvd: k + p exceeds the matrix dimensions");
        rc = run_rsvd(c, *o, omega, res.get());
    } else if (o->method == RTT_SVD_BLOCK_LANCZOS) {
        if (c.member == RTT_EACH_GEOMETRY) return fail(RTT_EINVAL, "lanczos: one geometry (or the whole operator) per call");
        if (o->block < 32 || o->steps < 1 || (int64_t)o->block * o->steps > 1024 || o->k < 1)
            return fail(RTT_EINVAL, "lanczos: need block >= 32 (multiple of 32), steps >= 1, block*steps <= 1024");
        if ((int64_t)o->block * o->steps > std::min(c.n_rows, c.n_cols))
            return fail(RTT_EINVAL, "lanczos: block*steps exceeds the matrix dimensions");
        rc = run_lanczos(c, *o, omega, res.get());
    } else {
        return fail(RTT_EINVAL, "rsvd: unknown method");
    }
    if (rc) return rc;
    RTT_HIP(hipMalloc((void**)&res->d_sigma, sizeof(double) * res->sigma.size()));
    RTT_HIP(hipMemcpy(res->d_sigma, res->sigma.data(), sizeof(double) * res->sigma.size(), hipMemcpyHostToDevice));
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
    if (sigma_host) std::memcpy(sigma_host, s->sigma.data(), sizeof(double) * s->sigma.size());
    if (resid_host) std::memcpy(resid_host, s->resid.data(), sizeof(double) * s->resid.size());
    if (V_dev) *V_dev = s->V;
    if (U_dev) *U_dev = s->U;
    return RTT_OK;
}

extern "C" int svd_converged(const rtt_svd* s, double rel_tol, int32_t* count)
{
    if (!s || s->magic != 0x53564431u) return fail(RTT_EINVAL, "invalid svd handle");
    if (!count) return fail(RTT_EINVAL, "svd_converged: NULL count");
    if (!(rel_tol >= 0.0)) return fail(RTT_EINVAL, "svd_converged: rel_tol must be >= 0");
    if (!s->has_resid) return fail(RTT_ESTATE, "svd_converged: these factors carry no residuals (rSVD without keep_u)");
    for (int q = 0; q < s->sets; ++q) {
        const double* sg = s->sigma.data() + (size_t)q * s->k;
        const double* rs = s->resid.data() + (size_t)q * s->k;
        const double thr = rel_tol * (s->k > 0 ? sg[0] : 0.0);
        int32_t n = 0;
        for (int i = 0; i < s->k; ++i) n += rs[i] <= thr ? 1 : 0;
        count[q] = n;
    }
    return RTT_OK;
}

// x = V_t diag(sigma_t^-2) V_t^T b with b = A^T y (from_data) or b = y (a coefficient block)
static int tsvd_apply(const rtt_geometry* g, const rtt_svd* sv, const float* y, int32_t nrhs, int32_t t,
                      double sigma_min, float* x, void* stream, bool from_data)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (!sv || sv->magic != 0x53564431u) return fail(RTT_EINVAL, "invalid svd handle");
    if (nrhs < 0 || nrhs > 4096) return fail(RTT_EINVAL, "nrhs must be 0..4096");
    if (nrhs > 0 && (!y || !x)) return fail(RTT_EINVAL, "NULL data pointer");
    if (sv->member >= (int)g->members.size() || (sv->member == RTT_EACH_GEOMETRY && sv->sets != (int)g->members.size()) ||
        sv->n_cols != (sv->member >= 0 ? g->members[sv->member].n_cols : g->n_cols))
        return fail(RTT_EINVAL, "tsvd: the factors belong to another geometry");
    if (t > sv->k) return fail(RTT_EINVAL, "tsvd: t exceeds the number of singular triplets");
    if (nrhs == 0) return RTT_OK;
    // kept components: i < t (t > 0), or sigma_i >= sigma_min (t <= 0); zero singular values never
    int tt = t;
    double smin = t > 0 ? 0.0 : sigma_min;
    if (t <= 0) {
        tt = 0;
        for (int q = 0; q < sv->sets; ++q) {
            int c = 0;
            while (c < sv->k && sv->sigma[(size_t)q * sv->k + c] >= sigma_min && sv->sigma[(size_t)q * sv->k + c] > 0.0)
                ++c;
            tt = std::max(tt, c);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = sv->n_cols;
    int rc;
    if (tt == 0) return fill(x, (int64_t)nrhs * n, 0.f, s);
    if (!sv->ws) const_cast<rtt_svd*>(sv)->ws = new (std::nothrow) Workspace();
    if (!sv->ws) return fail(RTT_ENOMEM, "tsvd workspace");
    Workspace& ws = *sv->ws;
    const int sets = sv->sets;
    double* Cd = (double*)ws.get("ts_c", sizeof(double) * (size_t)sets * tt * nrhs);
    float* Cf = (float*)ws.get("ts_cf", sizeof(float) * (size_t)sets * tt * nrhs);
    if (!Cd || !Cf) return fail(RTT_ENOMEM, "tsvd workspace");
    // b = A^T y (or the given block), then per set c = V_t b (coefficients), c_i /= sigma_i^2, x = V_t^T c
    const float* b = y;
    if (from_data) {
        if ((rc = apply_op(g, sv->member >= 0 ? sv->member : -1, true, y, x, nrhs, 0, s))) return rc;
        b = x;
    }
    for (int q = 0; q < sets; ++q) {
        const int64_t off = sets > 1 ? g->members[q].col_offset : 0;
        const int64_t len = sets > 1 ? g->members[q].n_cols : n;
        if ((rc = gram(ws, sv->V + off, n, b + off, n, tt, nrhs, len, Cd + (size_t)q * tt * nrhs, s))) return rc;
    }
    if ((rc = scale_inv_sq(Cd, sv->d_sigma, sets, tt, sv->k, nrhs, smin, Cf, s))) return rc;
    for (int q = 0; q < sets; ++q) {
        const int64_t off = sets > 1 ? g->members[q].col_offset : 0;
        const int64_t len = sets > 1 ? g->members[q].n_cols : n;
        if ((rc = combine(Cf + (size_t)q * tt * nrhs, tt, nrhs, sv->V + off, n, x + off, n, len, 0.f, s))) return rc;
    }
    return RTT_OK;
}

extern "C" int tsvd_solve(const rtt_geometry* g, const rtt_svd* sv, const float* y, int32_t nrhs, int32_t t,
                          double sigma_min, float* x, void* stream)
{
    return tsvd_apply(g, sv, y, nrhs, t, sigma_min, x, stream, true);
}

extern "C" int tsvd_project(const rtt_geometry* g, const rtt_svd* sv, const float* b, int32_t nrhs, int32_t t,
                            double sigma_min, float* x, void* stream)
{
    if (b && b == x) return fail(RTT_EINVAL, "tsvd_project: b and x must not overlap");
    return tsvd_apply(g, sv, b, nrhs, t, sigma_min, x, stream, false);
}
