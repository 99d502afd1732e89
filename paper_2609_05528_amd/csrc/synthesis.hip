// Representation synthesis Q_d of Sec. 3.2 eq. (5)-(8) and Sec. 7 on one geometry's coefficient
// nodes, and the rank audit of A^(d) = A Q_d (eq. (7)).
//
// Column (a, b, c) of Q (radial slowest, temporal fastest) holds R_a(r_i) Phi_b(phi_j) T_c(s_k) at
// node (cell centre (r_i, phi_j), hat centre s_k): R_a clamped cubic B-splines on uniform knots in
// log r over [r_in, r_out], Phi_b = 1, cos m phi, sin m phi (m <= m_max), T_c global DCT-II modes
// or degree-one B-splines (compact temporal functions) on a source-time window.  The three factor
// tables are built on the host in FP64; a kernel expands the rows of Q (d rows of n_cols) once, and
// the synthesis / its transpose are the MFMA combine / Gram kernels over those rows.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rtt.h"
#include "rtt_internal.h"
#include "dense.h"

namespace rtt {
namespace {
constexpr uint32_t SYN_MAGIC = 0x53594E51u;
}
}  // namespace rtt

struct rtt_synthesis {
    int32_t member = 0;
    int32_t n_radial = 0, m_max = 0, n_temporal = 0, temporal = 0;
    int32_t d = 0, n_az = 0;
    double t_lo = 0.0, t_hi = 0.0;
    int64_t n_cols = 0;       // the member's coefficient length
    float* d_Q = nullptr;     // [d][n_cols]: row (a, b, c) = column (a, b, c) of Q
    // FP32 factor tables of the separable path: R [n_radial][n_r], P [n_az][n_phi], T [n_temporal][K]
    float *d_R = nullptr, *d_P = nullptr, *d_T = nullptr;
    int32_t n_r = 0, n_phi = 0, K = 0;
    bool separable = false;   // the factor-by-factor kernels fit their LDS limits
    int device = 0;
    mutable rtt::Workspace ws;
    uint32_t magic = rtt::SYN_MAGIC;
};

namespace rtt {
namespace {

// Q rows from the factor tables R [n_radial][n_r], P [n_az][n_phi], T [n_t][K] (FP64)
__global__ void k_synth_rows(const double* __restrict__ R, const double* __restrict__ P, const double* __restrict__ T,
                             int n_r, int n_phi, int K, int n_az, int n_t, int64_t n_cols, float* __restrict__ Q)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n_cols) return;
    const int row = blockIdx.y;                   // (a * n_az + b) * n_t + c
    const int c = row % n_t, b = (row / n_t) % n_az, a = row / (n_t * n_az);
    const int k = (int)(col % K);
    const int64_t cell = col / K;
    const int j = (int)(cell % n_phi), i = (int)(cell / n_phi);
    Q[(int64_t)row * n_cols + col] = (float)(R[(int64_t)a * n_r + i] * P[(int64_t)b * n_phi + j] * T[(int64_t)c * K + k]);
}

// c[v][a] = (float) G[a][v]  (FP64 Gram [d][nvec] to coefficient rows)
__global__ void k_gram_to_rows(const double* __restrict__ G, int d, int nvec, float* __restrict__ c)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d * nvec) return;
    const int v = (int)(t / d), a = (int)(t % d);
    c[t] = (float)G[(int64_t)a * nvec + v];
}

// Ct[a][v] = c[v][a]
__global__ void k_transpose_f32(const float* __restrict__ c, int nvec, int d, float* __restrict__ Ct)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d * nvec) return;
    const int a = (int)(t / nvec), v = (int)(t % nvec);
    Ct[t] = c[(int64_t)v * d + a];
}

// FP64 Gram of d rows of length L (row stride ld): G[u][v] = sum_l Y[u][l] Y[v][l], FP32 inputs
// widened to FP64 before the products; 16 x 16 output tiles, rows staged through LDS in chunks.
// blockIdx.z = set * nsl + slice: independent row sets (d rows each, consecutive), each split into
// nsl slices of the row length with one partial d x d output per (set, slice), summed afterwards
// in slice order.
constexpr int GT = 16, GL = 64;
__global__ __launch_bounds__(GT * GT) void k_gram_f64(const float* __restrict__ Y, int64_t ld, int d, int64_t L,
                                                     int nsl, double* __restrict__ G)
{
    __shared__ double su[GT][GL + 1], sv[GT][GL + 1];
    const int set = blockIdx.z / nsl, sl = blockIdx.z % nsl;
    Y += (int64_t)set * d * ld;
    G += (int64_t)blockIdx.z * d * d;
    const int64_t span = ((L + nsl - 1) / nsl + GL - 1) / GL * GL;
    const int64_t lb = (int64_t)sl * span, le = min(L, lb + span);
    const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;
    const int u0 = blockIdx.y * GT, v0 = blockIdx.x * GT;
    if (v0 + GT <= u0) return;   // lower tiles: mirrored from the upper ones on the host
    double acc = 0.0;
    for (int64_t l0 = lb; l0 < le; l0 += GL) {
        for (int e = threadIdx.x; e < GT * GL; e += GT * GT) {
            const int r = e / GL, q = e % GL;
            const int64_t l = l0 + q;
            su[r][q] = (u0 + r < d && l < le) ? (double)Y[(int64_t)(u0 + r) * ld + l] : 0.0;
            sv[r][q] = (v0 + r < d && l < le) ? (double)Y[(int64_t)(v0 + r) * ld + l] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int q = 0; q < GL; ++q) acc += su[ty][q] * sv[tx][q];
        __syncthreads();
    }
    if (u0 + ty < d && v0 + tx < d) G[(int64_t)(u0 + ty) * d + v0 + tx] = acc;
}

// Separable synthesis x = Q c, one block per (radial node i, vector v): W[a][b][k] = sum_c T[c][k]
// c[a][b][c], V[b][k] = sum_a R[a][i] W[a][b][k], x[i][j][k] = sum_b P[b][j] V[b][k] (fixed order).
constexpr int SYN_LDS = 16384;   // floats of dynamic LDS the separable kernels may use (64 KiB)
__global__ __launch_bounds__(256) void k_synth_expand(const float* __restrict__ R, const float* __restrict__ P,
                                                      const float* __restrict__ T, int nR, int nA, int nT, int n_r,
                                                      int n_phi, int K, const float* __restrict__ c, float* __restrict__ x,
                                                      int64_t n_cols)
{
    extern __shared__ float lds[];
    const int d = nR * nA * nT;
    float* cs = lds;                  // d
    float* W = cs + d;                // nR * nA * K
    float* V = W + nR * nA * K;       // nA * K
    const int i = blockIdx.x;
    const int64_t v = blockIdx.y;
    for (int q = threadIdx.x; q < d; q += blockDim.x) cs[q] = c[v * d + q];
    __syncthreads();
    for (int e = threadIdx.x; e < nR * nA * K; e += blockDim.x) {
        const int k = e % K, ab = e / K;
        float acc = 0.f;
        for (int q = 0; q < nT; ++q) acc += T[q * K + k] * cs[ab * nT + q];
        W[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nA * K; e += blockDim.x) {
        const int k = e % K, b = e / K;
        float acc = 0.f;
        for (int a = 0; a < nR; ++a) acc += R[a * n_r + i] * W[(a * nA + b) * K + k];
        V[e] = acc;
    }
    __syncthreads();
    float* xr = x + v * n_cols + (int64_t)i * n_phi * K;
    for (int e = threadIdx.x; e < n_phi * K; e += blockDim.x) {
        const int k = e % K, j = e / K;
        float acc = 0.f;
        for (int b = 0; b < nA; ++b) acc += P[b * n_phi + j] * V[b * K + k];
        xr[e] = acc;
    }
}

// Separable transpose, one block per (radial node i, vector v): U[j][c] = sum_k T[c][k] x[i][j][k],
// Z[b][c] = sum_j P[b][j] U[j][c], part[v][i][a][b][c] = R[a][i] Z[b][c]; then the radial sum.
__global__ __launch_bounds__(256) void k_synth_project_part(const float* __restrict__ R, const float* __restrict__ P,
                                                            const float* __restrict__ T, int nR, int nA, int nT,
                                                            int n_r, int n_phi, int K, const float* __restrict__ x,
                                                            int64_t n_cols, float* __restrict__ part)
{
    extern __shared__ float lds[];
    float* xs = lds;                  // n_phi * K
    float* U = xs + n_phi * K;        // n_phi * nT
    float* Z = U + n_phi * nT;        // nA * nT
    const int i = blockIdx.x;
    const int64_t v = blockIdx.y;
    const float* xr = x + v * n_cols + (int64_t)i * n_phi * K;
    for (int e = threadIdx.x; e < n_phi * K; e += blockDim.x) xs[e] = xr[e];
    __syncthreads();
    for (int e = threadIdx.x; e < n_phi * nT; e += blockDim.x) {
        const int q = e % nT, j = e / nT;
        float acc = 0.f;
        for (int k = 0; k < K; ++k) acc += T[q * K + k] * xs[j * K + k];
        U[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nA * nT; e += blockDim.x) {
        const int q = e % nT, b = e / nT;
        float acc = 0.f;
        for (int j = 0; j < n_phi; ++j) acc += P[b * n_phi + j] * U[j * nT + q];
        Z[e] = acc;
    }
    __syncthreads();
    const int d = nR * nA * nT;
    float* pr = part + (v * n_r + i) * d;
    for (int e = threadIdx.x; e < d; e += blockDim.x) {
        const int bq = e % (nA * nT), a = e / (nA * nT);
        pr[e] = R[a * n_r + i] * Z[bq];
    }
}

// c[v][q] = sum over radial nodes i (ascending) of part[v][i][q], in FP64
__global__ void k_synth_project_sum(const float* __restrict__ part, int n_r, int d, int nvec, float* __restrict__ c)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)d * nvec) return;
    const int64_t v = t / d;
    const int q = (int)(t % d);
    double acc = 0.0;
    for (int i = 0; i < n_r; ++i) acc += (double)part[(v * n_r + i) * d + q];
    c[t] = (float)acc;
}

// Localised probes of eq. (14) on one geometry's nodes: row (age v, direction l = a n_az + b) holds
// R[a][i] P[b][j] exp(-(s_k + age_v)^2 / (2 h^2)) / N_l
__global__ void k_local_probe(const float* __restrict__ R, const float* __restrict__ P, const double* __restrict__ inv_n,
                              const double* __restrict__ ages, int nR, int nA, int n_r, int n_phi, int K, double s0,
                              double dt_src, double h, int64_t n_cols, float* __restrict__ X)
{
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n_cols) return;
    const int L = nR * nA;
    const int row = blockIdx.y;                 // v * L + l
    const int v = row / L, l = row % L, a = l / nA, b = l % nA;
    const int k = (int)(col % K);
    const int64_t cell = col / K;
    const int j = (int)(cell % n_phi), i = (int)(cell / n_phi);
    const double t = s0 + dt_src * k + ages[v];
    X[(int64_t)row * n_cols + col] =
        (float)((double)R[a * n_r + i] * (double)P[b * n_phi + j] * exp(-t * t / (2.0 * h * h)) * inv_n[l]);
}

bool valid_syn(const rtt_synthesis* s) { return s && s->magic == SYN_MAGIC; }

// row-length slices for the FP64 Gram: enough blocks to fill the chip, slices of >= 16384 rows
int gram_slices(int d, int64_t L, int sets)
{
    const int tiles = (d + GT - 1) / GT;
    const int64_t blocks = (int64_t)tiles * (tiles + 1) / 2 * sets;
    int64_t nsl = std::max<int64_t>(1, 4096 / std::max<int64_t>(blocks, 1));
    nsl = std::min<int64_t>(nsl, std::max<int64_t>(1, L / 16384));
    nsl = std::min<int64_t>(nsl, 65535 / std::max(sets, 1));
    return (int)std::max<int64_t>(1, nsl);
}

// clamped cubic B-splines with n functions on uniform knots of [0, 1], at u in [0, 1] (Cox-de Boor)
void cubic_bsplines(double u, int n, double* out)
{
    std::vector<double> t;
    for (int i = 0; i < 4; ++i) t.push_back(0.0);
    for (int j = 1; j <= n - 4; ++j) t.push_back((double)j / (n - 3));
    for (int i = 0; i < 4; ++i) t.push_back(1.0);
    const int m = (int)t.size();
    std::vector<double> N(m - 1, 0.0);
    // degree 0: the half-open span holding u (the last non-empty span for u = 1)
    int span = -1;
    for (int i = 0; i < m - 1; ++i)
        if (t[i] < t[i + 1] && u >= t[i] && (u < t[i + 1] || (u == 1.0 && t[i + 1] == 1.0))) span = i;
    if (span >= 0) N[span] = 1.0;
    for (int p = 1; p <= 3; ++p)
        for (int i = 0; i + p + 1 < m; ++i) {
            double v = 0.0;
            if (t[i + p] > t[i]) v += (u - t[i]) / (t[i + p] - t[i]) * N[i];
            if (t[i + p + 1] > t[i + 1]) v += (t[i + p + 1] - u) / (t[i + p + 1] - t[i + 1]) * N[i + 1];
            N[i] = v;
        }
    for (int a = 0; a < n; ++a) out[a] = N[a];
}

int check_syn(const rtt_synthesis* s, int nvec)
{
    if (!valid_syn(s)) return fail(RTT_EINVAL, "invalid synthesis handle");
    if (nvec < 0 || nvec > 65535) return fail(RTT_EINVAL, "nvec must be 0..65535");
    return RTT_OK;
}

}  // namespace
}  // namespace rtt

using namespace rtt;

extern "C" int synthesis_create(const rtt_geometry* g, int32_t gi, const rtt_synthesis_spec* spec, rtt_synthesis** out)
{
    if (!out) return fail(RTT_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (gi < 0 || gi >= (int)g->members.size()) return fail(RTT_EINVAL, "geometry index out of range");
    if (!spec) return fail(RTT_EINVAL, "NULL spec");
    const Member& m = g->members[gi];
    const int nR = spec->n_radial, mmax = spec->m_max, nT = spec->n_temporal;
    if (nR < 4 || nR > 64 || mmax < 0 || mmax > 32 || nT < 1 || nT > 256)
        return fail(RTT_EINVAL, "need 4 <= n_radial <= 64, 0 <= m_max <= 32, 1 <= n_temporal <= 256");
    if (spec->temporal != RTT_SYNTH_DCT && spec->temporal != RTT_SYNTH_HATS)
        return fail(RTT_EINVAL, "unknown temporal family");
    if (spec->temporal == RTT_SYNTH_HATS && nT < 2) return fail(RTT_EINVAL, "compact temporal functions need n_temporal >= 2");
    const int nA = 2 * mmax + 1;
    const int64_t d = (int64_t)nR * nA * nT;
    if (d > 4096) return fail(RTT_EINVAL, "at most 4096 synthesis columns");
    const rtt_grid& gr = m.grid;
    double t_lo = spec->t_lo, t_hi = spec->t_hi;
    if (!(t_hi > t_lo)) {
        t_lo = gr.s0 - 0.5 * gr.dt_src;
        t_hi = gr.s0 + (gr.n_hat - 0.5) * gr.dt_src;
    }
    // factor tables on the nodes
    std::vector<double> R((size_t)nR * gr.n_r), P((size_t)nA * gr.n_phi), T((size_t)nT * gr.n_hat);
    std::vector<double> tmp(nR);
    const double lr = std::log(gr.r_in), lw = std::log(gr.r_out) - std::log(gr.r_in);
    for (int i = 0; i < gr.n_r; ++i) {
        const double r = gr.r_in + (i + 0.5) * (gr.r_out - gr.r_in) / gr.n_r;
        const double u = std::min(1.0, std::max(0.0, (std::log(r) - lr) / lw));
        cubic_bsplines(u, nR, tmp.data());
        for (int a = 0; a < nR; ++a) R[(size_t)a * gr.n_r + i] = tmp[a];
    }
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < gr.n_phi; ++j) {
        const double phi = (j + 0.5) * two_pi / gr.n_phi;
        P[j] = 1.0;
        for (int q = 1; q <= mmax; ++q) {
            P[(size_t)(2 * q - 1) * gr.n_phi + j] = std::cos(q * phi);
            P[(size_t)(2 * q) * gr.n_phi + j] = std::sin(q * phi);
        }
    }
    const double pi = 3.14159265358979323846264338327950288;
    for (int k = 0; k < gr.n_hat; ++k) {
        const double t = gr.s0 + gr.dt_src * k;
        for (int c = 0; c < nT; ++c) {
            double v;
            if (spec->temporal == RTT_SYNTH_DCT) {
                v = std::cos(pi * c * (t - t_lo) / (t_hi - t_lo));
            } else {
                const double w = (t_hi - t_lo) / (nT - 1);
                v = std::max(0.0, 1.0 - std::fabs(t - (t_lo + c * w)) / w);
            }
            T[(size_t)c * gr.n_hat + k] = v;
        }
    }
    auto s = new rtt_synthesis();
    s->member = gi;
    s->n_radial = nR;
    s->m_max = mmax;
    s->n_temporal = nT;
    s->temporal = spec->temporal;
    s->d = (int)d;
    s->n_az = nA;
    s->t_lo = t_lo;
    s->t_hi = t_hi;
    s->n_cols = m.n_cols;
    s->device = g->device;
    hipError_t e = hipSetDevice(s->device);
    double *dR = nullptr, *dP = nullptr, *dT = nullptr;
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_Q, sizeof(float) * (size_t)d * m.n_cols);
    if (e == hipSuccess) e = hipMalloc((void**)&dR, sizeof(double) * R.size());
    if (e == hipSuccess) e = hipMalloc((void**)&dP, sizeof(double) * P.size());
    if (e == hipSuccess) e = hipMalloc((void**)&dT, sizeof(double) * T.size());
    if (e == hipSuccess) e = hipMemcpy(dR, R.data(), sizeof(double) * R.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dP, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dT, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_synth_rows, dim3((unsigned)((m.n_cols + 255) / 256), (unsigned)d), dim3(256), 0, 0, dR, dP,
                           dT, gr.n_r, gr.n_phi, gr.n_hat, nA, nT, m.n_cols, s->d_Q);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    for (double* p : {dR, dP, dT})
        if (p) (void)hipFree(p);
    s->n_r = gr.n_r;
    s->n_phi = gr.n_phi;
    s->K = gr.n_hat;
    s->separable = d + (int64_t)nR * nA * gr.n_hat + (int64_t)nA * gr.n_hat <= SYN_LDS &&
                   (int64_t)gr.n_phi * gr.n_hat + (int64_t)gr.n_phi * nT + (int64_t)nA * nT <= SYN_LDS;
    if (e == hipSuccess) {
        std::vector<float> fR(R.begin(), R.end()), fP(P.begin(), P.end()), fT(T.begin(), T.end());
        auto up = [&](float** dst, const std::vector<float>& h) {
            if (e != hipSuccess) return;
            e = hipMalloc((void**)dst, sizeof(float) * h.size());
            if (e == hipSuccess) e = hipMemcpy(*dst, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice);
        };
        up(&s->d_R, fR);
        up(&s->d_P, fP);
        up(&s->d_T, fT);
    }
    if (e != hipSuccess) {
        for (float* p : {s->d_Q, s->d_R, s->d_P, s->d_T})
            if (p) (void)hipFree(p);
        s->magic = 0;
        delete s;
        return e == hipErrorOutOfMemory ? fail(RTT_ENOMEM, "synthesis tables") : hip_fail(e, "synthesis_create");
    }
    *out = s;
    return RTT_OK;
}

extern "C" int synthesis_free(rtt_synthesis* s)
{
    if (!s) return RTT_OK;
    if (!valid_syn(s)) return fail(RTT_EINVAL, "invalid synthesis handle");
    (void)hipSetDevice(s->device);
    for (float* p : {s->d_Q, s->d_R, s->d_P, s->d_T})
        if (p) (void)hipFree(p);
    s->ws.release();
    s->magic = 0;
    delete s;
    return RTT_OK;
}

extern "C" int synthesis_info(const rtt_synthesis* s, int32_t* d, int64_t* n_cols, const float** rows)
{
    if (!valid_syn(s)) return fail(RTT_EINVAL, "invalid synthesis handle");
    if (d) *d = s->d;
    if (n_cols) *n_cols = s->n_cols;
    if (rows) *rows = s->d_Q;
    return RTT_OK;
}

extern "C" int synth_expand(const rtt_synthesis* s, const float* c, float* x, int32_t nvec, void* stream)
{
    int rc = check_syn(s, nvec);
    if (rc) return rc;
    if (nvec == 0) return RTT_OK;
    if (!c || !x) return fail(RTT_EINVAL, "NULL data pointer");
    hipStream_t st = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(s->device));
    if (s->separable) {
        const size_t lds = sizeof(float) * ((size_t)s->d + (size_t)s->n_radial * s->n_az * s->K + (size_t)s->n_az * s->K);
        hipLaunchKernelGGL(k_synth_expand, dim3((unsigned)s->n_r, (unsigned)nvec), dim3(256), lds, st, s->d_R, s->d_P,
                           s->d_T, s->n_radial, s->n_az, s->n_temporal, s->n_r, s->n_phi, s->K, c, x, s->n_cols);
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    float* Ct = (float*)s->ws.get("ct", sizeof(float) * (size_t)s->d * nvec);
    if (!Ct) return fail(RTT_ENOMEM, "synth_expand scratch");
    const int64_t tot = (int64_t)s->d * nvec;
    hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, c, nvec, s->d, Ct);
    RTT_HIP(hipGetLastError());
    return combine(Ct, s->d, nvec, s->d_Q, s->n_cols, x, s->n_cols, s->n_cols, 0.f, st);
}

extern "C" int synth_project(const rtt_synthesis* s, const float* x, float* c, int32_t nvec, void* stream)
{
    int rc = check_syn(s, nvec);
    if (rc) return rc;
    if (nvec == 0) return RTT_OK;
    if (!c || !x) return fail(RTT_EINVAL, "NULL data pointer");
    hipStream_t st = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(s->device));
    if (s->separable) {
        float* part = (float*)s->ws.get("part", sizeof(float) * (size_t)nvec * s->n_r * s->d);
        if (!part) return fail(RTT_ENOMEM, "synth_project scratch");
        const size_t lds = sizeof(float) * ((size_t)s->n_phi * s->K + (size_t)s->n_phi * s->n_temporal +
                                            (size_t)s->n_az * s->n_temporal);
        hipLaunchKernelGGL(k_synth_project_part, dim3((unsigned)s->n_r, (unsigned)nvec), dim3(256), lds, st, s->d_R,
                           s->d_P, s->d_T, s->n_radial, s->n_az, s->n_temporal, s->n_r, s->n_phi, s->K, x, s->n_cols,
                           part);
        const int64_t tot = (int64_t)s->d * nvec;
        hipLaunchKernelGGL(k_synth_project_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, s->n_r,
                           s->d, nvec, c);
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    double* G = (double*)s->ws.get("g", sizeof(double) * (size_t)s->d * nvec);
    if (!G) return fail(RTT_ENOMEM, "synth_project scratch");
    if ((rc = gram(s->ws, s->d_Q, s->n_cols, x, s->n_cols, s->d, nvec, s->n_cols, G, st))) return rc;
    const int64_t tot = (int64_t)s->d * nvec;
    hipLaunchKernelGGL(k_gram_to_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, G, s->d, nvec, c);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

extern "C" int synthesis_audit(const rtt_geometry* g, const rtt_synthesis* s, uint32_t order_mask, double* sigma,
                               uint8_t* zero, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    int rc = check_syn(s, 0);
    if (rc) return rc;
    if (s->member >= (int)g->members.size() || g->members[s->member].n_cols != s->n_cols)
        return fail(RTT_EINVAL, "the synthesis belongs to another geometry");
    if (!sigma && !zero) return RTT_OK;
    hipStream_t st = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(s->device));
    const Member& m = g->members[s->member];
    const int d = s->d;
    const int64_t rows = m.n_rows;
    Workspace ws;
    float* Y = (float*)ws.get("y", sizeof(float) * (size_t)d * rows);
    double* nrm = (double*)ws.get("n", sizeof(double) * (size_t)d);
    int64_t* seg = (int64_t*)ws.get("seg", sizeof(int64_t) * 2);
    if (!Y || !nrm || !seg) return fail(RTT_ENOMEM, "synthesis_audit scratch");
    // A^(d) rows: A applied to the rows of Q (rows of orders outside the mask stay zero)
    if ((rc = fill(Y, (int64_t)d * rows, 0.f, st))) return rc;
    if ((rc = apply_op(g, s->member, false, s->d_Q, Y, d, order_mask, st))) return rc;
    const int64_t hs[2] = {0, rows};
    RTT_HIP(hipMemcpyAsync(seg, hs, sizeof(hs), hipMemcpyHostToDevice, st));
    if ((rc = dots_seg(ws, Y, rows, Y, rows, seg, 1, rows, d, nrm, st))) return rc;
    const int tiles = (d + GT - 1) / GT;
    const int nsl = gram_slices(d, rows, 1);
    double* Gp = (double*)ws.get("gp", sizeof(double) * (size_t)nsl * d * d);
    if (!Gp) return fail(RTT_ENOMEM, "synthesis_audit scratch");
    hipLaunchKernelGGL(k_gram_f64, dim3((unsigned)tiles, (unsigned)tiles, (unsigned)nsl), dim3(GT * GT), 0, st, Y, rows,
                       d, rows, nsl, Gp);
    RTT_HIP(hipGetLastError());
    std::vector<double> hGp((size_t)nsl * d * d), hG((size_t)d * d, 0.0), hn(d);
    RTT_HIP(hipMemcpyAsync(hGp.data(), Gp, sizeof(double) * hGp.size(), hipMemcpyDeviceToHost, st));
    RTT_HIP(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * d, hipMemcpyDeviceToHost, st));
    RTT_HIP(hipStreamSynchronize(st));
    for (int z = 0; z < nsl; ++z)
        for (size_t e = 0; e < hG.size(); ++e) hG[e] += hGp[(size_t)z * d * d + e];
    if (zero)
        for (int c = 0; c < d; ++c) zero[c] = hn[c] == 0.0 ? 1 : 0;
    if (sigma) {
        // lower tiles were skipped: mirror the upper triangle
        for (int u = 0; u < d; ++u)
            for (int v = 0; v < u; ++v) hG[(size_t)u * d + v] = hG[(size_t)v * d + u];
        std::vector<double> U, sv, W;
        jacobi_svd(hG, d, U, sv, W);
        for (int i = 0; i < d; ++i) sigma[i] = std::sqrt(std::max(0.0, sv[i]));
    }
    return RTT_OK;
}

extern "C" int age_fisher(const rtt_geometry* g, const rtt_synthesis* s, const double* ages, int32_t n_ages, double h,
                          uint32_t order_mask, double* M, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    int rc = check_syn(s, 0);
    if (rc) return rc;
    if (s->member >= (int)g->members.size() || g->members[s->member].n_cols != s->n_cols)
        return fail(RTT_EINVAL, "the synthesis belongs to another geometry");
    if (n_ages < 0 || (n_ages > 0 && (!ages || !M))) return fail(RTT_EINVAL, "bad ages or output");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(RTT_EINVAL, "h must be positive and finite");
    if (n_ages == 0) return RTT_OK;
    const Member& m = g->members[s->member];
    const rtt_grid& gr = m.grid;
    const int nR = s->n_radial, nA = s->n_az, L = nR * nA;
    // N_l of eq. (14): h sqrt(pi) * int R_a(r)^2 r dr * int Phi_b^2 dphi (2 pi or pi); the radial
    // integral of the continuum B-spline by composite 8-point Gauss-Legendre on 256 panels
    static const double gx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                                 0.1834346424956498,  0.5255324099163290,  0.7966664774136267,  0.9602898564975363};
    static const double gw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                                 0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    std::vector<double> rad(nR, 0.0), bs(nR);
    const double lr = std::log(gr.r_in), lw = std::log(gr.r_out) - lr;
    const int panels = 256;
    const double hp = (gr.r_out - gr.r_in) / panels;
    for (int p = 0; p < panels; ++p)
        for (int q = 0; q < 8; ++q) {
            const double r = gr.r_in + hp * (p + 0.5 + 0.5 * gx[q]);
            cubic_bsplines(std::min(1.0, std::max(0.0, (std::log(r) - lr) / lw)), nR, bs.data());
            for (int a = 0; a < nR; ++a) rad[a] += 0.5 * hp * gw[q] * bs[a] * bs[a] * r;
        }
    const double pi = 3.14159265358979323846264338327950288;
    std::vector<double> inv_n(L);
    for (int a = 0; a < nR; ++a)
        for (int b = 0; b < nA; ++b)
            inv_n[a * nA + b] = 1.0 / std::sqrt(rad[a] * (b == 0 ? 2.0 * pi : pi) * h * std::sqrt(pi));
    hipStream_t st = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(s->device));
    const int64_t per_age = (int64_t)L * (m.n_rows + m.n_cols) * 4;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(n_ages, 2048 / L), (int64_t(1) << 30) / per_age));
    Workspace ws;
    float* X = (float*)ws.get("x", sizeof(float) * (size_t)chunk * L * m.n_cols);
    float* Y = (float*)ws.get("y", sizeof(float) * (size_t)chunk * L * m.n_rows);
    double* dn = (double*)ws.get("n", sizeof(double) * L);
    double* da = (double*)ws.get("a", sizeof(double) * n_ages);
    if (!X || !Y || !dn || !da) return fail(RTT_ENOMEM, "age_fisher scratch");
    RTT_HIP(hipMemcpyAsync(dn, inv_n.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
    RTT_HIP(hipMemcpyAsync(da, ages, sizeof(double) * n_ages, hipMemcpyHostToDevice, st));
    std::vector<double> hG((size_t)chunk * L * L);
    for (int a0 = 0; a0 < n_ages; a0 += chunk) {
        const int nv = std::min(chunk, n_ages - a0);
        hipLaunchKernelGGL(k_local_probe, dim3((unsigned)((m.n_cols + 255) / 256), (unsigned)(nv * L)), dim3(256), 0, st,
                           s->d_R, s->d_P, dn, da + a0, nR, nA, gr.n_r, gr.n_phi, gr.n_hat, gr.s0, gr.dt_src, h,
                           m.n_cols, X);
        RTT_HIP(hipGetLastError());
        if ((rc = fill(Y, (int64_t)nv * L * m.n_rows, 0.f, st))) return rc;
        if ((rc = apply_op(g, s->member, false, X, Y, nv * L, order_mask, st))) return rc;
        const int tiles = (L + GT - 1) / GT;
        const int nsl = gram_slices(L, m.n_rows, nv);
        double* Gp = (double*)ws.get("gp", sizeof(double) * (size_t)chunk * nsl * L * L);
        if (!Gp) return fail(RTT_ENOMEM, "age_fisher scratch");
        hipLaunchKernelGGL(k_gram_f64, dim3((unsigned)tiles, (unsigned)tiles, (unsigned)(nv * nsl)), dim3(GT * GT), 0, st,
                           Y, m.n_rows, L, m.n_rows, nsl, Gp);
        RTT_HIP(hipGetLastError());
        std::vector<double> hGp((size_t)nv * nsl * L * L);
        RTT_HIP(hipMemcpyAsync(hGp.data(), Gp, sizeof(double) * hGp.size(), hipMemcpyDeviceToHost, st));
        RTT_HIP(hipStreamSynchronize(st));
        for (int v = 0; v < nv; ++v) {
            double* out = M + (size_t)(a0 + v) * L * L;
            std::fill(hG.begin(), hG.begin() + (size_t)L * L, 0.0);
            for (int z = 0; z < nsl; ++z)
                for (size_t e = 0; e < (size_t)L * L; ++e) hG[e] += hGp[((size_t)v * nsl + z) * L * L + e];
            for (int u = 0; u < L; ++u)
                for (int w = 0; w < L; ++w) out[(size_t)u * L + w] = u <= w ? hG[(size_t)u * L + w] : hG[(size_t)w * L + u];
        }
    }
    return RTT_OK;
}
