// Age-localised probes and historical reach (Sec. 3.3 eq. (10)-(13), Sec. 3.5 eq. (17), Sec. 4.4
// eq. (29)-(30), Sec. 6.5 eq. (35)).
//
// age_information builds the probes q_a on the coefficient nodes (flat in space, a Gaussian of
// width h in source time, unit L2 norm over the annulus), applies A to a block of them with the
// operator kernels, and reduces the squared responses per (age, geometry, order) -- or, through an
// order mixer, the squared mixed responses weighted by the propagated inverse variances -- in
// FP64.  The threshold statistics (age_window, age_reach) are host arithmetic on those numbers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rtt.h"
#include "rtt_internal.h"
#include "dense.h"

namespace rtt {
namespace {

constexpr double PI = 3.14159265358979323846264338327950288;

// X[v][c] for the columns of one geometry: exp(-(s_k + a_v)^2 / (2 h^2)) / N_h, k = c mod K
__global__ void k_age_probe(float* __restrict__ X, int64_t ldx, int64_t col_off, int64_t n_cols, int K, double s0,
                            double dt_src, const double* __restrict__ ages, double h, double inv_norm)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cols) return;
    const int v = blockIdx.y;
    const double t = s0 + dt_src * (double)(c % K) + ages[v];
    X[(int64_t)v * ldx + col_off + c] = (float)(exp(-t * t / (2.0 * h * h)) * inv_norm);
}

// W[v][i] = D[v][i] / var[i] (0 where var[i] == 0)
__global__ void k_div_rows(const float* __restrict__ D, const float* __restrict__ var, int64_t n, float* __restrict__ W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t v = blockIdx.y;
    const float q = var[i];
    W[v * n + i] = q != 0.f ? D[v * n + i] / q : 0.f;
}

// Partial per-hat sums over a slice of cells: S[v][z][k] = sum (xh - x)^2, T[v][z][k] = sum x^2 (FP64)
__global__ void k_hat_sums(const float* __restrict__ xh, const float* __restrict__ x, int64_t ld, int64_t col_off,
                           int n_cells, int K, int cells_per_slice, double* __restrict__ S, double* __restrict__ T)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t v = blockIdx.y;
    const int z = blockIdx.z;
    const float* a = xh + v * ld + col_off;
    const float* b = x + v * ld + col_off;
    const int c0 = z * cells_per_slice, c1 = min(n_cells, c0 + cells_per_slice);
    double s = 0.0, t = 0.0;
    for (int c = c0; c < c1; ++c) {
        const double xb = (double)b[(int64_t)c * K + k];
        const double d = (double)a[(int64_t)c * K + k] - xb;
        s += d * d;
        t += xb * xb;
    }
    const int64_t o = (v * gridDim.z + z) * K + k;
    S[o] = s;
    T[o] = t;
}

// N_h of eq. (11)
double probe_norm(const rtt_grid& g, double h)
{
    return std::sqrt(PI * (g.r_out * g.r_out - g.r_in * g.r_in) * h * std::sqrt(PI));
}

// weight of the direct data (rays p, frames f) with age Delta_p - t_f <= a
double direct_weight_below(const Member& m, const std::vector<double>& d, const std::vector<double>& w, double a)
{
    const int64_t F = m.grid.n_frames;
    double acc = 0.0;
    for (size_t p = 0; p < d.size(); ++p) {
        // frames f with t0 + f dt >= Delta_p - a
        const double x = (d[p] - a - m.grid.t0) / m.grid.dt_obs;
        const double f0 = std::ceil(x);
        const int64_t first = f0 <= 0.0 ? 0 : (f0 >= (double)F ? F : (int64_t)f0);
        acc += w[p] * (double)(F - first);
    }
    return acc;
}

}  // namespace
}  // namespace rtt

using namespace rtt;

extern "C" int reference_response(const rtt_geometry* g, double* s_ref, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (!s_ref) return fail(RTT_EINVAL, "NULL output pointer");
    hipStream_t s = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(g->device));
    const int G = (int)g->members.size();
    Workspace ws;
    float* x = (float*)ws.get("ones", sizeof(float) * (size_t)g->n_cols);
    float* y = (float*)ws.get("y", sizeof(float) * (size_t)g->n_rows);
    int64_t* seg = (int64_t*)ws.get("seg", sizeof(int64_t) * 2 * (size_t)G);
    double* e = (double*)ws.get("e", sizeof(double) * (size_t)G);
    if (!x || !y || !seg || !e) return fail(RTT_ENOMEM, "reference_response scratch");
    std::vector<int64_t> hs;
    int64_t max_len = 1;
    for (const Member& m : g->members) {
        const int64_t len = m.rays_per_order[0] * m.grid.n_frames;
        hs.insert(hs.end(), {m.row_offset, len});
        max_len = std::max(max_len, len);
    }
    int rc = fill(x, g->n_cols, 1.0f, s);
    if (!rc) rc = apply_op(g, -1, false, x, y, 1, 1u, s);
    if (rc) return rc;
    RTT_HIP(hipMemcpyAsync(seg, hs.data(), hs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    rc = dots_seg(ws, y, g->n_rows, y, g->n_rows, seg, G, max_len, 1, e, s);
    if (rc) return rc;
    std::vector<double> he(G);
    RTT_HIP(hipMemcpyAsync(he.data(), e, sizeof(double) * G, hipMemcpyDeviceToHost, s));
    RTT_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < G; ++i) {
        const double m0 = (double)(g->members[i].rays_per_order[0] * g->members[i].grid.n_frames);
        s_ref[i] = m0 > 0 ? std::sqrt(he[i] / m0) : 0.0;
    }
    return RTT_OK;
}

extern "C" int age_information(const rtt_geometry* g, const double* ages, int32_t n_ages, double h,
                               const rtt_mixer* mixer, const float* var, double* energy, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (n_ages < 0) return fail(RTT_EINVAL, "n_ages must be >= 0");
    if (n_ages > 0 && (!ages || !energy)) return fail(RTT_EINVAL, "NULL ages or output");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(RTT_EINVAL, "h must be positive and finite");
    for (int i = 0; i < n_ages; ++i)
        if (!std::isfinite(ages[i])) return fail(RTT_EINVAL, "ages must be finite");
    if (mixer) {
        if (!mixer_ok(mixer)) return fail(RTT_EINVAL, "invalid mixer handle");
        if (mixer_src_rows(mixer) != g->n_rows) return fail(RTT_EINVAL, "the mixer was built for another geometry");
    }
    if (var && ((uintptr_t)var & 3)) return fail(RTT_EINVAL, "var must be 4-byte aligned");
    if (n_ages == 0) return RTT_OK;
    hipStream_t s = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(g->device));
    // segments: (geometry, order) row blocks, or every geometry's mixed rows
    std::vector<int64_t> hseg;
    if (!mixer) {
        for (const Member& m : g->members) {
            int64_t off = m.row_offset;
            for (int n = 0; n < 8; ++n) {
                const int64_t len = n < m.grid.n_orders ? m.rays_per_order[n] * m.grid.n_frames : 0;
                hseg.insert(hseg.end(), {off, len});
                off += len;
            }
        }
    } else {
        mixer_segments(mixer, hseg);
    }
    const int nseg = (int)(hseg.size() / 2);
    int64_t max_len = 1;
    for (int i = 0; i < nseg; ++i) max_len = std::max(max_len, hseg[2 * i + 1]);
    const int64_t rows_out = mixer ? mixer_rows(mixer) : g->n_rows;
    // ages per pass: the response block stays under 1 GiB
    const int64_t per_age = 4 * (g->n_rows + g->n_cols + (mixer ? 2 * rows_out : 0));
    const int chunk = (int)std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>(n_ages, 65535), (int64_t(1) << 30) / std::max<int64_t>(per_age, 1)));
    Workspace ws;
    float* X = (float*)ws.get("X", sizeof(float) * (size_t)chunk * g->n_cols);
    float* Y = (float*)ws.get("Y", sizeof(float) * (size_t)chunk * g->n_rows);
    double* dages = (double*)ws.get("ages", sizeof(double) * (size_t)n_ages);
    int64_t* seg = (int64_t*)ws.get("seg", sizeof(int64_t) * hseg.size());
    double* e = (double*)ws.get("e", sizeof(double) * (size_t)n_ages * nseg);
    float *D = nullptr, *W = nullptr, *varL = nullptr, *ones = nullptr;
    if (mixer) {
        D = (float*)ws.get("D", sizeof(float) * (size_t)chunk * rows_out);
        W = (float*)ws.get("W", sizeof(float) * (size_t)chunk * rows_out);
        varL = (float*)ws.get("varL", sizeof(float) * (size_t)std::max<int64_t>(rows_out, 1));
        if (!var) ones = (float*)ws.get("ones", sizeof(float) * (size_t)g->n_rows);
        if (!D || !W || !varL || (!var && !ones)) return fail(RTT_ENOMEM, "age_information scratch");
    }
    if (!X || !Y || !dages || !seg || !e) return fail(RTT_ENOMEM, "age_information scratch");
    RTT_HIP(hipMemcpyAsync(dages, ages, sizeof(double) * n_ages, hipMemcpyHostToDevice, s));
    RTT_HIP(hipMemcpyAsync(seg, hseg.data(), hseg.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    int rc = RTT_OK;
    if (mixer) {
        // propagated variances: diag(C_L) = (L kron I) var (every source row feeds one mixed row)
        if (!var) {
            rc = fill(ones, g->n_rows, 1.0f, s);
            if (rc) return rc;
        }
        rc = mix_forward(mixer, var ? var : ones, g->n_rows, varL, rows_out, 1, s);
        if (rc) return rc;
    }
    for (int a0 = 0; a0 < n_ages; a0 += chunk) {
        const int nv = std::min(chunk, n_ages - a0);
        for (const Member& m : g->members) {
            const dim3 grid((unsigned)((m.n_cols + 255) / 256), (unsigned)nv);
            hipLaunchKernelGGL(k_age_probe, grid, dim3(256), 0, s, X, g->n_cols, m.col_offset, m.n_cols,
                               m.grid.n_hat, m.grid.s0, m.grid.dt_src, dages + a0, h, 1.0 / probe_norm(m.grid, h));
        }
        RTT_HIP(hipGetLastError());
        rc = apply_op(g, -1, false, X, Y, nv, 0u, s);
        if (rc) return rc;
        if (!mixer) {
            rc = dots_seg(ws, Y, g->n_rows, Y, g->n_rows, seg, nseg, max_len, nv, e + (int64_t)a0 * nseg, s);
        } else {
            rc = mix_forward(mixer, Y, g->n_rows, D, rows_out, nv, s);
            if (!rc && rows_out > 0) {
                hipLaunchKernelGGL(k_div_rows, dim3((unsigned)((rows_out + 255) / 256), (unsigned)nv), dim3(256), 0, s,
                                   D, varL, rows_out, W);
                RTT_HIP(hipGetLastError());
            }
            if (!rc) rc = dots_seg(ws, D, rows_out, W, rows_out, seg, nseg, max_len, nv, e + (int64_t)a0 * nseg, s);
        }
        if (rc) return rc;
    }
    std::vector<double> he((size_t)n_ages * nseg);
    RTT_HIP(hipMemcpyAsync(he.data(), e, sizeof(double) * he.size(), hipMemcpyDeviceToHost, s));
    RTT_HIP(hipStreamSynchronize(s));
    // [age][geometry][8 orders], or [age][geometry] through a mixer
    std::memcpy(energy, he.data(), sizeof(double) * he.size());
    return RTT_OK;
}

extern "C" int age_window(const rtt_geometry* geom, int32_t gi, uint32_t order_mask, double h, double q,
                          double* a_min, double* a_max, double* boundary)
{
    if (!valid_handle(geom)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (gi < 0 || gi >= (int32_t)geom->members.size()) return fail(RTT_EINVAL, "geometry index out of range");
    if (!(h >= 0.0) || !std::isfinite(h)) return fail(RTT_EINVAL, "h must be finite and >= 0");
    if (boundary && !(q > 0.0 && q <= 1.0)) return fail(RTT_EINVAL, "q must be in (0, 1]");
    const Member& m = geom->members[gi];
    const uint32_t mask = order_mask ? order_mask : 0xFFu;
    double dmin = HUGE_VAL, dmax = -HUGE_VAL;
    for (int n = 0; n < m.grid.n_orders; ++n)
        if ((mask >> n) & 1u) {
            dmin = std::min(dmin, m.delay_min[n]);
            dmax = std::max(dmax, m.delay_max[n]);
        }
    // reached source times (eq. (13)): [t_first - dmax, t_last - dmin]; a probe centred at -a with
    // support |t + a| <= 3h fits when 3h - (t_last - dmin) <= a <= (dmax - t_first) - 3h
    const double t_first = m.grid.t0, t_last = m.grid.t0 + m.grid.dt_obs * (m.grid.n_frames - 1);
    if (a_min) *a_min = dmin <= dmax ? 3.0 * h - (t_last - dmin) : HUGE_VAL;
    if (a_max) *a_max = dmin <= dmax ? (dmax - t_first) - 3.0 * h : -HUGE_VAL;
    if (boundary) {
        const std::vector<double>& d = geom->dir_delay[gi];
        const std::vector<double>& w = geom->dir_weight[gi];
        if (d.empty()) {
            *boundary = std::nan("");
            return RTT_OK;
        }
        const double total = direct_weight_below(m, d, w, HUGE_VAL);
        const double target = q * total;
        double lo = *std::min_element(d.begin(), d.end()) - t_last - 1.0;
        double hi = *std::max_element(d.begin(), d.end()) - t_first;
        // smallest data age with weight below it >= target: bisection, then snap to that age
        for (int it = 0; it < 200 && hi - lo > 1e-12 * std::max(1.0, std::fabs(hi)); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (direct_weight_below(m, d, w, mid) >= target)
                hi = mid;
            else
                lo = mid;
        }
        const double tol = 1e-9 * std::max(1.0, std::fabs(hi));
        double best = -HUGE_VAL;
        for (size_t p = 0; p < d.size(); ++p) {
            const double f0 = std::ceil((d[p] - hi - t_first) / m.grid.dt_obs - 1e-9);
            const int64_t f = f0 <= 0.0 ? 0 : (int64_t)f0;
            if (f >= m.grid.n_frames) continue;
            const double age = d[p] - (t_first + m.grid.dt_obs * (double)f);
            if (age <= hi + tol) best = std::max(best, age);
        }
        *boundary = best;
    }
    return RTT_OK;
}

extern "C" int age_reach(const double* ages, const double* info, int32_t n, double rho, double a_min, double a_max,
                         double boundary, uint8_t* mask_out, rtt_reach* out)
{
    if (n < 1 || !ages || !info || !out) return fail(RTT_EINVAL, "need n >= 1 ages, info and an output");
    if (!(rho >= 0.0)) return fail(RTT_EINVAL, "rho must be >= 0");
    const double step = n > 1 ? ages[1] - ages[0] : 0.0;
    for (int i = 1; i < n; ++i)
        if (!(ages[i] - ages[i - 1] > 0.0) || std::fabs((ages[i] - ages[i - 1]) - step) > 1e-9 * std::max(1.0, std::fabs(step)))
            return fail(RTT_EINVAL, "ages must be ascending and equally spaced");
    std::memset(out, 0, sizeof *out);
    const double nan = std::nan("");
    out->t_reach = out->l_anchor = out->longest = nan;
    out->anchor = -1;
    std::vector<uint8_t> pass(n);
    for (int i = 0; i < n; ++i) {
        pass[i] = info[i] >= rho * rho;
        if (mask_out) mask_out[i] = pass[i];
        if (pass[i]) {
            out->t_reach = ages[i];
            out->n_pass++;
        }
    }
    for (int i = 0; i < n; ++i)
        if (ages[i] >= a_min && ages[i] <= a_max) {
            out->anchor = i;
            break;
        }
    if (out->anchor >= 0 && pass[out->anchor]) {
        int j = out->anchor;
        while (j + 1 < n && pass[j + 1]) ++j;
        out->l_anchor = ages[j] - ages[out->anchor];
    }
    for (int i = 0; i < n;) {
        if (!pass[i]) {
            ++i;
            continue;
        }
        int j = i;
        while (j + 1 < n && pass[j + 1]) ++j;
        const double ext = ages[j] - ages[i];
        if (std::isnan(out->longest) || ext > out->longest) out->longest = ext;
        i = j + 1;
    }
    double jo = 0.0;
    for (int i = 0; i < n; ++i)
        if (ages[i] > boundary) jo += std::log1p(info[i]) * step;
    out->j_old = std::isnan(boundary) ? nan : jo;
    return RTT_OK;
}

extern "C" int age_window_error(const rtt_geometry* g, const float* x_hat, const float* x, int32_t nvec,
                                const double* ages, int32_t n_ages, double half_width, double eta, double* err,
                                void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (nvec < 0 || nvec > 65535 || n_ages < 0) return fail(RTT_EINVAL, "nvec must be 0..65535, n_ages >= 0");
    if (nvec > 0 && n_ages > 0 && (!x_hat || !x || !ages || !err)) return fail(RTT_EINVAL, "NULL pointer");
    if (!(half_width >= 0.0) || !(eta >= 0.0)) return fail(RTT_EINVAL, "half_width and eta must be >= 0");
    if (nvec == 0 || n_ages == 0) return RTT_OK;
    hipStream_t s = (hipStream_t)stream;
    RTT_HIP(hipSetDevice(g->device));
    const int G = (int)g->members.size();
    int maxK = 1;
    for (const Member& m : g->members) maxK = std::max(maxK, (int)m.grid.n_hat);
    const int nsl = 64;
    Workspace ws;
    double* S = (double*)ws.get("S", sizeof(double) * (size_t)nvec * nsl * maxK);
    double* T = (double*)ws.get("T", sizeof(double) * (size_t)nvec * nsl * maxK);
    if (!S || !T) return fail(RTT_ENOMEM, "age_window_error scratch");
    std::vector<double> hS((size_t)nvec * nsl * maxK), hT(hS.size());
    for (int gi = 0; gi < G; ++gi) {
        const Member& m = g->members[gi];
        const int K = m.grid.n_hat, nc = m.grid.n_r * m.grid.n_phi;
        const int cps = (nc + nsl - 1) / nsl;
        const int z = (nc + cps - 1) / cps;
        hipLaunchKernelGGL(k_hat_sums, dim3((unsigned)((K + 63) / 64), (unsigned)nvec, (unsigned)z), dim3(64), 0, s,
                           x_hat, x, g->n_cols, m.col_offset, nc, K, cps, S, T);
        RTT_HIP(hipGetLastError());
        RTT_HIP(hipMemcpyAsync(hS.data(), S, sizeof(double) * (size_t)nvec * z * K, hipMemcpyDeviceToHost, s));
        RTT_HIP(hipMemcpyAsync(hT.data(), T, sizeof(double) * (size_t)nvec * z * K, hipMemcpyDeviceToHost, s));
        RTT_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < nvec; ++v) {
            // per-hat sums: slices added in slice order
            std::vector<double> sk(K, 0.0), tk(K, 0.0);
            for (int zz = 0; zz < z; ++zz)
                for (int k = 0; k < K; ++k) {
                    sk[k] += hS[((size_t)v * z + zz) * K + k];
                    tk[k] += hT[((size_t)v * z + zz) * K + k];
                }
            for (int i = 0; i < n_ages; ++i) {
                double num = 0.0, den = 0.0;
                for (int k = 0; k < K; ++k) {
                    const double sc = m.grid.s0 + m.grid.dt_src * k;
                    if (std::fabs(sc + ages[i]) <= half_width) {
                        num += sk[k];
                        den += tk[k];
                    }
                }
                err[((size_t)v * G + gi) * n_ages + i] = std::sqrt(num) / std::max(std::sqrt(den), eta);
            }
        }
    }
    return RTT_OK;
}
