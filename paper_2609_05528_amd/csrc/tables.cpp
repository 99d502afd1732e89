// geometry_load: host-side FP64 table build (stencils, hat origins, base-cell sort, CSR).
//
// Every ray's spatial stencil and time origin is evaluated once here in FP64
// and rounded to FP32 once; the kernels then step from frame to frame with
// exact integer arithmetic.  This keeps the retarded-time positions exact to
// FP64 accuracy even where absolute times reach 10^3 M.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <sstream>

#include "dense.h"

namespace rtt {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg)
{
    g_err = msg;
    if (std::getenv("RTT_LOG")) std::fprintf(stderr, "[rtt] error %d: %s\n", code, msg.c_str());
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(e);
    return fail(e == hipErrorOutOfMemory ? RTT_ENOMEM : RTT_EDEVICE, os.str());
}

bool valid_handle(const rtt_geometry* g) { return g && g->magic == 0x52545447u && g->d_rays; }

uint64_t fnv1a(const void* data, size_t n, uint64_t h)
{
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint32_t effective_mask(const Member& m, uint32_t mask)
{
    uint32_t all = (m.grid.n_orders >= 32) ? 0xffffffffu : ((1u << m.grid.n_orders) - 1u);
    return mask == 0 ? all : (mask & all);
}

// dt_obs/dt_src as an exact small rational P/Q
static bool exact_ratio(double dt_obs, double dt_src, int n_frames, int32_t* P, int32_t* Q)
{
    if (n_frames <= 1) { *P = 1; *Q = 1; return true; }  // only f = 0 exists
    double ratio = dt_obs / dt_src;
    if (!(ratio > 0.0) || !std::isfinite(ratio)) return false;
    for (int q = 1; q <= 64; ++q) {
        double p = std::round(ratio * q);
        if (p < 1.0 || p > 4096.0) continue;
        if (std::fabs(p / q - ratio) <= 1e-12 * ratio) {
            int pi = (int)p, g = std::gcd(pi, q);
            *P = pi / g; *Q = q / g;
            return true;
        }
    }
    return false;
}

static int check_grid(const rtt_grid& g, int idx)
{
    std::ostringstream os;
    os << "geometry " << idx << ": ";
    if (g.n_orders < 1 || g.n_orders > 8) return fail(RTT_EINVAL, os.str() + "n_orders must be 1..8");
    if (g.n_frames < 1 || g.n_frames > 65536) return fail(RTT_EINVAL, os.str() + "n_frames must be 1..65536");
    if (g.n_r < 2 || g.n_phi < 1) return fail(RTT_EINVAL, os.str() + "need n_r >= 2 and n_phi >= 1");
    if (g.n_hat < 2) return fail(RTT_EINVAL, os.str() + "need n_hat >= 2");
    if ((int64_t)g.n_r * g.n_phi > (1 << 26) || (int64_t)g.n_r * g.n_phi * g.n_hat > (1ll << 31) - 1)
        return fail(RTT_EINVAL, os.str() + "coefficient space too large");
    if (!std::isfinite(g.r_in) || !std::isfinite(g.r_out) || !(g.r_out > g.r_in))
        return fail(RTT_EINVAL, os.str() + "need finite r_in < r_out");
    if (!std::isfinite(g.s0) || !std::isfinite(g.t0) || !std::isfinite(g.dt_obs) || !(g.dt_src > 0.0) ||
        !std::isfinite(g.dt_src))
        return fail(RTT_EINVAL, os.str() + "need finite t0, s0, dt_obs and dt_src > 0");
    if (g.n_frames > 1 && !(g.dt_obs > 0.0)) return fail(RTT_EINVAL, os.str() + "need dt_obs > 0");
    int32_t P, Q;
    if (!exact_ratio(g.dt_obs, g.dt_src, g.n_frames, &P, &Q))
        return fail(RTT_EINVAL, os.str() + "dt_obs/dt_src must be a rational P/Q with Q <= 64, P <= 4096");
    if ((int64_t)(g.n_frames - 1) * P > (1 << 30))
        return fail(RTT_EINVAL, os.str() + "n_frames * P too large");
    return RTT_OK;
}

}  // namespace rtt

using namespace rtt;

// device memory of a handle (tables and the solver workspace)
static void release_tables(rtt_geometry* h)
{
    if (h->d_rays) hipFree(h->d_rays);
    if (h->d_cell_start) hipFree(h->d_cell_start);
    if (h->d_visits) hipFree(h->d_visits);
    if (h->d_vtask) hipFree(h->d_vtask);
    if (h->d_fwd) hipFree(h->d_fwd);
    if (h->d_fwd_row) hipFree(h->d_fwd_row);
    if (h->d_seg) hipFree(h->d_seg);
    delete h->solve_ws;
    h->d_rays = nullptr;
    h->solve_ws = nullptr;
}

extern "C" int geometry_load(const rtt_grid* grids, const rtt_raymap* maps, int32_t n_geometries,
                             const rtt_load_opts* opts, rtt_geometry** out)
{
    if (!out) return fail(RTT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grids || !maps) return fail(RTT_EINVAL, "grids/maps is NULL");
    if (n_geometries < 1 || n_geometries > 4096) return fail(RTT_EINVAL, "n_geometries must be 1..4096");
    const double sigma = (opts && opts->sigma_omega > 0.0) ? opts->sigma_omega : 1.0;
    const bool drop_invalid = opts && opts->drop_invalid;
    if (opts && !(opts->sigma_omega >= 0.0)) return fail(RTT_EINVAL, "sigma_omega must be >= 0");

    std::vector<Member> members(n_geometries);
    std::vector<std::vector<double>> dir_delay(n_geometries), dir_weight(n_geometries);
    std::vector<RayRec> recs;
    std::vector<int32_t> cstart;
    std::vector<Visit> visits;
    std::vector<int64_t> vtask;
    std::vector<FwdRec> fwd, fwd_row;
    int64_t row_off = 0, col_off = 0, map_idx = 0;
    const double two_pi = 6.283185307179586476925286766559;

    for (int gi = 0; gi < n_geometries; ++gi) {
        const rtt_grid& g = grids[gi];
        int rc = check_grid(g, gi);
        if (rc) return rc;
        Member& m = members[gi];
        std::memset(&m, 0, sizeof(m));
        m.grid = g;
        for (int n = 0; n < 8; ++n) {
            m.delay_min[n] = HUGE_VAL;
            m.delay_max[n] = -HUGE_VAL;
        }
        exact_ratio(g.dt_obs, g.dt_src, g.n_frames, &m.P, &m.Q);
        const double dr = (g.r_out - g.r_in) / g.n_r;
        const double dphi = two_pi / g.n_phi;
        const int64_t n_cells = (int64_t)g.n_r * g.n_phi;

        std::vector<RayRec> gr;
        int64_t caller = 0;
        for (int n = 0; n < g.n_orders; ++n, ++map_idx) {
            const rtt_raymap& rm = maps[map_idx];
            if (rm.n_rays < 0 || rm.n_rays > (1ll << 30)) return fail(RTT_EINVAL, "n_rays out of range");
            if (rm.n_rays > 0 && (!rm.r_src || !rm.phi_src || !rm.delay || !rm.weight))
                return fail(RTT_EINVAL, "ray map array is NULL");
            m.rays_per_order[n] = rm.n_rays;
            for (int64_t p = 0; p < rm.n_rays; ++p, ++caller) {
                double r = rm.r_src[p], phi = rm.phi_src[p], dl = rm.delay[p], w = rm.weight[p];
                if (!std::isfinite(r) || !std::isfinite(phi) || !std::isfinite(dl) || !std::isfinite(w)) {
                    std::ostringstream os;
                    os << "geometry " << gi << " order " << n << " ray " << p << ": non-finite value";
                    return fail(RTT_EINVAL, os.str());
                }
                if (rm.pixel_area) {
                    double a = rm.pixel_area[p];
                    if (!(a >= 0.0) || !std::isfinite(a)) return fail(RTT_EINVAL, "pixel_area must be finite and >= 0");
                    w *= std::sqrt(a) / sigma;
                }
                if (r < g.r_in || r > g.r_out) {
                    if (!drop_invalid) {
                        std::ostringstream os;
                        os << "geometry " << gi << " order " << n << " ray " << p << ": r_src=" << r
                           << " outside [r_in, r_out]";
                        return fail(RTT_EINVAL, os.str());
                    }
                    w = 0.0;  // chi = 0: the row is kept and reads as zero
                    r = std::min(std::max(r, g.r_in), g.r_out);
                }
                if (w != 0.0) {
                    m.delay_min[n] = std::min(m.delay_min[n], dl);
                    m.delay_max[n] = std::max(m.delay_max[n], dl);
                    if (n == 0) {
                        dir_delay[gi].push_back(dl);
                        dir_weight[gi].push_back(std::fabs(w));
                    }
                }
                // bilinear stencil on cell centres (uniform in r, periodic in phi)
                double ur = (r - g.r_in) / dr - 0.5;
                ur = std::min(std::max(ur, 0.0), (double)(g.n_r - 1));
                int i = std::min((int)std::floor(ur), g.n_r - 2);
                double fr = ur - i;
                double pf = std::fmod(phi, two_pi);
                if (pf < 0.0) pf += two_pi;
                double up = pf / dphi - 0.5;
                double jf = std::floor(up);
                double fp = up - jf;
                int j0 = (int)(((int64_t)jf % g.n_phi + g.n_phi) % g.n_phi);
                // hat origin of frame 0
                double u0 = (g.t0 - dl - g.s0) / g.dt_src;
                double k0 = std::floor(u0);
                if (std::fabs(k0) > (double)(1 << 29)) return fail(RTT_EINVAL, "delay too far from the hat window");
                RayRec rr;
                rr.cell = i * g.n_phi + j0;
                rr.fr = (float)fr;
                rr.fphi = (float)fp;
                rr.w = (float)w;
                rr.k0 = (int32_t)k0;
                rr.th0 = (float)(u0 - k0);
                rr.row = (int32_t)caller;
                rr.order = n;
                gr.push_back(rr);
            }
        }
        // sort by base cell (stable: keeps (order, caller) order inside a cell)
        std::stable_sort(gr.begin(), gr.end(), [](const RayRec& a, const RayRec& b) { return a.cell < b.cell; });
        m.ray_begin = (int64_t)recs.size();
        m.n_rays = (int64_t)gr.size();
        m.cell_begin = (int64_t)cstart.size();
        std::vector<int32_t> cs(n_cells + 1, 0);
        for (const RayRec& rr : gr) cs[rr.cell + 1]++;
        for (int64_t c = 0; c < n_cells; ++c) cs[c + 1] += cs[c];
        // visit lists: for cell row ci and segment sg (columns [jlo, jhi)), sweep the base
        // columns u = jlo-1 .. jhi-1; rays with base row ci-1 feed row ci with radial weight fr,
        // rays with base row ci with 1 - fr; azimuthal weights (1-fphi) -> column u, fphi -> u+1.
        // segment widths: set 0 uses 16 columns; set 1 the widest of 16/8/4 columns that still
        // gives >= 2048 (row, segment) tasks for a single vector
        int narrow = VISIT_SEG_MAX;
        while (narrow > 4 && (int64_t)g.n_r * ((g.n_phi + narrow - 1) / narrow) < 2048) narrow /= 2;
        for (int set = 0; set < 2; ++set) {
            const int vseg = set == 0 ? VISIT_SEG_MAX : narrow;
            const int nseg = (g.n_phi + vseg - 1) / vseg;
            m.nseg[set] = nseg;
            m.vseg[set] = vseg;
            m.visit_begin[set] = (int64_t)visits.size();
            m.vtask_begin[set] = (int64_t)vtask.size();
            for (int ci = 0; ci < g.n_r; ++ci) {
                for (int sg = 0; sg < nseg; ++sg) {
                    vtask.push_back((int64_t)visits.size() - m.visit_begin[set]);
                    const int jlo = sg * vseg, jhi = std::min(jlo + vseg, g.n_phi);
                    for (int c = 0; c <= jhi - jlo; ++c) {
                        const int u = jlo - 1 + c;
                        const int ub = ((u % g.n_phi) + g.n_phi) % g.n_phi;
                        for (int part = 0; part < 2; ++part) {
                            const int ib = part == 0 ? ci - 1 : ci;
                            if (ib < 0 || ib > g.n_r - 2) continue;
                            const int64_t cell = (int64_t)ib * g.n_phi + ub;
                            for (int32_t q = cs[cell]; q < cs[cell + 1]; ++q) {
                                const RayRec& rr = gr[q];
                                const double wr = part == 0 ? (double)rr.fr : 1.0 - (double)rr.fr;
                                Visit v;
                                v.row = rr.row;
                                v.k0 = rr.k0;
                                v.th0 = rr.th0;
                                v.wa = (float)((double)rr.w * wr * (1.0 - (double)rr.fphi));
                                v.wb = (float)((double)rr.w * wr * (double)rr.fphi);
                                v.col = c;
                                v.order = rr.order;
                                v.pad = 0;
                                visits.push_back(v);
                            }
                        }
                    }
                }
            }
            vtask.push_back((int64_t)visits.size() - m.visit_begin[set]);
        }
        // set 2: the same sweep for a pair of rows (2p, 2p+1): a ray with base row ib feeds rows ib
        // (1 - fr) and ib + 1 (fr); within a column the order is by base row, so each row sums its
        // rays in the order of the single-row lists
        {
            const int vseg = VISIT_SEG_MAX;
            const int nseg = (g.n_phi + vseg - 1) / vseg;
            const int npair = (g.n_r + 1) / 2;
            m.nseg[2] = nseg;
            m.vseg[2] = vseg;
            m.visit_begin[2] = (int64_t)visits.size();
            m.vtask_begin[2] = (int64_t)vtask.size();
            for (int pi = 0; pi < npair; ++pi) {
                for (int sg = 0; sg < nseg; ++sg) {
                    vtask.push_back((int64_t)visits.size() - m.visit_begin[2]);
                    const int jlo = sg * vseg, jhi = std::min(jlo + vseg, g.n_phi);
                    for (int c = 0; c <= jhi - jlo; ++c) {
                        const int u = jlo - 1 + c;
                        const int ub = ((u % g.n_phi) + g.n_phi) % g.n_phi;
                        for (int part = 0; part <= 2; ++part) {
                            const int ib = 2 * pi - 1 + part;   // base row; local rows part-1, part
                            if (ib < 0 || ib > g.n_r - 2) continue;
                            const int64_t cell = (int64_t)ib * g.n_phi + ub;
                            for (int32_t q = cs[cell]; q < cs[cell + 1]; ++q) {
                                const RayRec& rr = gr[q];
                                float wts[4];
                                for (int lr = 0; lr < 2; ++lr) {
                                    const double wr = lr == part ? (double)rr.fr : lr == part - 1 ? 1.0 - (double)rr.fr : 0.0;
                                    wts[2 * lr] = (float)((double)rr.w * wr * (1.0 - (double)rr.fphi));
                                    wts[2 * lr + 1] = (float)((double)rr.w * wr * (double)rr.fphi);
                                }
                                VisitHead h;
                                h.row = rr.row;
                                h.k0 = rr.k0;
                                h.th0 = rr.th0;
                                h.col_order = c | (rr.order << 16);
                                Visit raw;
                                std::memcpy(&raw, &h, sizeof h);
                                std::memcpy((char*)&raw + sizeof h, wts, sizeof wts);
                                visits.push_back(raw);
                            }
                        }
                    }
                }
            }
            vtask.push_back((int64_t)visits.size() - m.visit_begin[2]);
        }
        // set 3: the rays of one base row ib only, swept in column order, each record carrying its
        // weights into row ib (1 - fr) and row ib + 1 (fr).  A task covers columns [jlo, jhi) of a
        // base row and reads the rays of base columns jlo - 1 .. jhi - 1 (the first one feeds column
        // jlo only); columns are added to a task while its visits stay within BR_VISITS (and at most
        // VISIT_SEG_MAX columns), so tasks carry about equal work.  Every column of every row
        // belongs to one task (rows without rays too: their tasks write zeros).
        {
            constexpr int64_t BR_VISITS = 40;
            m.visit_begin[3] = (int64_t)visits.size();
            auto rays_at = [&](int ib, int u) -> int64_t {
                if (ib > g.n_r - 2) return 0;   // no ray has its base cell in the last row
                const int ub = ((u % g.n_phi) + g.n_phi) % g.n_phi;
                const int64_t cell = (int64_t)ib * g.n_phi + ub;
                return cs[cell + 1] - cs[cell];
            };
            for (int par = 0; par < 2; ++par) {
                std::vector<int64_t> offs, desc;
                for (int ib = par; ib < g.n_r; ib += 2) {
                    int jlo = 0;
                    while (jlo < g.n_phi) {
                        int64_t nv = rays_at(ib, jlo - 1) + rays_at(ib, jlo);
                        int jhi = jlo + 1;
                        while (jhi < g.n_phi && jhi - jlo < VISIT_SEG_MAX && nv + rays_at(ib, jhi) <= BR_VISITS) {
                            nv += rays_at(ib, jhi);
                            ++jhi;
                        }
                        offs.push_back((int64_t)visits.size() - m.visit_begin[3]);
                        desc.push_back(((int64_t)ib * g.n_phi + jlo) | ((int64_t)(jhi - jlo) << 32));
                        for (int c = 0; c <= jhi - jlo && ib <= g.n_r - 2; ++c) {
                            const int u = jlo - 1 + c;
                            const int ub = ((u % g.n_phi) + g.n_phi) % g.n_phi;
                            const int64_t cell = (int64_t)ib * g.n_phi + ub;
                            for (int32_t q = cs[cell]; q < cs[cell + 1]; ++q) {
                                const RayRec& rr = gr[q];
                                float wts[4];
                                for (int lr = 0; lr < 2; ++lr) {
                                    const double wr = lr == 0 ? 1.0 - (double)rr.fr : (double)rr.fr;
                                    wts[2 * lr] = (float)((double)rr.w * wr * (1.0 - (double)rr.fphi));
                                    wts[2 * lr + 1] = (float)((double)rr.w * wr * (double)rr.fphi);
                                }
                                VisitHead h;
                                h.row = rr.row;
                                h.k0 = rr.k0;
                                h.th0 = rr.th0;
                                h.col_order = c | (rr.order << 16);
                                Visit raw;
                                std::memcpy(&raw, &h, sizeof h);
                                std::memcpy((char*)&raw + sizeof h, wts, sizeof wts);
                                visits.push_back(raw);
                            }
                        }
                        jlo = jhi;
                    }
                }
                offs.push_back((int64_t)visits.size() - m.visit_begin[3]);
                m.br_task_begin[par] = (int64_t)vtask.size();
                m.br_ntask[par] = (int64_t)desc.size();
                vtask.insert(vtask.end(), offs.begin(), offs.end());
                vtask.insert(vtask.end(), desc.begin(), desc.end());
            }
        }
        for (const RayRec& rr : gr) {
            const int i = rr.cell / g.n_phi, j0 = rr.cell % g.n_phi;
            const int j1 = (j0 + 1 == g.n_phi) ? 0 : j0 + 1;
            FwdRec f;
            f.c00k = rr.cell * g.n_hat;
            f.d01k = (j1 - j0) * g.n_hat;
            const double fr = rr.fr, fp = rr.fphi, w = rr.w;
            f.b00 = (float)(w * (1.0 - fr) * (1.0 - fp));
            f.b10 = (float)(w * fr * (1.0 - fp));
            f.b01 = (float)(w * (1.0 - fr) * fp);
            f.b11 = (float)(w * fr * fp);
            f.k0 = rr.k0;
            f.th0 = rr.th0;
            f.row = rr.row;
            f.order = rr.order;
            f.cell = rr.cell;
            f.pad1 = 0;
            fwd.push_back(f);
            (void)i;
        }
        // the same records in data-row order: consecutive records write adjacent rows, so the
        // cache lines two rows share are written together
        {
            const size_t b0 = fwd.size() - gr.size();
            std::vector<FwdRec> byrow(fwd.begin() + b0, fwd.end());
            std::stable_sort(byrow.begin(), byrow.end(), [](const FwdRec& a, const FwdRec& b) { return a.row < b.row; });
            fwd_row.insert(fwd_row.end(), byrow.begin(), byrow.end());
        }
        m.k0_min = m.k0_max = 0;
        for (size_t r = 0; r < gr.size(); ++r) {
            m.k0_min = r ? std::min(m.k0_min, gr[r].k0) : gr[r].k0;
            m.k0_max = r ? std::max(m.k0_max, gr[r].k0) : gr[r].k0;
        }
        cstart.insert(cstart.end(), cs.begin(), cs.end());
        recs.insert(recs.end(), gr.begin(), gr.end());
        m.n_rows = m.n_rays * g.n_frames;
        m.n_cols = n_cells * g.n_hat;
        m.row_offset = row_off;
        m.col_offset = col_off;
        row_off += m.n_rows;
        col_off += m.n_cols;
        m.adj_variant = default_adjoint_variant(m);
        m.apply_variant = default_apply_variant(m);
        m.digest = fnv1a(&g, sizeof(g));
        m.digest = fnv1a(gr.data(), gr.size() * sizeof(RayRec), m.digest);
    }
    if (recs.empty()) return fail(RTT_EINVAL, "no rays");

    rtt_geometry* h = new (std::nothrow) rtt_geometry();
    if (!h) return fail(RTT_ENOMEM, "host allocation failed");
    h->members = std::move(members);
    h->dir_delay = std::move(dir_delay);
    h->dir_weight = std::move(dir_weight);
    h->n_rows = row_off;
    h->n_cols = col_off;
    h->n_rays = (int64_t)recs.size();
    hipGetDevice(&h->device);
    size_t rb = recs.size() * sizeof(RayRec), cb = cstart.size() * sizeof(int32_t);
    size_t vb = std::max<size_t>(visits.size(), 1) * sizeof(Visit), tb = vtask.size() * sizeof(int64_t);
    hipError_t e = hipMalloc((void**)&h->d_rays, rb);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_cell_start, cb);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_visits, vb);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_vtask, tb);
    const size_t fb = fwd.size() * sizeof(FwdRec);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_fwd, fb);
    if (e == hipSuccess) e = hipMemcpy(h->d_fwd, fwd.data(), fb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_fwd_row, fb);
    if (e == hipSuccess) e = hipMemcpy(h->d_fwd_row, fwd_row.data(), fb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_rays, recs.data(), rb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_cell_start, cstart.data(), cb, hipMemcpyHostToDevice);
    if (e == hipSuccess && !visits.empty())
        e = hipMemcpy(h->d_visits, visits.data(), visits.size() * sizeof(Visit), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_vtask, vtask.data(), tb, hipMemcpyHostToDevice);
    // (offset, length) of every member's column and row block, for per-member reductions
    std::vector<int64_t> seg;
    for (const Member& m : h->members) seg.insert(seg.end(), {m.col_offset, m.n_cols});
    for (const Member& m : h->members) seg.insert(seg.end(), {m.row_offset, m.n_rows});
    const size_t sb = seg.size() * sizeof(int64_t);
    if (e == hipSuccess) e = hipMalloc((void**)&h->d_seg, sb);
    if (e == hipSuccess) e = hipMemcpy(h->d_seg, seg.data(), sb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "geometry_load upload");
        release_tables(h);
        delete h;
        return rc;
    }
    h->table_bytes = (int64_t)(rb + cb + vb + tb + 2 * fb + sb);
    *out = h;
    return RTT_OK;
}

extern "C" int geometry_free(rtt_geometry* g)
{
    if (!g) return RTT_OK;
    if (g->magic != 0x52545447u) return fail(RTT_ESTATE, "not a geometry handle");
    release_tables(g);
    g->magic = 0;
    delete g;
    return RTT_OK;
}

extern "C" int geometry_info(const rtt_geometry* g, rtt_geometry_info* info)
{
    if (!valid_handle(g) || !info) return fail(RTT_EINVAL, "bad handle or info");
    info->n_geometries = (int32_t)g->members.size();
    info->n_rows = g->n_rows;
    info->n_cols = g->n_cols;
    info->n_rays = g->n_rays;
    info->table_bytes = g->table_bytes;
    info->batch_apply_mode = g->batch_apply_mode;
    info->batch_adjoint_mode = g->batch_adjoint_mode;
    info->apply_launches = whole_operator_launches(g, false);
    info->adjoint_launches = whole_operator_launches(g, true);
    return RTT_OK;
}

extern "C" int geometry_set_batch_mode(rtt_geometry* g, int32_t apply_mode, int32_t adjoint_mode)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (apply_mode < -1 || apply_mode > 2 || adjoint_mode < -1 || adjoint_mode > 2)
        return fail(RTT_EINVAL, "launch mode must be -1 (unchanged), 0, 1 or 2");
    if (apply_mode >= 0) g->batch_apply_mode = apply_mode;
    if (adjoint_mode >= 0) g->batch_adjoint_mode = adjoint_mode;
    return RTT_OK;
}

extern "C" int geometry_member(const rtt_geometry* g, int32_t idx, rtt_member_info* info)
{
    if (!valid_handle(g) || !info) return fail(RTT_EINVAL, "bad handle or info");
    if (idx < 0 || idx >= (int32_t)g->members.size()) return fail(RTT_EINVAL, "member index out of range");
    const Member& m = g->members[idx];
    info->grid = m.grid;
    info->row_offset = m.row_offset;
    info->n_rows = m.n_rows;
    info->col_offset = m.col_offset;
    info->n_cols = m.n_cols;
    for (int n = 0; n < 8; ++n) info->rays_per_order[n] = m.rays_per_order[n];
    info->apply_variant = m.apply_variant;
    info->adjoint_variant = m.adj_variant;
    info->digest = m.digest;
    return RTT_OK;
}

extern "C" int geometry_set_variant(rtt_geometry* g, int32_t idx, int32_t apply_variant, int32_t adjoint_variant)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (idx < -1 || idx >= (int32_t)g->members.size()) return fail(RTT_EINVAL, "member index out of range");
    if (apply_variant < -1 || apply_variant >= n_apply_variants()) return fail(RTT_EINVAL, "unknown apply variant");
    if (adjoint_variant < -1 || adjoint_variant >= n_adjoint_variants())
        return fail(RTT_EINVAL, "unknown adjoint variant");
    for (int i = 0; i < (int)g->members.size(); ++i) {
        if (idx >= 0 && i != idx) continue;
        Member& m = g->members[i];
        if ((apply_variant == 2 || apply_variant == 3) && m.P > m.Q)
            return fail(RTT_EINVAL, "batch/stream forward variants need dt_obs <= dt_src");
        if (apply_variant >= 0 && !apply_variant_ok(m, apply_variant))
            return fail(RTT_EINVAL, "lean/reg/strip/abs forward variants need dt_obs/dt_src = 1 or 1/2 "
                                    "(lean4q: n_hat a multiple of 4; abs: n_hat <= 128)");
        if (apply_variant >= 0) m.apply_variant = apply_variant;
        if (adjoint_variant >= 0 && !adjoint_variant_ok(m, adjoint_variant))
            return fail(RTT_EINVAL, "visit/rows adjoint variants need dt_obs/dt_src = 1 or 1/2 (rows: n_hat <= 256)");
        if (adjoint_variant >= 0) m.adj_variant = adjoint_variant;
    }
    return RTT_OK;
}

extern "C" const char* variant_name(int32_t adjoint, int32_t v)
{
    if (adjoint) return (v >= 0 && v < n_adjoint_variants()) ? adjoint_variant_name(v) : nullptr;
    return (v >= 0 && v < n_apply_variants()) ? apply_variant_name(v) : nullptr;
}

extern "C" const char* last_error(void) { return g_err.c_str(); }
