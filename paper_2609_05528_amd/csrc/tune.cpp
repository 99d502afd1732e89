// Autotuner: pick the fastest kernel variant of A and A^T for each member geometry and, for a
// handle with several members, the fastest way to launch the whole operator: the per-member
// choices one launch per member, or one variant shared by all members in one launch (plain or
// persistent).
//
// Every applicable variant is timed with HIP events on the caller's stream
// over `reps` launches on `nvec` random vectors (median), each member at its place in the handle's
// data layout.  Choices are cached in a plain text file, one line "digest nvec apply adjoint" per
// entry, where digest is the member's FNV-1a content hash combined with that place.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "dense.h"

using namespace rtt;

namespace {

struct CacheEntry {
    uint64_t digest;
    int nvec, apply, adjoint;
    int uni_apply = -1, uni_adjoint = -1;   // multi lines: variant shared by every member, or -1
};

// Member lines are "digest nvec apply adjoint"; whole-handle lines (handles with several
// members) are "multi digest nvec apply_mode adjoint_mode apply_shared adjoint_shared", where a
// shared variant (or -1) replaces every member's own choice.
std::vector<CacheEntry> read_cache(const char* path, std::vector<CacheEntry>* multi)
{
    std::vector<CacheEntry> out;
    if (!path) return out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        CacheEntry e;
        if (line.compare(0, 6, "multi ") == 0) {
            std::string tag;
            if (is >> tag >> std::hex >> e.digest >> std::dec >> e.nvec >> e.apply >> e.adjoint) {
                if (!(is >> e.uni_apply >> e.uni_adjoint)) e.uni_apply = e.uni_adjoint = -1;
                multi->push_back(e);
            }
            continue;
        }
        if (is >> std::hex >> e.digest >> std::dec >> e.nvec >> e.apply >> e.adjoint) out.push_back(e);
    }
    return out;
}

// Every member images the same source grid: the forward of such a handle is timed as
// op_apply_shared (one coefficient block per vector read by every member), its batched use.
bool shares_source_grid(const rtt_geometry* g)
{
    const rtt_grid& g0 = g->members[0].grid;
    for (const Member& m : g->members) {
        const rtt_grid& q = m.grid;
        if (q.n_r != g0.n_r || q.n_phi != g0.n_phi || q.n_hat != g0.n_hat || q.r_in != g0.r_in ||
            q.r_out != g0.r_out || q.s0 != g0.s0 || q.dt_src != g0.dt_src)
            return false;
    }
    return true;
}

// Median time of the whole-operator call under launch mode `mode` (see rtt_geometry).
int time_mode(rtt_geometry* g, bool adjoint, int mode, const float* in, float* out, int nvec, int reps,
              hipStream_t s, float* ms_out)
{
    const bool shared = !adjoint && shares_source_grid(g);
    int32_t& slot = adjoint ? g->batch_adjoint_mode : g->batch_apply_mode;
    const int32_t keep = slot;
    slot = mode;
    hipEvent_t e0, e1;
    RTT_HIP(hipEventCreate(&e0));
    RTT_HIP(hipEventCreate(&e1));
    std::vector<float> t;
    int rc = RTT_OK;
    for (int r = 0; r <= reps && !rc; ++r) {
        RTT_HIP(hipEventRecord(e0, s));
        rc = apply_op(g, -1, adjoint, in, out, nvec, 0u, s, shared);
        if (rc) break;
        RTT_HIP(hipEventRecord(e1, s));
        RTT_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RTT_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) t.push_back(ms);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    slot = keep;
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return RTT_OK;
}

// A member's place in the handle's data layout: in a handle with several members its rows start at
// its row offset in every vector of [nvec][n_rows], so the 128-byte phase of its row block (which
// decides how many partly written lines its row stores leave, up to twice the time of the same
// kernel on line-aligned rows) is set by the row offset and the handle's row count.
struct Place {
    int64_t row_offset, y_stride;
};
Place member_place(const rtt_geometry* g, const Member& m)
{
    if (g->members.size() > 1) return {m.row_offset, g->n_rows};
    return {0, m.n_rows};
}

// The cache key of a member: its content digest and the 128-byte phase of its place.
uint64_t place_digest(const rtt_geometry* g, const Member& m)
{
    const Place p = member_place(g, m);
    const int32_t ph[2] = {(int32_t)(p.row_offset % 32), (int32_t)(p.y_stride % 32)};
    return fnv1a(ph, sizeof(ph), m.digest);
}

// Median time of one variant of member m: x holds [nvec][m.n_cols] (the columns a member reads in
// the shared-grid call), y is the handle-layout buffer already offset to the member's rows.
int time_variant(const rtt_geometry* g, const Member& m, bool adjoint, int variant, float* x, float* y,
                 int64_t y_stride, int nvec, int reps, hipStream_t s, float* ms_out)
{
    hipEvent_t e0, e1;
    RTT_HIP(hipEventCreate(&e0));
    RTT_HIP(hipEventCreate(&e1));
    std::vector<float> t;
    const uint32_t mask = effective_mask(m, 0);
    for (int r = 0; r <= reps; ++r) {
        RTT_HIP(hipEventRecord(e0, s));
        int rc = adjoint ? launch_adjoint(g, m, y, x, nvec, y_stride, m.n_cols, mask, s, variant)
                         : launch_apply(g, m, x, y, nvec, m.n_cols, y_stride, mask, s, variant);
        if (rc) return rc;
        RTT_HIP(hipEventRecord(e1, s));
        RTT_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RTT_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) t.push_back(ms);   // first launch is a warm-up
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return RTT_OK;
}

}  // namespace

extern "C" int geometry_tune(rtt_geometry* g, int32_t nvec, int32_t reps, const char* cache_path, void* stream)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (nvec < 1 || nvec > 4096 || reps < 1 || reps > 1000) return fail(RTT_EINVAL, "need 1 <= nvec <= 4096, 1 <= reps <= 1000");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CacheEntry> multi_cache;
    std::vector<CacheEntry> cache = read_cache(cache_path, &multi_cache);
    int64_t max_cols = 0;
    for (const Member& m : g->members) max_cols = std::max(max_cols, m.n_cols);
    // rows of the per-member timing buffer: the handle's layout (every member at its place)
    const int64_t y_rows = g->members.size() > 1 ? g->n_rows : g->members[0].n_rows;
    Workspace ws;
    float* xb = nullptr;
    float* yb = nullptr;
    std::vector<CacheEntry> added;
    for (Member& m : g->members) {
        bool hit = false;
        const uint64_t key = place_digest(g, m);
        for (const CacheEntry& e : cache)
            if (e.digest == key && e.nvec == nvec && apply_variant_ok(m, e.apply) &&
                adjoint_variant_ok(m, e.adjoint)) {
                m.apply_variant = e.apply;
                m.adj_variant = e.adjoint;
                hit = true;
            }
        if (hit) continue;
        if (!xb) {
            xb = (float*)ws.get("tune_x", sizeof(float) * (size_t)nvec * max_cols);
            // a handle with several members times its whole-operator launch modes on a buffer of the
            // same shape below: both use one allocation
            yb = (float*)ws.get(g->members.size() > 1 ? "tune_ya" : "tune_y", sizeof(float) * (size_t)nvec * y_rows);
            if (!xb || !yb) return fail(RTT_ENOMEM, "tune buffers");
            int rc = normal_fill(xb, (int64_t)nvec * max_cols, 12345, s);
            if (!rc) rc = normal_fill(yb, (int64_t)nvec * y_rows, 54321, s);
            if (rc) return rc;
        }
        const Place pl = member_place(g, m);
        float* ym = yb + pl.row_offset;
        float best = 1e30f;
        int best_v = m.apply_variant;
        for (int v = 0; v < n_apply_variants(); ++v) {
            if (!apply_variant_ok(m, v)) continue;
            float ms;
            int rc = time_variant(g, m, false, v, xb, ym, pl.y_stride, nvec, reps, s, &ms);
            if (rc) return rc;
            if (std::getenv("RTT_LOG")) std::fprintf(stderr, "[rtt] tune apply %s: %.4f ms\n", apply_variant_name(v), ms);
            if (ms < best) { best = ms; best_v = v; }
        }
        m.apply_variant = best_v;
        best = 1e30f;
        best_v = m.adj_variant;
        for (int v = 0; v < n_adjoint_variants(); ++v) {
            if (!adjoint_variant_ok(m, v)) continue;
            float ms;
            int rc = time_variant(g, m, true, v, xb, ym, pl.y_stride, nvec, reps, s, &ms);
            if (rc) return rc;
            if (std::getenv("RTT_LOG")) std::fprintf(stderr, "[rtt] tune adjoint %s: %.4f ms\n", adjoint_variant_name(v), ms);
            if (ms < best) { best = ms; best_v = v; }
        }
        m.adj_variant = best_v;
        added.push_back({key, nvec, m.apply_variant, m.adj_variant});
    }
    // several members: the per-member choices launched one by one, or one variant shared by every
    // member (the ones with a single-launch form) launched as one launch or one persistent launch
    bool multi_added = false;
    uint64_t hd = 1469598103934665603ull;
    int uni[2] = {-1, -1};   // variant given to every member (-1: keep the per-member choices)
    if (g->members.size() > 1) {
        for (const Member& m : g->members) {
            const int32_t v[2] = {m.apply_variant, m.adj_variant};
            hd = fnv1a(&m.digest, sizeof(m.digest), hd);
            hd = fnv1a(v, sizeof(v), hd);
        }
        bool hit = false;
        for (const CacheEntry& e : multi_cache)
            if (e.digest == hd && e.nvec == nvec && e.apply >= 0 && e.apply <= 2 && e.adjoint >= 0 && e.adjoint <= 2) {
                g->batch_apply_mode = e.apply;
                g->batch_adjoint_mode = e.adjoint;
                uni[0] = e.uni_apply;
                uni[1] = e.uni_adjoint;
                hit = true;
            }
        if (hit) {
            for (Member& m : g->members) {
                if (uni[0] >= 0 && apply_variant_ok(m, uni[0])) m.apply_variant = uni[0];
                if (uni[1] >= 0 && adjoint_variant_ok(m, uni[1])) m.adj_variant = uni[1];
            }
        } else {
            float* xa = (float*)ws.get("tune_xa", sizeof(float) * (size_t)nvec * g->n_cols);
            float* ya = (float*)ws.get("tune_ya", sizeof(float) * (size_t)nvec * g->n_rows);
            if (!xa || !ya) return fail(RTT_ENOMEM, "tune buffers");
            int rc = normal_fill(xa, (int64_t)nvec * g->n_cols, 12345, s);
            if (!rc) rc = normal_fill(ya, (int64_t)nvec * g->n_rows, 54321, s);
            if (rc) return rc;
            for (int adj = 0; adj < 2; ++adj) {
                std::vector<int32_t> tuned;
                for (const Member& m : g->members) tuned.push_back(adj ? m.adj_variant : m.apply_variant);
                // candidates: -1 = the per-member choices; then the single-launch variants
                std::vector<int> cands = {-1};
                for (int v : adj ? std::vector<int>{11, 16, 19, 20} : std::vector<int>{4, 6, 7, 11, 13}) {
                    bool ok = true;
                    for (const Member& m : g->members) ok = ok && (adj ? adjoint_variant_ok(m, v) : apply_variant_ok(m, v));
                    if (ok) cands.push_back(v);
                }
                float best = 1e30f;
                int best_m = 0, best_u = -1;
                for (int u : cands) {
                    for (size_t i = 0; i < g->members.size(); ++i) {
                        int32_t& slot = adj ? g->members[i].adj_variant : g->members[i].apply_variant;
                        slot = u >= 0 ? u : tuned[i];
                    }
                    for (int mode = 0; mode <= 2; ++mode) {
                        // a shared variant is timed in every mode: launched per member (mode 0) it can beat
                        // the per-member choices, each timed alone with noise at small sizes
                        float ms;
                        rc = adj ? time_mode(g, true, mode, ya, xa, nvec, reps, s, &ms)
                                 : time_mode(g, false, mode, xa, ya, nvec, reps, s, &ms);
                        if (rc) return rc;
                        if (std::getenv("RTT_LOG"))
                            std::fprintf(stderr, "[rtt] tune %s shared variant %d launch mode %d: %.4f ms\n",
                                         adj ? "adjoint" : "apply", u, mode, ms);
                        if (ms < best) {
                            best = ms;
                            best_m = mode;
                            best_u = u;
                        }
                    }
                }
                for (size_t i = 0; i < g->members.size(); ++i) {
                    int32_t& slot = adj ? g->members[i].adj_variant : g->members[i].apply_variant;
                    slot = best_u >= 0 ? best_u : tuned[i];
                }
                (adj ? g->batch_adjoint_mode : g->batch_apply_mode) = best_m;
                uni[adj] = best_u;
            }
            multi_added = true;
        }
    }
    if (cache_path && (!added.empty() || multi_added)) {
        std::ofstream f(cache_path, std::ios::app);
        for (const CacheEntry& e : added)
            f << std::hex << e.digest << std::dec << " " << e.nvec << " " << e.apply << " " << e.adjoint << "\n";
        if (multi_added)
            f << "multi " << std::hex << hd << std::dec << " " << nvec << " " << g->batch_apply_mode << " "
              << g->batch_adjoint_mode << " " << uni[0] << " " << uni[1] << "\n";
    }
    RTT_HIP(hipStreamSynchronize(s));
    return RTT_OK;
}
