// Autotuner: pick the fastest kernel variant of A and A^T for each member geometry.
//
// Every applicable variant is timed with HIP events on the caller's stream
// over `reps` launches on `nvec` random vectors (median).  Choices are cached
// in a plain text file, one line "digest nvec apply adjoint" per entry, where
// digest is the member's FNV-1a content hash.
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
};

std::vector<CacheEntry> read_cache(const char* path)
{
    std::vector<CacheEntry> out;
    if (!path) return out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        CacheEntry e;
        if (is >> std::hex >> e.digest >> std::dec >> e.nvec >> e.apply >> e.adjoint) out.push_back(e);
    }
    return out;
}

int time_variant(const rtt_geometry* g, const Member& m, bool adjoint, int variant, const float* in, float* out,
                 int nvec, int reps, hipStream_t s, float* ms_out)
{
    hipEvent_t e0, e1;
    RTT_HIP(hipEventCreate(&e0));
    RTT_HIP(hipEventCreate(&e1));
    std::vector<float> t;
    const uint32_t mask = effective_mask(m, 0);
    for (int r = 0; r <= reps; ++r) {
        RTT_HIP(hipEventRecord(e0, s));
        int rc = adjoint ? launch_adjoint(g, m, in, out, nvec, m.n_rows, m.n_cols, mask, s, variant)
                         : launch_apply(g, m, in, out, nvec, m.n_cols, m.n_rows, mask, s, variant);
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
    std::vector<CacheEntry> cache = read_cache(cache_path);
    int64_t max_rows = 0, max_cols = 0;
    for (const Member& m : g->members) {
        max_rows = std::max(max_rows, m.n_rows);
        max_cols = std::max(max_cols, m.n_cols);
    }
    Workspace ws;
    float* xb = nullptr;
    float* yb = nullptr;
    std::vector<CacheEntry> added;
    for (Member& m : g->members) {
        bool hit = false;
        for (const CacheEntry& e : cache)
            if (e.digest == m.digest && e.nvec == nvec && e.apply >= 0 && e.apply < n_apply_variants() &&
                e.adjoint >= 0 && e.adjoint < n_adjoint_variants() && !((e.apply == 2 || e.apply == 3) && m.P > m.Q) &&
                !((e.apply == 4 || e.apply == 5) && !lean_supported(m))) {
                m.apply_variant = e.apply;
                m.adj_variant = e.adjoint;
                hit = true;
            }
        if (hit) continue;
        if (!xb) {
            xb = (float*)ws.get("tune_x", sizeof(float) * (size_t)nvec * max_cols);
            yb = (float*)ws.get("tune_y", sizeof(float) * (size_t)nvec * max_rows);
            if (!xb || !yb) return fail(RTT_ENOMEM, "tune buffers");
            int rc = normal_fill(xb, (int64_t)nvec * max_cols, 12345, s);
            if (!rc) rc = normal_fill(yb, (int64_t)nvec * max_rows, 54321, s);
            if (rc) return rc;
        }
        float best = 1e30f;
        int best_v = m.apply_variant;
        for (int v = 0; v < n_apply_variants(); ++v) {
            if ((v == 2 || v == 3) && m.P > m.Q) continue;
            if ((v == 4 || v == 5) && !lean_supported(m)) continue;
            float ms;
            int rc = time_variant(g, m, false, v, xb, yb, nvec, reps, s, &ms);
            if (rc) return rc;
            if (std::getenv("RTT_LOG")) std::fprintf(stderr, "[rtt] tune apply %s: %.4f ms\n", apply_variant_name(v), ms);
            if (ms < best) { best = ms; best_v = v; }
        }
        m.apply_variant = best_v;
        best = 1e30f;
        best_v = m.adj_variant;
        for (int v = 0; v < n_adjoint_variants(); ++v) {
            if (v == 11 && !visit_supported(m)) continue;
            float ms;
            int rc = time_variant(g, m, true, v, yb, xb, nvec, reps, s, &ms);
            if (rc) return rc;
            if (std::getenv("RTT_LOG")) std::fprintf(stderr, "[rtt] tune adjoint %s: %.4f ms\n", adjoint_variant_name(v), ms);
            if (ms < best) { best = ms; best_v = v; }
        }
        m.adj_variant = best_v;
        added.push_back({m.digest, nvec, m.apply_variant, m.adj_variant});
    }
    if (cache_path && !added.empty()) {
        std::ofstream f(cache_path, std::ios::app);
        for (const CacheEntry& e : added)
            f << std::hex << e.digest << std::dec << " " << e.nvec << " " << e.apply << " " << e.adjoint << "\n";
    }
    RTT_HIP(hipStreamSynchronize(s));
    return RTT_OK;
}
