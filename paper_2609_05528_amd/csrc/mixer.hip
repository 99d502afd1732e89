// Order mixer L of Sec. 3.1, eq. (4): d_L = (L kron I) d_R on the rows of a handle -- the
// unresolved spatial image (rays of every order landing on one pixel added) and the total-flux
// readout (every ray added) -- its transpose, and the propagation of a diagonal data covariance
// C_L = (L kron I) C_R (L^T kron I).
//
// Tables (built on the host at mixer_create): the mixed rows are split into chunks of at most
// MIX_CHUNK source rays, each a run of consecutive entries of one mixed row's source list
// (source lists in data-row order).  A mixed row with one chunk is written directly; a longer
// one (the total flux) first writes one partial row per chunk and then adds the partial rows in
// chunk order, so every sum has a fixed order and the result is bitwise reproducible.
//
// Kernels: a wave owns one chunk (or one source ray for the transpose) of one vector, lanes
// over frames, so every access is a contiguous run of a data row.  HBM-bound (read the source
// rows once, write the mixed rows once).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rtt.h"
#include "rtt_internal.h"
#include "dense.h"

namespace rtt {
namespace {

constexpr int WAVE = 64;
constexpr int MIX_CHUNK = 64;     // source rays per chunk
constexpr int MIX_WAVES = 4;      // waves per block
constexpr int64_t MIX_MIN_WAVES = 32768;   // launch size below which fewer vectors go to a wave
constexpr uint32_t MIX_MAGIC = 0x4D495852u;

}  // namespace
}  // namespace rtt

struct rtt_mixer {
    int32_t kind = 0;
    int32_t n_geometries = 0;
    int64_t n_rows = 0;        // mixed rows (elements of one mixed data vector)
    int64_t n_src_rows = 0;    // rows of the handle's data vectors
    std::vector<int64_t> g_off, g_rows, g_out;   // per geometry: offset, elements, mixed rows (pixels or 1)
    int64_t n_chunks = 0, n_multi = 0, n_src = 0, n_slots = 0;
    int64_t pitch = 0;         // floats per partial slot (largest n_frames rounded up to 4)
    // frames words below hold F | (vector width 1, 2 or 4 that keeps every address aligned) << 32
    int64_t* d_chunk = nullptr;    // [n_chunks][4]: first list entry, entries, target (element offset of the
                                   // mixed row, or -1 - partial slot), frames word
    int64_t* d_list = nullptr;     // [n_src]: element offset of each source row, in chunk order
    int64_t* d_multi = nullptr;    // [n_multi][4]: mixed row offset, first entry of d_slots, slots, frames word
    int64_t* d_slots = nullptr;    // [n_slots]: element offset of each partial slot (slot * pitch)
    int64_t* d_src = nullptr;      // [n_src][4]: source row offset, mixed row offset, frames word, 0
    int32_t vb_apply = 0, vb_adjoint = 0;   // pinned vectors per wave (0: chosen per call)
    int device = 0;
    mutable rtt::Workspace ws;
    uint32_t magic = rtt::MIX_MAGIC;
};

namespace rtt {
namespace {

template <int VW> struct Vec;
template <> struct Vec<1> { typedef float type; };
template <> struct Vec<2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec<4> { typedef float type __attribute__((ext_vector_type(4))); };

// For nv <= VB vectors j (strides ys, os): out_j[f] = sum over the cnt rows y_j + lst[i], in list
// order, of row[f], f < F.  Lane l covers frames l*VW .. l*VW+VW-1 of every 64*VW-frame pass (F
// and every offset multiples of VW).  Rows are taken U at a time so that U * nv loads are in flight
// before they are added (still in list order).  FULL: nv == VB, no per-vector tests.
template <int VW, int VB, bool FULL>
__device__ __forceinline__ void sum_rows(const float* __restrict__ y, int64_t ys, int nv,
                                         const int64_t* __restrict__ lst, int64_t cnt, int64_t F,
                                         float* __restrict__ out, int64_t os, int lane)
{
    typedef typename Vec<VW>::type V;
    constexpr int U = VB >= 16 ? 1 : 16 / VB;
    for (int64_t f = (int64_t)lane * VW; f < F; f += WAVE * VW) {
        V acc[VB];
#pragma unroll
        for (int j = 0; j < VB; ++j) acc[j] = (V)(0.f);
        int64_t i = 0;
        for (; i + U <= cnt; i += U) {
            V t[U][VB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float* row = y + lst[i + u] + f;
#pragma unroll
                for (int j = 0; j < VB; ++j)
                    if (FULL || j < nv) t[u][j] = *(const V*)(row + j * ys);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < VB; ++j)
                    if (FULL || j < nv) acc[j] += t[u][j];
        }
        for (; i < cnt; ++i) {
            const float* row = y + lst[i] + f;
#pragma unroll
            for (int j = 0; j < VB; ++j)
                if (FULL || j < nv) acc[j] += *(const V*)(row + j * ys);
        }
#pragma unroll
        for (int j = 0; j < VB; ++j)
            if (FULL || j < nv) *(V*)(out + j * os + f) = acc[j];
    }
}

// out_j[f] = in_j[f], f < F, for nv <= VB vectors (VW as in sum_rows)
template <int VW, int VB, bool FULL>
__device__ __forceinline__ void copy_row(const float* __restrict__ in, int64_t is, int nv, int64_t F,
                                         float* __restrict__ out, int64_t os, int lane)
{
    typedef typename Vec<VW>::type V;
    for (int64_t f = (int64_t)lane * VW; f < F; f += WAVE * VW) {
        V t[VB];
#pragma unroll
        for (int j = 0; j < VB; ++j)
            if (FULL || j < nv) t[j] = *(const V*)(in + j * is + f);
#pragma unroll
        for (int j = 0; j < VB; ++j)
            if (FULL || j < nv) *(V*)(out + j * os + f) = t[j];
    }
}

template <int VB>
__device__ __forceinline__ void sum_rows_any(int vw, const float* y, int64_t ys, int nv, const int64_t* lst,
                                             int64_t cnt, int64_t F, float* out, int64_t os, int lane)
{
    if (nv == VB) {
        if (vw == 4)
            sum_rows<4, VB, true>(y, ys, nv, lst, cnt, F, out, os, lane);
        else if (vw == 2)
            sum_rows<2, VB, true>(y, ys, nv, lst, cnt, F, out, os, lane);
        else
            sum_rows<1, VB, true>(y, ys, nv, lst, cnt, F, out, os, lane);
    } else {
        if (vw == 4)
            sum_rows<4, VB, false>(y, ys, nv, lst, cnt, F, out, os, lane);
        else if (vw == 2)
            sum_rows<2, VB, false>(y, ys, nv, lst, cnt, F, out, os, lane);
        else
            sum_rows<1, VB, false>(y, ys, nv, lst, cnt, F, out, os, lane);
    }
}

template <int VB>
__device__ __forceinline__ void copy_row_any(int vw, const float* in, int64_t is, int nv, int64_t F, float* out,
                                             int64_t os, int lane)
{
    if (nv == VB) {
        if (vw == 4)
            copy_row<4, VB, true>(in, is, nv, F, out, os, lane);
        else if (vw == 2)
            copy_row<2, VB, true>(in, is, nv, F, out, os, lane);
        else
            copy_row<1, VB, true>(in, is, nv, F, out, os, lane);
    } else {
        if (vw == 4)
            copy_row<4, VB, false>(in, is, nv, F, out, os, lane);
        else if (vw == 2)
            copy_row<2, VB, false>(in, is, nv, F, out, os, lane);
        else
            copy_row<1, VB, false>(in, is, nv, F, out, os, lane);
    }
}

// one wave per (chunk, group of VB vectors): the chunk's source rows added in list order, written
// to the mixed row (single-chunk rows) or to the chunk's partial slot
template <int VB>
__global__ __launch_bounds__(MIX_WAVES * WAVE) void k_mix_chunks(const int64_t* __restrict__ chunk,
                                                                   const int64_t* __restrict__ list, int64_t n_chunks,
                                                                   const float* __restrict__ y, int64_t y_stride,
                                                                   float* __restrict__ d, int64_t d_stride,
                                                                   float* __restrict__ part, int64_t part_stride,
                                                                   int64_t pitch, int nvec, int vmax)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t c = (int64_t)blockIdx.x * MIX_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (c >= n_chunks) return;
    const int64_t v0 = (int64_t)blockIdx.y * VB;
    const int nv = min(VB, nvec - (int)v0);
    const int64_t* ch = chunk + 4 * c;
    const int64_t first = ch[0], cnt = ch[1], target = ch[2];
    const int64_t F = ch[3] & 0xffffffffll;
    const int vw = min((int)(ch[3] >> 32), vmax);
    const float* yv = y + v0 * y_stride;
    float* out;
    int64_t os;
    if (target >= 0) {
        out = d + v0 * d_stride + target;
        os = d_stride;
    } else {
        out = part + v0 * part_stride + (-1 - target) * pitch;
        os = part_stride;
    }
    sum_rows_any<VB>(vw, yv, y_stride, nv, list + first, cnt, F, out, os, lane);
}

// one wave per (multi-chunk row, group of VB vectors): the row = its partial rows added in
// chunk order
template <int VB>
__global__ __launch_bounds__(MIX_WAVES * WAVE) void k_mix_partials(const int64_t* __restrict__ multi,
                                                                     const int64_t* __restrict__ slots_off,
                                                                     int64_t n_multi, const float* __restrict__ part,
                                                                     int64_t part_stride, float* __restrict__ d,
                                                                     int64_t d_stride, int nvec, int vmax)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t r = (int64_t)blockIdx.x * MIX_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= n_multi) return;
    const int64_t v0 = (int64_t)blockIdx.y * VB;
    const int nv = min(VB, nvec - (int)v0);
    const int64_t* m = multi + 4 * r;
    const int64_t off = m[0], first = m[1], slots = m[2];
    const int64_t F = m[3] & 0xffffffffll;
    const int vw = min((int)(m[3] >> 32), vmax);
    const float* p = part + v0 * part_stride;
    float* out = d + v0 * d_stride + off;
    sum_rows_any<VB>(vw, p, part_stride, nv, slots_off + first, slots, F, out, d_stride, lane);
}

// one wave per (source ray, group of VB vectors): the ray's rows receive the mixed row it feeds
template <int VB>
__global__ __launch_bounds__(MIX_WAVES * WAVE) void k_mix_transpose(const int64_t* __restrict__ src, int64_t n_src,
                                                                      const float* __restrict__ d, int64_t d_stride,
                                                                      float* __restrict__ y, int64_t y_stride,
                                                                      int nvec, int vmax)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t r = (int64_t)blockIdx.x * MIX_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= n_src) return;
    const int64_t v0 = (int64_t)blockIdx.y * VB;
    const int nv = min(VB, nvec - (int)v0);
    const int64_t* e = src + 4 * r;
    const int64_t so = e[0], mo = e[1];
    const int64_t F = e[2] & 0xffffffffll;
    const int vw = min((int)(e[2] >> 32), vmax);
    const float* in = d + v0 * d_stride + mo;
    float* out = y + v0 * y_stride + so;
    copy_row_any<VB>(vw, in, d_stride, nv, F, out, y_stride, lane);
}

// vectors per wave (1, 2, 4 or 8): the pinned choice, else `pref`, halved while the launch would
// have fewer than MIX_MIN_WAVES waves for `tasks` tasks
int pick_vb(int pinned, int pref, int64_t tasks, int nvec)
{
    if (pinned) return pinned;
    int vb = pref;
    while (vb > 1 && tasks * ((nvec + vb - 1) / vb) < MIX_MIN_WAVES) vb /= 2;
    return vb;
}

// widest vector (4, 2 or 1 floats) that every address of a call keeps aligned
int call_vmax(const void* a, const void* b, int64_t sa, int64_t sb)
{
    for (int v = 4; v > 1; v /= 2)
        if (((uintptr_t)a % (4 * v)) == 0 && ((uintptr_t)b % (4 * v)) == 0 && sa % v == 0 && sb % v == 0) return v;
    return 1;
}

bool valid_mixer(const rtt_mixer* m) { return m && m->magic == MIX_MAGIC; }

int check_mix_call(const rtt_mixer* m, const void* a, const void* b, int32_t nvec)
{
    if (!valid_mixer(m)) return fail(RTT_EINVAL, "invalid mixer handle");
    if (nvec < 0 || nvec > 65535) return fail(RTT_EINVAL, "nvec must be in [0, 65535]");
    if (nvec > 0 && (!a || !b)) return fail(RTT_EINVAL, "NULL data pointer");
    if (((uintptr_t)a & 3) || ((uintptr_t)b & 3)) return fail(RTT_EINVAL, "pointers must be 4-byte aligned");
    return RTT_OK;
}

void release(rtt_mixer* m)
{
    for (int64_t** p : {&m->d_chunk, &m->d_list, &m->d_multi, &m->d_slots, &m->d_src})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
}

}  // namespace

namespace {

// The forward with the partial rows of multi-chunk mixed rows in `part` (n_slots * pitch * nvec
// floats, NULL when the mixer has none); the device of m is current.
int mix_forward_parts(const rtt_mixer* m, const float* y, int64_t y_stride, float* d, int64_t d_stride, int nvec,
                      float* part, hipStream_t s)
{
    const int64_t part_stride = m->n_slots * m->pitch;
    const int vmax = call_vmax(y, d, y_stride, d_stride);
    const dim3 blk(MIX_WAVES * WAVE);
    // short source lists (the unresolved image: one to a few rays per pixel): 8 vectors a wave so
    // that enough loads are in flight; long lists already keep 16 rows in flight with one vector
    const int vb = pick_vb(m->vb_apply, m->n_src >= 16 * m->n_chunks ? 1 : 8, m->n_chunks, nvec);
    const unsigned groups = (unsigned)((nvec + vb - 1) / vb);
    const dim3 gc((unsigned)((m->n_chunks + MIX_WAVES - 1) / MIX_WAVES), groups);
    const dim3 gp((unsigned)((m->n_multi + MIX_WAVES - 1) / MIX_WAVES), groups);
    const int vmax_p = std::min(vmax, call_vmax(part, d, part_stride, d_stride));
#define RTT_MIX_FWD(VB)                                                                                          \
    do {                                                                                                         \
        hipLaunchKernelGGL(k_mix_chunks<VB>, gc, blk, 0, s, m->d_chunk, m->d_list, m->n_chunks, y, y_stride, d,  \
                           d_stride, part, part_stride, m->pitch, nvec, vmax);                                  \
        if (m->n_multi > 0)                                                                                      \
            hipLaunchKernelGGL(k_mix_partials<VB>, gp, blk, 0, s, m->d_multi, m->d_slots, m->n_multi, part,      \
                               part_stride, d, d_stride, nvec, vmax_p);                                          \
    } while (0)
    switch (vb) {
    case 8: RTT_MIX_FWD(8); break;
    case 4: RTT_MIX_FWD(4); break;
    case 2: RTT_MIX_FWD(2); break;
    default: RTT_MIX_FWD(1); break;
    }
#undef RTT_MIX_FWD
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

}  // namespace

int mix_forward(const rtt_mixer* m, const float* y, int64_t y_stride, float* d, int64_t d_stride, int nvec,
                hipStream_t s)
{
    if (nvec == 0 || m->n_chunks == 0) return RTT_OK;
    RTT_HIP(hipSetDevice(m->device));
    float* part = nullptr;
    if (m->n_multi > 0) {
        part = (float*)m->ws.get("mix_partials", sizeof(float) * (size_t)(m->n_slots * m->pitch) * nvec);
        if (!part) return fail(RTT_ENOMEM, "mixer partial rows");
    }
    return mix_forward_parts(m, y, y_stride, d, d_stride, nvec, part, s);
}

bool mixer_ok(const rtt_mixer* m) { return valid_mixer(m); }
int64_t mixer_rows(const rtt_mixer* m) { return m->n_rows; }
int64_t mixer_src_rows(const rtt_mixer* m) { return m->n_src_rows; }

void mixer_segments(const rtt_mixer* m, std::vector<int64_t>& seg)
{
    for (size_t g = 0; g < m->g_off.size(); ++g) seg.insert(seg.end(), {m->g_off[g], m->g_rows[g]});
}

}  // namespace rtt

using namespace rtt;

extern "C" int mixer_create(const rtt_geometry* g, int32_t kind, const int64_t* const* pixels, rtt_mixer** out)
{
    if (!out) return fail(RTT_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (kind != RTT_MIX_UNRESOLVED && kind != RTT_MIX_TOTAL_FLUX) return fail(RTT_EINVAL, "unknown mixer kind");
    if (kind == RTT_MIX_UNRESOLVED && !pixels) return fail(RTT_EINVAL, "the unresolved mixer needs pixel indices");
    int64_t max_frames = 0;
    for (const Member& mb : g->members) max_frames = std::max<int64_t>(max_frames, mb.grid.n_frames);
    const int64_t pitch = (max_frames + 3) / 4 * 4;
    // widest vector width dividing F and every offset in offs
    auto width = [](int64_t F, std::initializer_list<int64_t> offs) {
        for (int v = 4; v > 1; v /= 2) {
            bool ok = F % v == 0;
            for (int64_t o : offs) ok = ok && o % v == 0;
            if (ok) return v;
        }
        return 1;
    };
    std::vector<int64_t> chunk, list, multi, slots, src;
    std::vector<int64_t> g_off, g_rows, g_out;
    int64_t out_off = 0, map_index = 0, n_slots = 0;
    for (const Member& mb : g->members) {
        const int64_t F = mb.grid.n_frames;
        int64_t n_rays = 0;
        for (int n = 0; n < mb.grid.n_orders; ++n) n_rays += mb.rays_per_order[n];
        // mixed row of every ray of this geometry, rays in data-row order
        std::vector<int64_t> target(n_rays, 0);
        int64_t n_out = 1;
        if (kind == RTT_MIX_UNRESOLVED) {
            std::vector<int64_t> pix;
            pix.reserve(n_rays);
            for (int n = 0; n < mb.grid.n_orders; ++n) {
                const int64_t* p = pixels[map_index + n];
                if (mb.rays_per_order[n] > 0 && !p) return fail(RTT_EINVAL, "NULL pixel array for a non-empty order");
                for (int64_t r = 0; r < mb.rays_per_order[n]; ++r) {
                    if (p[r] < 0) return fail(RTT_EINVAL, "pixel indices must be >= 0");
                    pix.push_back(p[r]);
                }
            }
            std::vector<int64_t> uniq(pix);
            std::sort(uniq.begin(), uniq.end());
            uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
            n_out = (int64_t)uniq.size();
            for (int64_t r = 0; r < n_rays; ++r)
                target[r] = std::lower_bound(uniq.begin(), uniq.end(), pix[r]) - uniq.begin();
        }
        map_index += mb.grid.n_orders;
        // source list of every mixed row (ascending data row)
        std::vector<std::vector<int64_t>> lists(n_out);
        for (int64_t r = 0; r < n_rays; ++r) lists[target[r]].push_back(mb.row_offset + r * F);
        for (int64_t o = 0; o < n_out; ++o) {
            const int64_t off = out_off + o * F;
            const std::vector<int64_t>& ls = lists[o];
            const int64_t nch = std::max<int64_t>(1, ((int64_t)ls.size() + MIX_CHUNK - 1) / MIX_CHUNK);
            const int64_t slot0 = n_slots;
            if (nch > 1) {
                multi.insert(multi.end(), {off, (int64_t)slots.size(), nch, F | (int64_t)width(F, {off}) << 32});
                for (int64_t c = 0; c < nch; ++c) slots.push_back((slot0 + c) * pitch);
                n_slots += nch;
            }
            for (int64_t c = 0; c < nch; ++c) {
                const int64_t b = c * MIX_CHUNK, e = std::min<int64_t>((int64_t)ls.size(), b + MIX_CHUNK);
                int vw = width(F, {nch == 1 ? off : 0});
                for (int64_t i = b; i < e; ++i) vw = std::min(vw, width(F, {ls[i]}));
                chunk.insert(chunk.end(), {(int64_t)list.size(), e - b, nch == 1 ? off : -1 - (slot0 + c),
                                           F | (int64_t)vw << 32});
                list.insert(list.end(), ls.begin() + b, ls.begin() + e);
            }
            for (int64_t so : ls) src.insert(src.end(), {so, off, F | (int64_t)width(F, {so, off}) << 32, 0});
        }
        g_off.push_back(out_off);
        g_rows.push_back(n_out * F);
        g_out.push_back(n_out);
        out_off += n_out * F;
    }
    auto m = new rtt_mixer();
    m->kind = kind;
    m->n_geometries = (int32_t)g->members.size();
    m->n_src_rows = g->n_rows;
    m->n_rows = out_off;
    m->g_off = std::move(g_off);
    m->g_rows = std::move(g_rows);
    m->g_out = std::move(g_out);
    m->n_chunks = (int64_t)chunk.size() / 4;
    m->n_multi = (int64_t)multi.size() / 4;
    m->n_src = (int64_t)src.size() / 4;
    m->n_slots = n_slots;
    m->pitch = pitch;
    m->device = g->device;
    hipError_t e = hipSetDevice(m->device);
    auto up = [&](int64_t** dst, const std::vector<int64_t>& v) {
        if (e != hipSuccess || v.empty()) return;
        e = hipMalloc((void**)dst, v.size() * sizeof(int64_t));
        if (e == hipSuccess) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    };
    up(&m->d_chunk, chunk);
    up(&m->d_list, list);
    up(&m->d_multi, multi);
    up(&m->d_slots, slots);
    up(&m->d_src, src);
    if (e != hipSuccess) {
        release(m);
        m->magic = 0;
        delete m;
        return e == hipErrorOutOfMemory ? fail(RTT_ENOMEM, "mixer tables") : hip_fail(e, "mixer_create");
    }
    *out = m;
    return RTT_OK;
}

extern "C" int mixer_free(rtt_mixer* m)
{
    if (!m) return RTT_OK;
    if (!valid_mixer(m)) return fail(RTT_EINVAL, "invalid mixer handle");
    (void)hipSetDevice(m->device);
    release(m);
    m->ws.release();
    m->magic = 0;
    delete m;
    return RTT_OK;
}

extern "C" int mixer_info(const rtt_mixer* m, rtt_mixer_info* info)
{
    if (!valid_mixer(m)) return fail(RTT_EINVAL, "invalid mixer handle");
    if (!info) return fail(RTT_EINVAL, "NULL info pointer");
    std::memset(info, 0, sizeof *info);
    info->kind = m->kind;
    info->n_geometries = m->n_geometries;
    info->n_rows = m->n_rows;
    info->n_src_rows = m->n_src_rows;
    return RTT_OK;
}

extern "C" int mixer_member(const rtt_mixer* m, int32_t gi, int64_t* row_offset, int64_t* n_rows, int64_t* n_out)
{
    if (!valid_mixer(m)) return fail(RTT_EINVAL, "invalid mixer handle");
    if (gi < 0 || gi >= m->n_geometries) return fail(RTT_EINVAL, "geometry index out of range");
    if (row_offset) *row_offset = m->g_off[gi];
    if (n_rows) *n_rows = m->g_rows[gi];
    if (n_out) *n_out = m->g_out[gi];
    return RTT_OK;
}

extern "C" int mixer_set_variant(rtt_mixer* m, int32_t apply_vectors, int32_t adjoint_vectors)
{
    if (!valid_mixer(m)) return fail(RTT_EINVAL, "invalid mixer handle");
    auto ok = [](int32_t v) { return v == -1 || v == 0 || v == 1 || v == 2 || v == 4 || v == 8; };
    if (!ok(apply_vectors) || !ok(adjoint_vectors)) return fail(RTT_EINVAL, "vectors per wave must be 0, 1, 2, 4 or 8");
    if (apply_vectors >= 0) m->vb_apply = apply_vectors;
    if (adjoint_vectors >= 0) m->vb_adjoint = adjoint_vectors;
    return RTT_OK;
}

extern "C" int mix_apply(const rtt_mixer* m, const float* y, float* d, int32_t nvec, void* stream)
{
    int rc = check_mix_call(m, y, d, nvec);
    if (rc) return rc;
    return mix_forward(m, y, m->n_src_rows, d, m->n_rows, nvec, (hipStream_t)stream);
}

// Partial rows of mix_apply_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes its name to a kernel: that is a host-side stand-in, not a
// device address.  The device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) float scratch[RTT_MIX_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// the device address of the scratch array on device `dev` (current)
int noalloc_scratch(int dev, float** out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(RTT_EDEVICE, "mix_apply_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RTT_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = (float*)p;
    }
    *out = g_scratch_dev[dev];
    return RTT_OK;
}

}  // namespace

extern "C" int mix_apply_noalloc(const rtt_mixer* m, const float* y, float* d, int32_t nvec, void* stream)
{
    int rc = check_mix_call(m, y, d, nvec);
    if (rc) return rc;
    const uint64_t need = sizeof(float) * (uint64_t)(m->n_slots * m->pitch) * (uint64_t)nvec;
    if (m->n_multi > 0 && need > RTT_MIX_NOALLOC_SCRATCH_BYTES) {
        const uint64_t per = sizeof(float) * (uint64_t)(m->n_slots * m->pitch);
        return fail(RTT_EINVAL, "mix_apply_noalloc: " + std::to_string(nvec) + " vectors need " +
                                    std::to_string(need) + " bytes of partial rows, more than the " +
                                    std::to_string((uint64_t)RTT_MIX_NOALLOC_SCRATCH_BYTES) +
                                    "-byte scratch (at most " + std::to_string(RTT_MIX_NOALLOC_SCRATCH_BYTES / per) +
                                    " vectors per call for this mixer)");
    }
    if (nvec == 0 || m->n_chunks == 0) return RTT_OK;
    RTT_HIP(hipSetDevice(m->device));
    float* part = nullptr;
    if (m->n_multi > 0 && (rc = noalloc_scratch(m->device, &part))) return rc;
    return mix_forward_parts(m, y, m->n_src_rows, d, m->n_rows, nvec, part, (hipStream_t)stream);
}

extern "C" int mix_adjoint(const rtt_mixer* m, const float* d, float* y, int32_t nvec, void* stream)
{
    int rc = check_mix_call(m, d, y, nvec);
    if (rc) return rc;
    if (nvec == 0 || m->n_src == 0) return RTT_OK;
    RTT_HIP(hipSetDevice(m->device));
    const int vb = pick_vb(m->vb_adjoint, 4, m->n_src, nvec);
    const dim3 grid((unsigned)((m->n_src + MIX_WAVES - 1) / MIX_WAVES), (unsigned)((nvec + vb - 1) / vb));
    const int vmax = call_vmax(d, y, m->n_rows, m->n_src_rows);
    hipStream_t s = (hipStream_t)stream;
#define RTT_MIX_ADJ(VB)                                                                                         \
    hipLaunchKernelGGL(k_mix_transpose<VB>, grid, dim3(MIX_WAVES * WAVE), 0, s, m->d_src, m->n_src, d, m->n_rows, y, \
                       m->n_src_rows, nvec, vmax)
    switch (vb) {
    case 8: RTT_MIX_ADJ(8); break;
    case 4: RTT_MIX_ADJ(4); break;
    case 2: RTT_MIX_ADJ(2); break;
    default: RTT_MIX_ADJ(1); break;
    }
#undef RTT_MIX_ADJ
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

extern "C" int mix_covariance(const rtt_mixer* m, const float* var, float* var_out, void* stream)
{
    // every source row feeds exactly one mixed row, so (L kron I) diag(var) (L^T kron I) is
    // diagonal with the added variances: the forward mix of the variance vector
    int rc = check_mix_call(m, var, var_out, 1);
    if (rc) return rc;
    return mix_forward(m, var, m->n_src_rows, var_out, m->n_rows, 1, (hipStream_t)stream);
}
