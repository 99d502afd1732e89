// The retarded-time operator A and its transpose on gfx950 (CDNA4, wave64).
//
// A (eq. (2)-(3), App. A.2 eq. (47)): one wavefront owns one ray.  For a chunk
// of frames it first forms the spatially combined series
//     z[k] = sum_{c in 2x2 stencil} b_c x[c][k]
// over the hats the chunk touches (lanes run over hats; four coalesced loads
// per hat from L2-resident x), parks z in LDS, then evaluates every frame as
// the two-tap hat interpolation of z scaled by the ray weight and streams the
// ray's contiguous row of y to HBM with non-temporal stores.  Rays are
// processed in base-cell order and workgroups are spread over the 8 XCDs in
// contiguous chunks, so each XCD's L2 holds about one eighth of x.
//
// A^T: owner computes.  A workgroup owns a tile of TR x TC cells and 64 hats.
// It walks the rays whose stencil can touch the tile (base rows i0-1 ..
// i0+TR-1, base columns j0-1 .. j0+TC-1 with periodic wrap: at most 2(TR+1)
// contiguous ranges of the base-cell-sorted ray array), each wave a
// contiguous slice of them.  Lanes run over the 64 hats: lane k gathers the
// frames whose hat window contains s_k, forms the transposed hat sum, and
// accumulates b_c w v into four registers (one per stencil corner) for as
// long as consecutive rays share a base cell (a segmented reduction over the
// sorted run).  At the end of a run the four partial sums are added into the
// wave's private LDS copy of the tile.  The copies are summed in a fixed order
// and every tile entry is written exactly once: no atomics, bitwise
// reproducible.
//
// Frame stepping.  With dt_obs/dt_src = P/Q, frame f has
//     u_f = k0 + th0 + f P / Q,  kf = k0 + (fP div Q) + [th0 + (fP mod Q)/Q >= 1]
// and the hat fraction th = th0 + (fP mod Q)/Q - carry.  Both kernels use the
// same function, so A^T is the exact transpose of A.
#include "rtt_internal.h"

namespace rtt {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

struct FrameStep {
    int kf;
    float th;
};

template <int TP, int TQ>
__device__ __forceinline__ FrameStep frame_step(int f, int k0, float th0, int P, int Q, float invQ)
{
    const int p = TP ? TP : P;
    const int q = TQ ? TQ : Q;
    const float iq = TQ ? 1.0f / (float)TQ : invQ;
    int m = f * p;
    int qd = m / q;
    int rm = m - qd * q;
    float u = th0 + (float)rm * iq;
    int c = u >= 1.0f ? 1 : 0;
    FrameStep s;
    s.kf = k0 + qd + c;
    s.th = u - (float)c;
    return s;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    // consecutive logical blocks go to the same XCD (hardware deals blocks round robin over 8)
    int64_t x = b & 7, i = b >> 3;
    int64_t per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + i;
}

// --------------------------------------------------------------------------------------------
// A: y = A x
// --------------------------------------------------------------------------------------------
struct ApplyArgs {
    const RayRec* rays;
    int64_t n_rays;
    int n_phi, K, F, P, Q;
    float invQ;
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
    uint32_t mask;
};

constexpr int A_WAVES = 4;
constexpr int A_FCHUNK = 256;
constexpr int A_ZMAX = A_FCHUNK + 8;   // (A_FCHUNK-1)*P/Q + 3 for P <= Q

template <int TP, int TQ, int RPW>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply(ApplyArgs a)
{
    __shared__ float zs_all[A_WAVES][A_ZMAX];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    float* zs = zs_all[wave];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const float* __restrict__ x = a.x + (int64_t)blockIdx.y * a.x_stride;
    float* __restrict__ y = a.y + (int64_t)blockIdx.y * a.y_stride;
    const int K = a.K, F = a.F;
    const bool staged = (TP && TQ) ? (TP <= TQ) : (a.P <= a.Q);
    const bool vec4 = ((F & 3) == 0) && ((((uintptr_t)y) & 15) == 0);

    for (int rpw = 0; rpw < RPW; ++rpw) {
        int64_t ri = (blk * A_WAVES + wave) * RPW + rpw;
        if (ri >= a.n_rays) break;
        ri = __builtin_amdgcn_readfirstlane((int)ri);
        const RayRec rr = a.rays[ri];
        if (!((a.mask >> rr.order) & 1u)) continue;
        const int i = rr.cell / a.n_phi;
        const int j0 = rr.cell - i * a.n_phi;
        const int j1 = (j0 + 1 == a.n_phi) ? 0 : j0 + 1;
        const float* __restrict__ x00 = x + (int64_t)(i * a.n_phi + j0) * K;
        const float* __restrict__ x10 = x + (int64_t)((i + 1) * a.n_phi + j0) * K;
        const float* __restrict__ x01 = x + (int64_t)(i * a.n_phi + j1) * K;
        const float* __restrict__ x11 = x + (int64_t)((i + 1) * a.n_phi + j1) * K;
        const float b00 = (1.0f - rr.fr) * (1.0f - rr.fphi), b10 = rr.fr * (1.0f - rr.fphi);
        const float b01 = (1.0f - rr.fr) * rr.fphi, b11 = rr.fr * rr.fphi;
        float* __restrict__ yrow = y + (int64_t)rr.row * F;

        if (!staged) {
            // frames sparser than hats: evaluate each frame directly (8 gathers)
            for (int f = lane; f < F; f += WAVE) {
                FrameStep st = frame_step<TP, TQ>(f, rr.k0, rr.th0, a.P, a.Q, a.invQ);
                float z0 = 0.f, z1 = 0.f;
                int k = st.kf;
                if (k >= 0 && k < K) z0 = b00 * x00[k] + b10 * x10[k] + b01 * x01[k] + b11 * x11[k];
                k += 1;
                if (k >= 0 && k < K) z1 = b00 * x00[k] + b10 * x10[k] + b01 * x01[k] + b11 * x11[k];
                __builtin_nontemporal_store(rr.w * ((1.0f - st.th) * z0 + st.th * z1), yrow + f);
            }
            continue;
        }

        for (int f0 = 0; f0 < F; f0 += A_FCHUNK) {
            const int fend = min(F, f0 + A_FCHUNK);
            const int klo = frame_step<TP, TQ>(f0, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf;
            const int khi = frame_step<TP, TQ>(fend - 1, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf + 1;
            const int W = khi - klo + 1;
            for (int j = lane; j < W; j += WAVE) {
                const int k = klo + j;
                float z = 0.f;
                if (k >= 0 && k < K) z = b00 * x00[k] + b10 * x10[k] + b01 * x01[k] + b11 * x11[k];
                zs[j] = z;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (vec4) {
                const int ng = (fend - f0) >> 2;
                for (int gq = lane; gq < ng; gq += WAVE) {
                    const int f = f0 + 4 * gq;
                    f4 v;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        FrameStep st = frame_step<TP, TQ>(f + t, rr.k0, rr.th0, a.P, a.Q, a.invQ);
                        const int jz = st.kf - klo;
                        v[t] = rr.w * ((1.0f - st.th) * zs[jz] + st.th * zs[jz + 1]);
                    }
                    __builtin_nontemporal_store(v, (f4*)(yrow + f));
                }
            } else {
                for (int f = f0 + lane; f < fend; f += WAVE) {
                    FrameStep st = frame_step<TP, TQ>(f, rr.k0, rr.th0, a.P, a.Q, a.invQ);
                    const int jz = st.kf - klo;
                    __builtin_nontemporal_store(rr.w * ((1.0f - st.th) * zs[jz] + st.th * zs[jz + 1]),
                                                yrow + f);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// --------------------------------------------------------------------------------------------
// A^T: x = A^T y
// --------------------------------------------------------------------------------------------
struct AdjArgs {
    const RayRec* rays;      // this member's sorted records
    const int32_t* cstart;   // this member's CSR (n_cells + 1)
    int n_r, n_phi, K, F, P, Q;
    float invQ;
    const float* y;
    float* x;
    int64_t y_stride, x_stride;
    uint32_t mask;
};

constexpr int T_WAVES = 4;
constexpr int KC = 64;   // hats per tile = lanes

template <int TP, int TQ>
__device__ __forceinline__ float hat_gather(const float* __restrict__ yrow, int k, int k0, float th0, int F,
                                            int P, int Q, float invQ)
{
    // sum over frames f of tau_k(t_f - delay) * y[f]  (frames whose kf is k or k-1)
    float v = 0.f;
    if (TP == 1 && TQ == 1) {
        const int f = k - k0;   // kf = k0 + f exactly (th0 < 1 => no carry)
        if (f >= 0 && f < F) v += (1.0f - th0) * yrow[f];
        if (f >= 1 && f - 1 < F) v += th0 * yrow[f - 1];
        return v;
    }
    const int p = TP ? TP : P;
    const int q = TQ ? TQ : Q;
    const int d = k - k0;
    // candidates: floor(fP/Q) in {d-2, d-1, d}  <=>  f in [ceil((d-2)Q/P), ceil((d+1)Q/P) - 1]
    auto ceil_div = [](int n, int dd) { return n >= 0 ? (n + dd - 1) / dd : -((-n) / dd); };
    int flo = ceil_div((d - 2) * q, p);
    int fhi = ceil_div((d + 1) * q, p) - 1;
    flo = max(flo, 0);
    fhi = min(fhi, F - 1);
    for (int f = flo; f <= fhi; ++f) {
        FrameStep st = frame_step<TP, TQ>(f, k0, th0, P, Q, invQ);
        const float yv = yrow[f];
        if (st.kf == k) v += (1.0f - st.th) * yv;
        else if (st.kf == k - 1) v += st.th * yv;
    }
    return v;
}

template <int TR, int TC, int TP, int TQ>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint(AdjArgs a)
{
    __shared__ float acc[T_WAVES][TR * TC][KC];
    __shared__ int rng_lo[2 * (TR + 1)], rng_hi[2 * (TR + 1)];
    __shared__ int n_rng_s;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;

    const int tiles_k = (a.K + KC - 1) / KC;
    const int tiles_c = (a.n_phi + TC - 1) / TC;
    const int tiles_r = (a.n_r + TR - 1) / TR;
    const int64_t lin = xcd_remap(blockIdx.x, (int64_t)tiles_r * tiles_c * tiles_k);
    const int tk = (int)(lin % tiles_k);
    const int tcell = (int)(lin / tiles_k);
    const int tc = tcell % tiles_c, tr = tcell / tiles_c;
    const int i0 = tr * TR, jlo = tc * TC;
    const int jhi = min(jlo + TC, a.n_phi);
    const int kc = tk * KC;
    const float* __restrict__ y = a.y + (int64_t)blockIdx.y * a.y_stride;
    float* __restrict__ x = a.x + (int64_t)blockIdx.y * a.x_stride;

    for (int e = threadIdx.x; e < T_WAVES * TR * TC * KC; e += blockDim.x) (&acc[0][0][0])[e] = 0.f;
    if (threadIdx.x == 0) {
        // ray ranges of the base cells whose 2x2 stencil can reach the tile
        int n = 0;
        const bool full_ring = (jhi - jlo) == a.n_phi;
        const int ib_lo = max(i0 - 1, 0), ib_hi = min(i0 + TR - 1, a.n_r - 2);
        for (int ib = ib_lo; ib <= ib_hi; ++ib) {
            const int rowc = ib * a.n_phi;
            if (full_ring) {
                rng_lo[n] = a.cstart[rowc]; rng_hi[n] = a.cstart[rowc + a.n_phi]; ++n;
            } else if (jlo == 0) {
                rng_lo[n] = a.cstart[rowc + a.n_phi - 1]; rng_hi[n] = a.cstart[rowc + a.n_phi]; ++n;
                rng_lo[n] = a.cstart[rowc]; rng_hi[n] = a.cstart[rowc + jhi]; ++n;
            } else {
                rng_lo[n] = a.cstart[rowc + jlo - 1]; rng_hi[n] = a.cstart[rowc + jhi]; ++n;
            }
        }
        n_rng_s = n;
    }
    __syncthreads();
    const int n_rng = n_rng_s;
    int total = 0;
    for (int r = 0; r < n_rng; ++r) total += rng_hi[r] - rng_lo[r];
    const int vlo = (int)(((int64_t)total * wave) / T_WAVES);
    const int vhi = (int)(((int64_t)total * (wave + 1)) / T_WAVES);

    float* accw = &acc[wave][0][0];
    float a00 = 0.f, a10 = 0.f, a01 = 0.f, a11 = 0.f;
    int l00 = -1, l10 = -1, l01 = -1, l11 = -1;
    int cur_cell = -1;
    const int k = kc + lane;

    auto flush = [&]() {
        if (l00 >= 0) accw[l00 * KC + lane] += a00;
        if (l10 >= 0) accw[l10 * KC + lane] += a10;
        if (l01 >= 0) accw[l01 * KC + lane] += a01;
        if (l11 >= 0) accw[l11 * KC + lane] += a11;
        a00 = a10 = a01 = a11 = 0.f;
    };
    auto local_of = [&](int ci, int cj) -> int {
        if (ci < i0 || ci >= i0 + TR || cj < jlo || cj >= jhi) return -1;
        return (ci - i0) * TC + (cj - jlo);
    };

    int base = 0;
    for (int r = 0; r < n_rng; ++r) {
        const int len = rng_hi[r] - rng_lo[r];
        const int s0 = max(vlo, base), s1 = min(vhi, base + len);
        for (int v = s0; v < s1; ++v) {
            const int ri = __builtin_amdgcn_readfirstlane(rng_lo[r] + (v - base));
            const RayRec rr = a.rays[ri];
            if (!((a.mask >> rr.order) & 1u)) continue;
            const int klast = frame_step<TP, TQ>(a.F - 1, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf + 1;
            if (rr.k0 > kc + KC - 1 || klast < kc) continue;
            if (rr.cell != cur_cell) {
                flush();
                cur_cell = rr.cell;
                const int ci = rr.cell / a.n_phi;
                const int cj0 = rr.cell - ci * a.n_phi;
                const int cj1 = (cj0 + 1 == a.n_phi) ? 0 : cj0 + 1;
                l00 = local_of(ci, cj0);
                l10 = local_of(ci + 1, cj0);
                l01 = local_of(ci, cj1);
                l11 = local_of(ci + 1, cj1);
            }
            const float* __restrict__ yrow = y + (int64_t)rr.row * a.F;
            float hv = (k < a.K) ? hat_gather<TP, TQ>(yrow, k, rr.k0, rr.th0, a.F, a.P, a.Q, a.invQ) : 0.f;
            hv *= rr.w;
            a00 += (1.0f - rr.fr) * (1.0f - rr.fphi) * hv;
            a10 += rr.fr * (1.0f - rr.fphi) * hv;
            a01 += (1.0f - rr.fr) * rr.fphi * hv;
            a11 += rr.fr * rr.fphi * hv;
        }
        base += len;
    }
    flush();
    __syncthreads();
    for (int e = threadIdx.x; e < TR * TC * KC; e += blockDim.x) {
        const int lc = e / KC, kk = kc + (e % KC);
        const int ci = i0 + lc / TC, cj = jlo + lc % TC;
        if (ci < a.n_r && cj < jhi && kk < a.K) {
            float s = acc[0][lc][e % KC];
#pragma unroll
            for (int w = 1; w < T_WAVES; ++w) s += acc[w][lc][e % KC];
            x[(int64_t)(ci * a.n_phi + cj) * a.K + kk] = s;
        }
    }
}

// --------------------------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------------------------
struct AdjVariant {
    const char* name;
    int tr, tc;
};
static const AdjVariant kAdjVariants[] = {{"tile8x8", 8, 8}, {"tile4x8", 4, 8}, {"tile4x4", 4, 4}};

int n_adjoint_variants() { return 3; }
const char* adjoint_variant_name(int v) { return kAdjVariants[v].name; }
int n_apply_variants() { return 2; }
const char* apply_variant_name(int v) { return v == 0 ? "rpw1" : "rpw2"; }

int default_adjoint_variant(const Member& m)
{
    // small grids need smaller tiles to fill the chip
    int64_t cells = (int64_t)m.grid.n_r * m.grid.n_phi;
    if (cells >= 128 * 128) return 0;
    if (cells >= 64 * 64) return 1;
    return 2;
}
int default_apply_variant(const Member& m) { return m.n_rays >= 65536 ? 1 : 0; }

template <int TP, int TQ>
static void apply_dispatch(const ApplyArgs& a, int nvec, int variant, hipStream_t s)
{
    const int rpw = variant == 1 ? 2 : 1;
    const int64_t rays_per_block = (int64_t)A_WAVES * rpw;
    dim3 grid((unsigned)((a.n_rays + rays_per_block - 1) / rays_per_block), (unsigned)nvec);
    if (rpw == 2)
        hipLaunchKernelGGL((k_apply<TP, TQ, 2>), grid, dim3(A_WAVES * WAVE), 0, s, a);
    else
        hipLaunchKernelGGL((k_apply<TP, TQ, 1>), grid, dim3(A_WAVES * WAVE), 0, s, a);
}

int launch_apply(const rtt_geometry* g, const Member& m, const float* x, float* y, int nvec,
                 int64_t x_stride, int64_t y_stride, uint32_t mask, hipStream_t s, int variant)
{
    if (m.n_rays == 0 || nvec == 0) return RTT_OK;
    ApplyArgs a;
    a.rays = g->d_rays + m.ray_begin;
    a.n_rays = m.n_rays;
    a.n_phi = m.grid.n_phi;
    a.K = m.grid.n_hat;
    a.F = m.grid.n_frames;
    a.P = m.P;
    a.Q = m.Q;
    a.invQ = 1.0f / (float)m.Q;
    a.x = x;
    a.y = y;
    a.x_stride = x_stride;
    a.y_stride = y_stride;
    a.mask = mask;
    if (variant < 0 || variant >= n_apply_variants()) variant = m.apply_variant;
    if (m.P == 1 && m.Q == 1) apply_dispatch<1, 1>(a, nvec, variant, s);
    else if (m.P == 1 && m.Q == 2) apply_dispatch<1, 2>(a, nvec, variant, s);
    else apply_dispatch<0, 0>(a, nvec, variant, s);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

template <int TR, int TC>
static void adjoint_dispatch_tile(const AdjArgs& a, int P, int Q, int nvec, hipStream_t s)
{
    const int64_t tiles = (int64_t)((a.n_r + TR - 1) / TR) * ((a.n_phi + TC - 1) / TC) * ((a.K + KC - 1) / KC);
    dim3 grid((unsigned)tiles, (unsigned)nvec);
    if (P == 1 && Q == 1)
        hipLaunchKernelGGL((k_adjoint<TR, TC, 1, 1>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else if (P == 1 && Q == 2)
        hipLaunchKernelGGL((k_adjoint<TR, TC, 1, 2>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<TR, TC, 0, 0>), grid, dim3(T_WAVES * WAVE), 0, s, a);
}

int launch_adjoint(const rtt_geometry* g, const Member& m, const float* y, float* x, int nvec,
                   int64_t y_stride, int64_t x_stride, uint32_t mask, hipStream_t s, int variant)
{
    if (nvec == 0) return RTT_OK;
    AdjArgs a;
    a.rays = g->d_rays + m.ray_begin;
    a.cstart = g->d_cell_start + m.cell_begin;
    a.n_r = m.grid.n_r;
    a.n_phi = m.grid.n_phi;
    a.K = m.grid.n_hat;
    a.F = m.grid.n_frames;
    a.P = m.P;
    a.Q = m.Q;
    a.invQ = 1.0f / (float)m.Q;
    a.y = y;
    a.x = x;
    a.y_stride = y_stride;
    a.x_stride = x_stride;
    a.mask = mask;
    if (variant < 0 || variant >= n_adjoint_variants()) variant = m.adj_variant;
    switch (variant) {
    case 0: adjoint_dispatch_tile<8, 8>(a, m.P, m.Q, nvec, s); break;
    case 1: adjoint_dispatch_tile<4, 8>(a, m.P, m.Q, nvec, s); break;
    default: adjoint_dispatch_tile<4, 4>(a, m.P, m.Q, nvec, s); break;
    }
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

}  // namespace rtt

namespace rtt {

int apply_op(const rtt_geometry* g, int member, bool adjoint, const float* in, float* out, int nvec,
             uint32_t mask, hipStream_t s)
{
    if (member >= 0) {
        const Member& m = g->members[member];
        const uint32_t em = effective_mask(m, mask);
        return adjoint ? launch_adjoint(g, m, in, out, nvec, m.n_rows, m.n_cols, em, s, -1)
                       : launch_apply(g, m, in, out, nvec, m.n_cols, m.n_rows, em, s, -1);
    }
    for (const Member& m : g->members) {
        const uint32_t em = effective_mask(m, mask);
        int rc = adjoint ? launch_adjoint(g, m, in + m.row_offset, out + m.col_offset, nvec, g->n_rows, g->n_cols,
                                          em, s, -1)
                         : launch_apply(g, m, in + m.col_offset, out + m.row_offset, nvec, g->n_cols, g->n_rows,
                                        em, s, -1);
        if (rc) return rc;
    }
    return RTT_OK;
}

}  // namespace rtt

using namespace rtt;

static int check_call(const rtt_geometry* g, const void* a, const void* b, int32_t nvec)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    if (nvec < 0) return fail(RTT_EINVAL, "nvec must be >= 0");
    if (nvec > 65535) return fail(RTT_EINVAL, "nvec must be <= 65535 per call");
    if (nvec > 0 && (!a || !b)) return fail(RTT_EINVAL, "NULL data pointer");
    if (((uintptr_t)a & 3) || ((uintptr_t)b & 3)) return fail(RTT_EINVAL, "pointers must be 4-byte aligned");
    return RTT_OK;
}

extern "C" int op_apply(const rtt_geometry* g, const float* x, float* y, int32_t nvec, uint32_t order_mask,
                        void* stream)
{
    int rc = check_call(g, x, y, nvec);
    if (rc) return rc;
    return apply_op(g, -1, false, x, y, nvec, order_mask, (hipStream_t)stream);
}

extern "C" int op_apply_adjoint(const rtt_geometry* g, const float* y, float* x, int32_t nvec,
                                uint32_t order_mask, void* stream)
{
    int rc = check_call(g, y, x, nvec);
    if (rc) return rc;
    return apply_op(g, -1, true, y, x, nvec, order_mask, (hipStream_t)stream);
}
