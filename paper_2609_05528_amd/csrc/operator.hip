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
#include <algorithm>
#include <cstdlib>

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
__device__ __forceinline__ uint32_t xcd_remap32(uint32_t b, uint32_t nb)
{
    uint32_t x = b & 7, i = b >> 3;
    uint32_t per = nb >> 3, rem = nb & 7;
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

// hat_gather with a fixed candidate count and clamped, unconditional loads (no divergent
// branches around the loads, so a batch of rays keeps all its loads in flight).
template <int TP, int TQ>
__device__ __forceinline__ float hat_gather_clamped(const float* __restrict__ yrow, int k, int k0, float th0, int F,
                                                    int P, int Q, float invQ)
{
    const int p = TP ? TP : P;
    const int q = TQ ? TQ : Q;
    const int d = k - k0;
    auto ceil_div = [](int n, int dd) { return n >= 0 ? (n + dd - 1) / dd : -((-n) / dd); };
    const int flo = ceil_div((d - 2) * q, p);
    const int fhi = ceil_div((d + 1) * q, p) - 1;
    float v = 0.f;
    if (TP && TQ) {
        constexpr int NC = (3 * (TQ > 0 ? TQ : 1) + (TP > 0 ? TP : 1) - 1) / (TP > 0 ? TP : 1) + 1;
        float yv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) yv[c] = yrow[min(max(flo + c, 0), F - 1)];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int f = flo + c;
            if (f > fhi || f < 0 || f >= F) continue;
            const FrameStep st = frame_step<TP, TQ>(f, k0, th0, P, Q, invQ);
            if (st.kf == k) v += (1.0f - st.th) * yv[c];
            else if (st.kf == k - 1) v += st.th * yv[c];
        }
        return v;
    }
    for (int f = max(flo, 0); f <= min(fhi, F - 1); ++f) {
        const FrameStep st = frame_step<TP, TQ>(f, k0, th0, P, Q, invQ);
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
// A^T, batched tile form: the owner-computes LDS tile of k_adjoint, but each wave walks its
// slice of the tile's ray ranges NB rays at a time: the range table lives in scalar registers,
// all NB ray records and data loads are issued before any is consumed, then the NB
// contributions are folded into the corner registers in order (flushing to the wave's LDS copy
// whenever the base cell changes).
// --------------------------------------------------------------------------------------------
template <int TR, int TC, int TP, int TQ, int NB>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint_tb(AdjArgs a)
{
    constexpr int NR = 2 * (TR + 1);
    __shared__ float acc[T_WAVES][TR * TC][KC];
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

    // ray ranges of the base cells whose stencil reaches the tile (uniform, compile-time indexed)
    int rlo[NR], rln[NR];
    const bool full_ring = (jhi - jlo) == a.n_phi;
#pragma unroll
    for (int t = 0; t <= TR; ++t) {
        const int ib = i0 - 1 + t;
        rlo[2 * t] = rln[2 * t] = rlo[2 * t + 1] = rln[2 * t + 1] = 0;
        if (ib < 0 || ib > a.n_r - 2) continue;
        const int rowc = ib * a.n_phi;
        if (full_ring) {
            rlo[2 * t] = a.cstart[rowc];
            rln[2 * t] = a.cstart[rowc + a.n_phi] - rlo[2 * t];
        } else if (jlo == 0) {
            rlo[2 * t] = a.cstart[rowc + a.n_phi - 1];
            rln[2 * t] = a.cstart[rowc + a.n_phi] - rlo[2 * t];
            rlo[2 * t + 1] = a.cstart[rowc];
            rln[2 * t + 1] = a.cstart[rowc + jhi] - rlo[2 * t + 1];
        } else {
            rlo[2 * t] = a.cstart[rowc + jlo - 1];
            rln[2 * t] = a.cstart[rowc + jhi] - rlo[2 * t];
        }
    }
    int total = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) total += rln[r];
    const int vlo = (int)(((int64_t)total * wave) / T_WAVES);
    const int vhi = (int)(((int64_t)total * (wave + 1)) / T_WAVES);
    __syncthreads();

    float* accw = &acc[wave][0][0];
    float a00 = 0.f, a10 = 0.f, a01 = 0.f, a11 = 0.f;
    int l00 = -1, l10 = -1, l01 = -1, l11 = -1;
    int cur_cell = -1;
    const int k = kc + lane;
    auto local_of = [&](int ci, int cj) -> int {
        if (ci < i0 || ci >= i0 + TR || cj < jlo || cj >= jhi) return -1;
        return (ci - i0) * TC + (cj - jlo);
    };

    for (int v0 = vlo; v0 < vhi; v0 += NB) {
        // phase 1: ray indices (scalar) and records (independent scalar loads)
        int ri[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int v = min(v0 + j, vhi - 1);
            int r_ = rlo[0], off = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (v >= off && v < off + rln[r]) r_ = rlo[r] + (v - off);
                off += rln[r];
            }
            ri[j] = __builtin_amdgcn_readfirstlane(r_);
        }
        RayRec rr[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) rr[j] = a.rays[ri[j]];
        // phase 2: every data load of the batch, unconditional (clamped indices)
        float hv[NB];
        if (TP == 1 && TQ == 1) {
            float ya[NB], yb[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const float* __restrict__ yrow = y + (int64_t)rr[j].row * a.F;
                const int f = k - rr[j].k0;
                ya[j] = yrow[min(max(f, 0), a.F - 1)];
                yb[j] = yrow[min(max(f - 1, 0), a.F - 1)];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int f = k - rr[j].k0;
                const float h = ((f >= 0 && f < a.F) ? (1.0f - rr[j].th0) * ya[j] : 0.f) +
                                ((f >= 1 && f - 1 < a.F) ? rr[j].th0 * yb[j] : 0.f);
                hv[j] = h;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const float* __restrict__ yrow = y + (int64_t)rr[j].row * a.F;
                hv[j] = hat_gather_clamped<TP, TQ>(yrow, k, rr[j].k0, rr[j].th0, a.F, a.P, a.Q, a.invQ);
            }
        }
        // phase 3: fold the batch into the corner registers in order
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const bool valid = v0 + j < vhi;
            if (!valid) continue;
            const int klast = frame_step<TP, TQ>(a.F - 1, rr[j].k0, rr[j].th0, a.P, a.Q, a.invQ).kf + 1;
            const bool on = ((a.mask >> rr[j].order) & 1u) && !(rr[j].k0 > kc + KC - 1 || klast < kc) && k < a.K;
            const float h = on ? hv[j] * rr[j].w : 0.f;
            if (rr[j].cell != cur_cell) {
                if (l00 >= 0) accw[l00 * KC + lane] += a00;
                if (l10 >= 0) accw[l10 * KC + lane] += a10;
                if (l01 >= 0) accw[l01 * KC + lane] += a01;
                if (l11 >= 0) accw[l11 * KC + lane] += a11;
                a00 = a10 = a01 = a11 = 0.f;
                cur_cell = rr[j].cell;
                const int ci = cur_cell / a.n_phi;
                const int cj0 = cur_cell - ci * a.n_phi;
                const int cj1 = (cj0 + 1 == a.n_phi) ? 0 : cj0 + 1;
                l00 = local_of(ci, cj0);
                l10 = local_of(ci + 1, cj0);
                l01 = local_of(ci, cj1);
                l11 = local_of(ci + 1, cj1);
            }
            const float fr = rr[j].fr, fp = rr[j].fphi;
            a00 += (1.0f - fr) * (1.0f - fp) * h;
            a10 += fr * (1.0f - fp) * h;
            a01 += (1.0f - fr) * fp * h;
            a11 += fr * fp * h;
        }
    }
    if (l00 >= 0) accw[l00 * KC + lane] += a00;
    if (l10 >= 0) accw[l10 * KC + lane] += a10;
    if (l01 >= 0) accw[l01 * KC + lane] += a01;
    if (l11 >= 0) accw[l11 * KC + lane] += a11;
    __syncthreads();
    for (int e = threadIdx.x; e < TR * TC * KC; e += blockDim.x) {
        const int lc = e / KC, kk = kc + (e % KC);
        const int ci = i0 + lc / TC, cj = jlo + lc % TC;
        if (ci < a.n_r && cj < jhi && kk < a.K) {
            float sum = acc[0][lc][e % KC];
#pragma unroll
            for (int w = 1; w < T_WAVES; ++w) sum += acc[w][lc][e % KC];
            x[(int64_t)(ci * a.n_phi + cj) * a.K + kk] = sum;
        }
    }
}

// --------------------------------------------------------------------------------------------
// A, batched form: a wave owns NB consecutive (base-cell sorted) rays and one chunk of frames.
// All ray records and x gathers of the batch are issued before any is consumed, the combined
// series z of every ray goes to LDS, then the wave streams NB row segments with float4 stores
// using all 64 lanes.  Used when frames are at least as dense as hats (P <= Q).
// --------------------------------------------------------------------------------------------
template <int TP, int TQ, int NB, int ZI>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_batch(ApplyArgs a, int fc)
{
    constexpr int ZW = ZI * WAVE + 4;
    __shared__ float zs_all[A_WAVES][NB][ZW];
    __shared__ int pi_all[A_WAVES][NB][4];     // klo, k0, row, active
    __shared__ float pf_all[A_WAVES][NB][2];   // th0, w
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t r0 = (blk * A_WAVES + wave) * NB;
    if (r0 >= a.n_rays) return;   // no block-wide barrier below: a wave may leave early
    const float* __restrict__ x = a.x + (int64_t)blockIdx.y * a.x_stride;
    float* __restrict__ y = a.y + (int64_t)blockIdx.y * a.y_stride;
    const int K = a.K, F = a.F;
    const int f0 = blockIdx.z * fc;
    const int fend = min(F, f0 + fc);
    float (*zs)[ZW] = zs_all[wave];

    float xv[NB][ZI][4];
    float bw[NB][4];
    int klo[NB], W[NB];
    bool act[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int64_t ri = r0 + j;
        act[j] = ri < a.n_rays;
        const RayRec rr = a.rays[__builtin_amdgcn_readfirstlane((int)(act[j] ? ri : r0))];
        act[j] = act[j] && ((a.mask >> rr.order) & 1u);
        const int i = rr.cell / a.n_phi;
        const int j0 = rr.cell - i * a.n_phi;
        const int j1 = (j0 + 1 == a.n_phi) ? 0 : j0 + 1;
        klo[j] = frame_step<TP, TQ>(f0, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf;
        const int khi = frame_step<TP, TQ>(fend - 1, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf + 1;
        W[j] = khi - klo[j] + 1;
        bw[j][0] = (1.0f - rr.fr) * (1.0f - rr.fphi);
        bw[j][1] = rr.fr * (1.0f - rr.fphi);
        bw[j][2] = (1.0f - rr.fr) * rr.fphi;
        bw[j][3] = rr.fr * rr.fphi;
        const int64_t c00 = (int64_t)(i * a.n_phi + j0) * K, c10 = (int64_t)((i + 1) * a.n_phi + j0) * K;
        const int64_t c01 = (int64_t)(i * a.n_phi + j1) * K, c11 = (int64_t)((i + 1) * a.n_phi + j1) * K;
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const int jj = lane + it * WAVE;
            const int k = klo[j] + jj;
            const bool ok = act[j] && jj < W[j] && k >= 0 && k < K;
            const int kk = ok ? k : 0;
            xv[j][it][0] = ok ? x[c00 + kk] : 0.f;
            xv[j][it][1] = ok ? x[c10 + kk] : 0.f;
            xv[j][it][2] = ok ? x[c01 + kk] : 0.f;
            xv[j][it][3] = ok ? x[c11 + kk] : 0.f;
        }
        if (lane == 0) {
            pi_all[wave][j][0] = klo[j];
            pi_all[wave][j][1] = rr.k0;
            pi_all[wave][j][2] = rr.row;
            pi_all[wave][j][3] = act[j] ? 1 : 0;
            pf_all[wave][j][0] = rr.th0;
            pf_all[wave][j][1] = rr.w;
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const int jj = lane + it * WAVE;
            if (jj < W[j])
                zs[j][jj] = bw[j][0] * xv[j][it][0] + bw[j][1] * xv[j][it][1] + bw[j][2] * xv[j][it][2] +
                            bw[j][3] * xv[j][it][3];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const bool vec4 = ((F & 3) == 0) && ((fend - f0) & 3) == 0 && ((((uintptr_t)y) & 15) == 0);
    if (vec4) {
        const int ng = (fend - f0) >> 2;
        for (int g = lane; g < NB * ng; g += WAVE) {
            const int j = g / ng, q = g - j * ng;
            if (!pi_all[wave][j][3]) continue;
            const int kl = pi_all[wave][j][0], k0 = pi_all[wave][j][1];
            const float th0 = pf_all[wave][j][0], w = pf_all[wave][j][1];
            const int f = f0 + 4 * q;
            f4 v;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const FrameStep st = frame_step<TP, TQ>(f + t, k0, th0, a.P, a.Q, a.invQ);
                const int jz = st.kf - kl;
                v[t] = w * ((1.0f - st.th) * zs[j][jz] + st.th * zs[j][jz + 1]);
            }
            __builtin_nontemporal_store(v, (f4*)(y + (int64_t)pi_all[wave][j][2] * F + f));
        }
    } else {
        const int ng = fend - f0;
        for (int g = lane; g < NB * ng; g += WAVE) {
            const int j = g / ng, q = g - j * ng;
            if (!pi_all[wave][j][3]) continue;
            const int kl = pi_all[wave][j][0], k0 = pi_all[wave][j][1];
            const float th0 = pf_all[wave][j][0], w = pf_all[wave][j][1];
            const int f = f0 + q;
            const FrameStep st = frame_step<TP, TQ>(f, k0, th0, a.P, a.Q, a.invQ);
            const int jz = st.kf - kl;
            __builtin_nontemporal_store(w * ((1.0f - st.th) * zs[j][jz] + st.th * zs[j][jz + 1]),
                                        y + (int64_t)pi_all[wave][j][2] * F + f);
        }
    }
}

// --------------------------------------------------------------------------------------------
// A, lean form for dt_obs/dt_src = 1/Q (Q = 1, 2).  Per ray the wave reads a 48-byte record with
// corner offsets and weights precomputed (no division, no weight arithmetic), stages the
// combined series z over the chunk's hats in LDS (hats clamped into [0, K) for addressing and
// masked with one compare; one buffer descriptor per x vector, the radial corner step in the
// scalar offset), then writes the rows: 4 frames per lane from one 16-byte LDS read
// plus one 4-byte read (Q = 1) or two 8-byte reads with the half-step weights of the ray
// (Q = 2).  Frame chunks are 128 Q frames so the lane -> (ray, frame group) split is a shift.
// --------------------------------------------------------------------------------------------
struct LeanArgs {
    const FwdRec* rec;
    int64_t n_rays;
    int K, F, nk;       // nk = n_phi * K (row offset of the i+1 corners)
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
    int x_bytes;        // bytes of one coefficient vector
    uint32_t mask;
    int fc;             // frames per chunk (multiple of 4, at most lean_fcmax(Q))
};

// A forward record read through the constant address space (the tables never change while a
// kernel runs), so uniform reads stay scalar loads.
typedef int i4v __attribute__((ext_vector_type(4)));
struct RecWords {
    i4v w0, w1, w2;
};
static_assert(sizeof(RecWords) == sizeof(FwdRec), "FwdRec is three 16-byte words");
__device__ __forceinline__ FwdRec load_const_rec(const FwdRec* p)
{
    typedef const __attribute__((address_space(4))) i4v* cptr;
    const cptr q = (cptr)p;
    RecWords r;
    r.w0 = q[0];
    r.w1 = q[1];
    r.w2 = q[2];
    return __builtin_bit_cast(FwdRec, r);
}

// Output phase shared by the staged forward kernels: the wave's NB combined series z (LDS rows
// of ZS floats starting at zs0, hat h of ray j at zs0[j*ZS + h]) are interpolated to the frames
// [f0, fend) of each ray and written to its data row.  With aligned rows (VEC4): Q = 1 takes one
// ray per pass with two frames per lane (8-byte stores), Q = 2 four frames per lane (16-byte
// stores); otherwise one frame per lane.
// Hats staged per ray chunk (LDS row length) and the longest frame chunk they serve: a chunk
// of fc frames starting at hat klo reads hats klo .. klo + fc/Q + 1.
constexpr int LEAN_ZI = 3;
constexpr int LEAN_ZS = LEAN_ZI * WAVE;
constexpr int lean_fcmax(int Q) { return Q * (LEAN_ZS - 4); }

template <int Q, int NB, bool VEC4>
__device__ __forceinline__ void lean_emit(const float* zs0, const float* th0, const int* row, const bool* on,
                                          int f0, int fend, int F, float* __restrict__ y)
{
    constexpr int ZS = LEAN_ZS;
    const int lane = threadIdx.x & (WAVE - 1);
    const float(*zs)[ZS] = (const float(*)[ZS])zs0;
    const int nf = fend - f0;   // frames of this chunk (at most lean_fcmax(Q))
    if constexpr (VEC4 && Q == 1 && NB % 2 == 0) {
        if ((F & 3) == 0 && (((uintptr_t)y) & 15) == 0) {
            // rows of a multiple of 4 frames, 16-byte aligned (chunks start at multiples of 4): two
            // rays per pass (lanes 0-31 ray j, lanes 32-63 ray j + 1), four frames per lane in one
            // 16-byte store, the same values as the two-frame form below
            const int lane2 = lane & 31;
            const bool hi = lane >= 32;
#pragma unroll
            for (int j = 0; j < NB; j += 2) {
                const int jj = hi ? j + 1 : j;
                const bool o = hi ? on[j + 1] : on[j];
                const float th = th0[jj];
                float* yr = y + (int64_t)row[jj] * F;
#pragma unroll
                for (int p = 0; p < (lean_fcmax(1) + 127) / 128; ++p) {
                    if (p * 128 >= nf) break;
                    const int q = p * 128 + 4 * lane2;
                    if (!o || q >= nf) continue;   // frames q .. q + 4 of the LDS row exist below nf
                    const float* zr = &zs[0][0] + jj * ZS + q;
                    const f4 za = *(const f4*)zr;
                    const float z4 = zr[4];
                    f4 v;
                    v[0] = za[0] + th * (za[1] - za[0]);
                    v[1] = za[1] + th * (za[2] - za[1]);
                    v[2] = za[2] + th * (za[3] - za[2]);
                    v[3] = za[3] + th * (z4 - za[3]);
                    __builtin_nontemporal_store(v, (f4*)(yr + f0 + q));
                }
            }
            return;
        }
    }
    if (VEC4 && Q == 1) {
        // one ray per pass of 128 frames, two frames per lane (8-byte stores): ray values stay uniform
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (!on[j]) continue;
            const float th = th0[j];
            float* yr = y + (int64_t)row[j] * F;
#pragma unroll
            for (int p = 0; p < (lean_fcmax(1) + 127) / 128; ++p) {
                if (p * 128 >= nf) break;
                const int q = p * 128 + 2 * lane;
                const float* zr = &zs[0][0] + j * ZS + q;
                const f2 za = *(const f2*)zr;
                const float zc = zr[2];
                f2 v;
                v[0] = za[0] + th * (za[1] - za[0]);
                v[1] = za[1] + th * (zc - za[1]);
                if (q < nf) __builtin_nontemporal_store(v, (f2*)(yr + f0 + q));
            }
        }
    } else if (VEC4) {
        // Q = 2: one ray per pass of 256 frames, four frames per lane (16-byte stores)
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (!on[j]) continue;
            const float th = th0[j];
            const bool c1 = th >= 0.5f;
            const float th1 = c1 ? th - 0.5f : th + 0.5f;
            float* yr = y + (int64_t)row[j] * F;
#pragma unroll
            for (int p = 0; p < (lean_fcmax(2) + 255) / 256; ++p) {
                if (p * 256 >= nf) break;
                const int g = p * 64 + lane;
                const float* zr = &zs[0][0] + j * ZS + 2 * g;
                const f2 za = *(const f2*)zr;
                const f2 zb = *(const f2*)(zr + 2);
                const float z0 = za[0], z1 = za[1], z2 = zb[0], z3 = zb[1];
                const float a1 = c1 ? z1 : z0, b1 = c1 ? z2 : z1;
                const float a3 = c1 ? z2 : z1, b3 = c1 ? z3 : z2;
                f4 v;
                v[0] = z0 + th * (z1 - z0);
                v[1] = a1 + th1 * (b1 - a1);
                v[2] = z1 + th * (z2 - z1);
                v[3] = a3 + th1 * (b3 - a3);
                if (4 * g < nf) __builtin_nontemporal_store(v, (f4*)(yr + f0 + 4 * g));
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (!on[j]) continue;
            float* yr = y + (int64_t)row[j] * F;
#pragma unroll
            for (int t = 0; t < (lean_fcmax(Q) + WAVE - 1) / WAVE; ++t) {
                if (t * WAVE >= nf) break;
                const int q = lane + t * WAVE;
                if (q >= nf) continue;
                int jz;
                float th;
                if (Q == 1) {
                    jz = q;
                    th = th0[j];
                } else {
                    const bool odd = q & 1;
                    const bool c1 = th0[j] >= 0.5f;
                    jz = (q >> 1) + ((odd && c1) ? 1 : 0);
                    th = odd ? (c1 ? th0[j] - 0.5f : th0[j] + 0.5f) : th0[j];
                }
                const float za = zs[j][jz], zb = zs[j][jz + 1];
                __builtin_nontemporal_store(za + th * (zb - za), yr + f0 + q);
            }
        }
    }
}

// The staged forward's LDS rows, one array per batch size shared by every form of the body a
// kernel inlines (so a kernel that branches between output forms allocates it once).
template <int NB>
__device__ __forceinline__ float (*lean_lds())[NB][LEAN_ZS]
{
    __shared__ __attribute__((aligned(16))) float zs_all[A_WAVES][NB][LEAN_ZS];
    return zs_all;
}

// Output staging rows of the lean forward at Q = 1: NB rows of up to lean_fcmax(1) frames per wave,
// plus up to 3 floats that put the block in the same 16-byte phase as its destination.
template <int NB>
constexpr int lean_ob_floats() { return (NB * lean_fcmax(1) + 3 + 3) / 4 * 4; }

template <int NB>
__device__ __forceinline__ float (*lean_obuf())[lean_ob_floats<NB>()]
{
    __shared__ __attribute__((aligned(16))) float ob_all[A_WAVES][lean_ob_floats<NB>()];
    return ob_all;
}

// The n values staged in ob[pad ..] leave for yb[0 .. n) (yb at the 16-byte phase pad) in 16-byte
// stores aligned to the range, 4-byte stores only for the at most 3 + 3 values at its two ends.
template <int NB>
__device__ __forceinline__ void range_store(const float* ob, int pad, int n, float* __restrict__ yb)
{
    const int lane = threadIdx.x & (WAVE - 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int h = (4 - pad) & 3;                  // head: values before the first 16-byte boundary
    const int nq = (n - h) >> 2;                  // whole quads after it
    if (lane < h && lane < n) __builtin_nontemporal_store(ob[pad + lane], yb + lane);
    for (int g = lane; g < nq; g += WAVE) {
        const int d = h + 4 * g;                  // yb + d and ob + pad + d are 16-byte aligned
        const f4 v = *(const f4*)(ob + pad + d);
        __builtin_nontemporal_store(v, (f4*)(yb + d));
    }
    const int tail0 = h + 4 * nq;
    if (lane < n - tail0) __builtin_nontemporal_store(ob[pad + tail0 + lane], yb + tail0 + lane);
    // the next task of a persistent block writes this wave's staging row again
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Q = 1 output of NB rays that are consecutive data rows, their whole rows in one chunk: the values
// (as lean_emit forms them) go to LDS at the 16-byte phase of the destination, then the contiguous
// NB * F range goes out in 16-byte stores aligned to it, 4-byte stores only for the at most 3 + 3
// values at its two ends.  A per-ray store starts wherever its row starts, so rows of a length that
// is not a multiple of the sector split sectors between store instructions and waves.
template <int NB>
__device__ __forceinline__ void lean_emit_staged(const float* zs0, const float* th0, int row0, int F,
                                                 float* __restrict__ y, float* ob)
{
    constexpr int ZS = LEAN_ZS;
    const int lane = threadIdx.x & (WAVE - 1);
    const float(*zs)[ZS] = (const float(*)[ZS])zs0;
    float* yb = y + (int64_t)row0 * F;
    const int pad = (int)(((uintptr_t)yb >> 2) & 3);   // floats of yb past a 16-byte boundary
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const float th = th0[j];
#pragma unroll
        for (int t = 0; t < (lean_fcmax(1) + WAVE - 1) / WAVE; ++t) {
            const int q = lane + t * WAVE;
            if (q >= F) break;
            const float za = zs[j][q], zb = zs[j][q + 1];
            ob[pad + j * F + q] = za + th * (zb - za);
        }
    }
    range_store<NB>(ob, pad, NB * F, yb);
}

// One block of the lean forward: rays [blk*A_WAVES*NB, +A_WAVES*NB) of one member, frame chunk
// `chunk`, one vector (x, y already offset to the member's blocks).
template <int Q, int NB, bool VEC4>
__device__ __forceinline__ void lean_body(const LeanArgs& a, const float* __restrict__ x, float* __restrict__ y,
                                          int64_t blk, int chunk)
{
    constexpr int ZI = LEAN_ZI;
    constexpr int ZS = LEAN_ZS;          // LDS row length: hats staged per ray
    float(*zs_all)[NB][ZS] = lean_lds<NB>();
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (blk * A_WAVES + wave) * NB;
    if (r0 >= a.n_rays) return;
    const int f0 = chunk * a.fc;
    const int fend = min(a.F, f0 + a.fc);
    float(*zs)[ZS] = zs_all[wave];
    // the previous task of a persistent block may still be reading this wave's LDS rows
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, a.x_bytes, 0x00020000);

    // phase 1: every record of the batch (independent scalar loads)
    FwdRec rc[NB];
    bool on[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int64_t ri = r0 + j;
        // scalar loads even after the stores of an earlier task of a persistent block
        rc[j] = load_const_rec(a.rec + __builtin_amdgcn_readfirstlane((int)(ri < a.n_rays ? ri : r0)));
    }
    // phase 2: every gather of the batch
    float xv[NB][ZI][4];
    bool live[NB][ZI];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        on[j] = (r0 + j < a.n_rays) && ((a.mask >> rc[j].order) & 1u);
        const int klo = rc[j].k0 + f0 / Q;
        // The scalar offset is unsigned and not range checked: it only carries the
        // non-negative row step n_phi*K.  The column step to the periodic neighbour can be
        // negative (wrap at 2 pi), so it goes into the vector offset, which is either an
        // element offset inside the x vector or, for a hat outside [0, K), a value past its end.
        const int s10 = a.nk * 4;
        // rays sorted by base cell: a ray with the same cell and hat origin as the previous one
        // needs exactly the same x values (uniform branch)
        if (j > 0 && rc[j].c00k == rc[j - 1].c00k && rc[j].d01k == rc[j - 1].d01k && rc[j].k0 == rc[j - 1].k0) {
#pragma unroll
            for (int it = 0; it < ZI; ++it) {
                live[j][it] = live[j - 1][it];
#pragma unroll
                for (int c = 0; c < 4; ++c) xv[j][it][c] = xv[j - 1][it][c];
            }
            continue;
        }
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            // hats outside [0, K) carry no basis function: a chunk with none inside is skipped
            // (uniform branch), lanes outside get an offset past the end of x, which returns 0
            // without a memory access
            const int kb = klo + it * WAVE;
            live[j][it] = kb < a.K && kb + WAVE > 0;
            if (!live[j][it]) continue;
            const int k = kb + lane;
            const bool in = (unsigned)k < (unsigned)a.K;
            const int off0 = in ? (rc[j].c00k + k) * 4 : 0x7FFFFFF0;
            const int off1 = in ? off0 + rc[j].d01k * 4 : 0x7FFFFFF0;
            xv[j][it][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off0, 0, 0));
            xv[j][it][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off0, s10, 0));
            xv[j][it][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off1, 0, 0));
            xv[j][it][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off1, s10, 0));
        }
    }
    // phase 3: combined series into LDS (hats outside [0, K) and inactive rays give 0)
    float th0[NB];
    int row[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        th0[j] = rc[j].th0;
        row[j] = rc[j].row;
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            // lanes of hats outside [0, K) loaded zeros; rays that are off are not written
            const float z = live[j][it] ? rc[j].b00 * xv[j][it][0] + rc[j].b10 * xv[j][it][1] +
                                              rc[j].b01 * xv[j][it][2] + rc[j].b11 * xv[j][it][3]
                                        : 0.f;
            zs[j][lane + it * WAVE] = z;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    if constexpr (Q == 1) {
        // rays in data-row order (lean4r) that are consecutive rows: one staged contiguous range
        bool flat = f0 == 0 && fend == a.F;
#pragma unroll
        for (int j = 0; j < NB; ++j) flat = flat && on[j] && row[j] == row[0] + j;
        if (flat) {
            lean_emit_staged<NB>(&zs[0][0], th0, row[0], a.F, y, lean_obuf<NB>()[wave]);
            return;
        }
    }
    lean_emit<Q, NB, VEC4>(&zs[0][0], th0, row, on, f0, fend, a.F, y);
}

// Quad-gather form of the lean forward, for K % 4 == 0: every x row then starts 16-byte aligned,
// so the hats a chunk needs are read as aligned quads, one 16-byte load per stencil corner on
// at most 35 lanes instead of one 4-byte load per hat; a quad lies wholly inside or wholly
// outside [0, K) and is fetched or skipped as a whole.  The combined series is written to LDS
// shifted to the ray's first hat, and the output phase is the lean one.
template <int Q, int NB, bool VEC4>
__device__ __forceinline__ void leanq_body(const LeanArgs& a, const float* __restrict__ x, float* __restrict__ y,
                                           int64_t blk, int chunk)
{
    constexpr int FC = 128 * Q;
    constexpr int W = FC / Q + 4;
    constexpr int ZI = (W + WAVE - 1) / WAVE;
    constexpr int ZS = ZI * WAVE;
    constexpr int NQ = (W + 3) / 4 + 1;   // quads covering W hats from any start (35)
    __shared__ __attribute__((aligned(16))) float zs_all[A_WAVES][NB][ZS];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (blk * A_WAVES + wave) * NB;
    if (r0 >= a.n_rays) return;
    const int f0 = chunk * FC;
    const int fend = min(a.F, f0 + FC);
    float(*zs)[ZS] = zs_all[wave];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, a.x_bytes, 0x00020000);
    const int s10 = a.nk * 4;

    FwdRec rc[NB];
    bool on[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int64_t ri = r0 + j;
        rc[j] = load_const_rec(a.rec + __builtin_amdgcn_readfirstlane((int)(ri < a.n_rays ? ri : r0)));
    }
    f4 xq[NB][4];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        on[j] = (r0 + j < a.n_rays) && ((a.mask >> rc[j].order) & 1u);
        // same base cell and hat origin as the previous ray: the same x values (uniform branch)
        if (j > 0 && rc[j].c00k == rc[j - 1].c00k && rc[j].d01k == rc[j - 1].d01k && rc[j].k0 == rc[j - 1].k0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) xq[j][c] = xq[j - 1][c];
            continue;
        }
        const int klo = rc[j].k0 + f0 / Q;
        const int ka = klo & ~3;                      // aligned start (floor, also for klo < 0)
        const int kq = ka + 4 * lane;                 // this lane's quad
        const bool in = lane < NQ && kq >= 0 && kq < a.K;
        const int off0 = in ? (rc[j].c00k + kq) * 4 : 0x7FFFFFF0;
        const int off1 = in ? off0 + rc[j].d01k * 4 : 0x7FFFFFF0;
        xq[j][0] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, off0, 0, 0));
        xq[j][1] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, off0, s10, 0));
        xq[j][2] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, off1, 0, 0));
        xq[j][3] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, off1, s10, 0));
    }
    float th0[NB];
    int row[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        th0[j] = rc[j].th0;
        row[j] = rc[j].row;
        const int klo = rc[j].k0 + f0 / Q;
        const int base = 4 * lane - (klo - (klo & ~3));   // LDS position of the quad's first hat
        const f4 z = rc[j].b00 * xq[j][0] + rc[j].b10 * xq[j][1] + rc[j].b01 * xq[j][2] + rc[j].b11 * xq[j][3];
        // every position of z[j][0 .. W) is written by exactly one lane
        if (lane < NQ) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int h = base + t;
                if (h >= 0 && h < W) zs[j][h] = z[t];
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    lean_emit<Q, NB, VEC4>(&zs[0][0], th0, row, on, f0, fend, a.F, y);
}

template <int Q, int NB, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_leanq(LeanArgs a)
{
    leanq_body<Q, NB, VEC4>(a, a.x + (int64_t)blockIdx.y * a.x_stride, a.y + (int64_t)blockIdx.y * a.y_stride,
                            xcd_remap(blockIdx.x, gridDim.x), blockIdx.z);
}

template <int Q, int NB, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_lean(LeanArgs a)
{
    lean_body<Q, NB, VEC4>(a, a.x + (int64_t)blockIdx.y * a.x_stride, a.y + (int64_t)blockIdx.y * a.y_stride,
                           xcd_remap(blockIdx.x, gridDim.x), blockIdx.z);
}

// --------------------------------------------------------------------------------------------
// A, absolute-hat form of the lean forward, for n_hat <= 128 and dt_obs/dt_src = 1/Q.  Gather
// lane l of pass it holds hat k = l + 64 it of a corner row whatever the ray's time origin, so
// the rays of one base cell need exactly the same x values: consecutive rays of a cell (the
// records are sorted by base cell) share one set of gathers.  Each ray's combined series over
// all K hats goes to an LDS row and its whole frame range is written from it (no frame chunks);
// hats outside [0, K) read as 0.  The products and the order of the sums are those of the lean
// form (the two agree to rounding: FMA contraction may differ).
// --------------------------------------------------------------------------------------------
constexpr int ABS_KMAX = 2 * WAVE;

// One block of the absolute-hat forward: rays [blk*A_WAVES*NB, +A_WAVES*NB) of one member, one
// vector (x, y already offset to the member's blocks), every frame.
// STAGE (records in data-row order, Q = 1): NB rays that are consecutive data rows with rows of at
// most lean_fcmax(1) frames leave as one staged, 16-byte aligned range (as lean4r).
template <int Q, int NB, bool VEC4, bool REUSE, bool STAGE = false>
__device__ __forceinline__ void abs_body(const LeanArgs& a, const float* __restrict__ x, float* __restrict__ y,
                                         int64_t blk)
{
    float(*zs_all)[NB][LEAN_ZS] = lean_lds<NB>();
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (blk * A_WAVES + wave) * NB;
    if (r0 >= a.n_rays) return;
    float(*zs)[LEAN_ZS] = zs_all[wave];
    if (REUSE) {
        // the previous task of a persistent block may still be reading this wave's LDS rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, a.x_bytes, 0x00020000);
    const int K = a.K;
    const bool two = K > WAVE;   // second gather pass (hats 64..127)

    FwdRec rc[NB];
    bool on[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int64_t ri = r0 + j;
        rc[j] = load_const_rec(a.rec + __builtin_amdgcn_readfirstlane((int)(ri < a.n_rays ? ri : r0)));
    }
    float xv[NB][2][4];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        on[j] = (r0 + j < a.n_rays) && ((a.mask >> rc[j].order) & 1u);
        if (j > 0 && rc[j].c00k == rc[j - 1].c00k && rc[j].d01k == rc[j - 1].d01k) {
            // same base cell as the previous ray (uniform branch): same corner rows, same hats
#pragma unroll
            for (int it = 0; it < 2; ++it)
#pragma unroll
                for (int c = 0; c < 4; ++c) xv[j][it][c] = xv[j - 1][it][c];
            continue;
        }
        const int s10 = a.nk * 4;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            if (it == 1 && !two) {
#pragma unroll
                for (int c = 0; c < 4; ++c) xv[j][it][c] = 0.f;
                continue;
            }
            const int k = lane + it * WAVE;
            const bool in = k < K;
            // lanes past the last hat read past the end of x (0, no memory access); the column
            // step to the periodic neighbour can be negative, so it stays in the vector offset
            const int off0 = in ? (rc[j].c00k + k) * 4 : 0x7FFFFFF0;
            const int off1 = in ? off0 + rc[j].d01k * 4 : 0x7FFFFFF0;
            xv[j][it][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off0, 0, 0));
            xv[j][it][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off0, s10, 0));
            xv[j][it][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off1, 0, 0));
            xv[j][it][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, off1, s10, 0));
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int it = 0; it < 2; ++it)
            zs[j][lane + it * WAVE] = rc[j].b00 * xv[j][it][0] + rc[j].b10 * xv[j][it][1] +
                                      rc[j].b01 * xv[j][it][2] + rc[j].b11 * xv[j][it][3];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int F = a.F;
    if constexpr (STAGE && Q == 1) {
        bool flat = F <= lean_fcmax(1);
#pragma unroll
        for (int j = 0; j < NB; ++j) flat = flat && on[j] && rc[j].row == rc[0].row + j;
        if (flat) {
            // the values of the per-ray path below, staged at the 16-byte phase of the range
            float* ob = lean_obuf<NB>()[wave];
            float* yb = y + (int64_t)rc[0].row * F;
            const int pad = (int)(((uintptr_t)yb >> 2) & 3);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const float* zr = zs[j];
                auto zat = [&](int k) { return (unsigned)k < (unsigned)K ? zr[k] : 0.f; };
                const float th = rc[j].th0;
                const int k0 = rc[j].k0;
                for (int q = lane; q < F; q += WAVE) {
                    const float za = zat(k0 + q), zb = zat(k0 + q + 1);
                    ob[pad + j * F + q] = za + th * (zb - za);
                }
            }
            range_store<NB>(ob, pad, NB * F, yb);
            return;
        }
    }
    if constexpr (VEC4 && Q == 1 && NB % 2 == 0) {
        if ((F & 3) == 0 && (((uintptr_t)y) & 15) == 0) {
            // rows of a multiple of 4 frames, 16-byte aligned: two rays per pass (lanes 0-31 ray j,
            // lanes 32-63 ray j + 1), four frames per lane in one 16-byte store, the same values
            // as the per-ray path below
            const bool hi = lane >= 32;
#pragma unroll
            for (int j = 0; j < NB; j += 2) {
                const float* zr = zs[hi ? j + 1 : j];
                auto zat = [&](int k) { return (unsigned)k < (unsigned)K ? zr[k] : 0.f; };
                const float th = hi ? rc[j + 1].th0 : rc[j].th0;
                const int k0 = hi ? rc[j + 1].k0 : rc[j].k0;
                const bool o = hi ? on[j + 1] : on[j];
                float* yr = y + (int64_t)(hi ? rc[j + 1].row : rc[j].row) * F;
                for (int f = 4 * (lane & 31); f < F; f += 128) {
                    const float z0 = zat(k0 + f), z1 = zat(k0 + f + 1), z2 = zat(k0 + f + 2);
                    const float z3 = zat(k0 + f + 3), z4 = zat(k0 + f + 4);
                    f4 v;
                    v[0] = z0 + th * (z1 - z0);
                    v[1] = z1 + th * (z2 - z1);
                    v[2] = z2 + th * (z3 - z2);
                    v[3] = z3 + th * (z4 - z3);
                    if (o) __builtin_nontemporal_store(v, (f4*)(yr + f));
                }
            }
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (!on[j]) continue;
        const float* zr = zs[j];
        // z at hat k, 0 outside [0, K)
        auto zat = [&](int k) { return (unsigned)k < (unsigned)K ? zr[k] : 0.f; };
        const float th = rc[j].th0;
        const int k0 = rc[j].k0;
        float* yr = y + (int64_t)rc[j].row * F;
        if (VEC4 && Q == 1) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            for (int f = 2 * lane; f < F; f += 2 * WAVE) {
                const float z0 = zat(k0 + f), z1 = zat(k0 + f + 1), z2 = zat(k0 + f + 2);
                f2 v;
                v[0] = z0 + th * (z1 - z0);
                v[1] = z1 + th * (z2 - z1);
                __builtin_nontemporal_store(v, (f2*)(yr + f));
            }
        } else if (VEC4) {
            const bool c1 = th >= 0.5f;
            const float th1 = c1 ? th - 0.5f : th + 0.5f;
            for (int g = lane; 4 * g < F; g += WAVE) {
                const int kb = k0 + 2 * g;
                const float z0 = zat(kb), z1 = zat(kb + 1), z2 = zat(kb + 2), z3 = zat(kb + 3);
                const float a1 = c1 ? z1 : z0, b1 = c1 ? z2 : z1;
                const float a3 = c1 ? z2 : z1, b3 = c1 ? z3 : z2;
                f4 v;
                v[0] = z0 + th * (z1 - z0);
                v[1] = a1 + th1 * (b1 - a1);
                v[2] = z1 + th * (z2 - z1);
                v[3] = a3 + th1 * (b3 - a3);
                __builtin_nontemporal_store(v, (f4*)(yr + 4 * g));
            }
        } else {
            for (int q = lane; q < F; q += WAVE) {
                int jz;
                float t;
                if (Q == 1) {
                    jz = q;
                    t = th;
                } else {
                    const bool odd = q & 1;
                    const bool c1 = th >= 0.5f;
                    jz = (q >> 1) + ((odd && c1) ? 1 : 0);
                    t = odd ? (c1 ? th - 0.5f : th + 0.5f) : th;
                }
                const float za = zat(k0 + jz), zb = zat(k0 + jz + 1);
                __builtin_nontemporal_store(za + t * (zb - za), yr + q);
            }
        }
    }
}

template <int Q, int NB, bool VEC4, bool STAGE = false>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_abs(LeanArgs a)
{
    abs_body<Q, NB, VEC4, false, STAGE>(a, a.x + (int64_t)blockIdx.y * a.x_stride,
                                        a.y + (int64_t)blockIdx.y * a.y_stride, xcd_remap(blockIdx.x, gridDim.x));
}

// Every member of a handle (up to MULTI_MAX) in one launch.  Tasks are (vector, member, frame
// chunk, ray block), numbered with the ray block fastest; a member's tasks start at blk_begin
// inside each vector.  With gridDim.x < total the launch is persistent: block b takes tasks
// b, b + gridDim.x, ... (gridDim.x is a multiple of 8, so every task of a block stays on the
// block's XCD and the XCD-contiguous numbering of xcd_remap still holds).
constexpr int MULTI_MAX = 16;
struct LeanMember {
    const FwdRec* rec;
    int64_t n_rays;
    int64_t x_off, y_off;
    uint32_t blk_begin;  // first task of this member inside one vector
    uint32_t nrb;        // ray blocks per frame chunk
    int K, F, nk, x_bytes;
    uint32_t mask;
    int fc;              // frames per chunk
    int wide;            // rows aligned for the wide output stores
};
struct LeanMulti {
    LeanMember m[MULTI_MAX];
    int G;
    uint32_t per_vec, total;   // tasks per vector and in all (below 2^31, checked by the host)
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
};

template <int Q, int NB, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_lean_multi(LeanMulti a)
{
    for (uint32_t t = blockIdx.x; t < a.total; t += gridDim.x) {
        const uint32_t lt = xcd_remap32(t, a.total);
        const uint32_t v = lt / a.per_vec;
        uint32_t b = lt - v * a.per_vec;
        int g = 0;
        while (g + 1 < a.G && b >= a.m[g + 1].blk_begin) ++g;
        const LeanMember& mm = a.m[g];
        b -= mm.blk_begin;
        LeanArgs la;
        la.rec = mm.rec;
        la.n_rays = mm.n_rays;
        la.K = mm.K;
        la.F = mm.F;
        la.nk = mm.nk;
        la.x_bytes = mm.x_bytes;
        la.mask = mm.mask;
        la.fc = mm.fc;
        const uint32_t chunk = b / mm.nrb;
        const float* xv = a.x + (int64_t)v * a.x_stride + mm.x_off;
        float* yv = a.y + (int64_t)v * a.y_stride + mm.y_off;
        if (VEC4 && mm.wide)
            lean_body<Q, NB, true>(la, xv, yv, (int64_t)(b - chunk * mm.nrb), (int)chunk);
        else
            lean_body<Q, NB, false>(la, xv, yv, (int64_t)(b - chunk * mm.nrb), (int)chunk);
    }
}

// The absolute-hat forward of every member in one launch: tasks are (vector, member, ray block),
// numbered as in k_apply_lean_multi with a single frame chunk per member.
template <int Q, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_abs_multi(LeanMulti a)
{
    for (uint32_t t = blockIdx.x; t < a.total; t += gridDim.x) {
        const uint32_t lt = xcd_remap32(t, a.total);
        const uint32_t v = lt / a.per_vec;
        uint32_t b = lt - v * a.per_vec;
        int g = 0;
        while (g + 1 < a.G && b >= a.m[g + 1].blk_begin) ++g;
        const LeanMember& mm = a.m[g];
        b -= mm.blk_begin;
        LeanArgs la;
        la.rec = mm.rec;
        la.n_rays = mm.n_rays;
        la.K = mm.K;
        la.F = mm.F;
        la.nk = mm.nk;
        la.x_bytes = mm.x_bytes;
        la.mask = mm.mask;
        la.fc = mm.fc;
        const float* xv = a.x + (int64_t)v * a.x_stride + mm.x_off;
        float* yv = a.y + (int64_t)v * a.y_stride + mm.y_off;
        if (VEC4 && mm.wide)
            abs_body<Q, 4, true, true>(la, xv, yv, (int64_t)b);
        else
            abs_body<Q, 4, false, true>(la, xv, yv, (int64_t)b);
    }
}

// --------------------------------------------------------------------------------------------
// A, strip form for dt_obs/dt_src = 1/Q (Q = 1, 2).  A workgroup owns a strip of SC base cells
// of one cell row i (rays are sorted by base cell, so the strip's rays are one contiguous run)
// and one frame chunk.  It first copies the x rows of every corner cell the strip can touch --
// cells (i, j) and (i+1, j) for the SC + 1 columns j of the strip, over the hats the chunk can
// reach -- into LDS with coalesced loads, then each wave forms the combined series z of its
// rays from LDS and writes the rows as the lean form does.  Every x value is fetched through
// L1 once per strip instead of once per ray and corner, which is what limits the lean form.
// --------------------------------------------------------------------------------------------
struct StripArgs {
    const FwdRec* rec;       // the member's records, sorted by base cell
    const int32_t* cstart;   // the member's CSR over base cells (n_cells + 1 entries)
    int n_r, n_phi, K, F;
    int SC, nstrip;          // strip width in base cells, strips per cell row
    int w_alloc;             // hats per staged row (LDS row length)
    int k0min, k0max;        // range of the records' k0
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
    uint32_t mask;
};

template <int Q, int NB, bool VEC4>
__device__ __forceinline__ void strip_body(const StripArgs& a, const float* __restrict__ x, float* __restrict__ y,
                                           int64_t blk, int chunk)
{
    constexpr int FC = 128 * Q;
    constexpr int W = FC / Q + 4;
    constexpr int ZI = (W + WAVE - 1) / WAVE;
    constexpr int ZS = ZI * WAVE;
    extern __shared__ __attribute__((aligned(16))) float lds_dyn[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = (int)(blk / a.nstrip), sg = (int)(blk % a.nstrip);
    const int j0 = sg * a.SC;
    const int ncs = min(a.SC, a.n_phi - j0);           // base columns of this strip
    const int cbase = i * a.n_phi + j0;
    const int r_begin = a.cstart[cbase], r_end = a.cstart[cbase + ncs];
    if (r_begin >= r_end) return;                       // uniform over the workgroup
    const int f0 = chunk * FC;
    const int fend = min(a.F, f0 + FC);
    const int hlo = max(0, a.k0min + f0 / Q);
    const int hhi = min(a.K, a.k0max + f0 / Q + FC / Q + 2);
    const int wst = hhi - hlo;                          // staged hats (may be <= 0: all zero)
    const int ws = a.w_alloc;
    float* st = lds_dyn;                                // [2][SC + 1][w_alloc]
    // stage the corner rows: rr = 0 (row i), 1 (row i+1); cc = 0 .. ncs (periodic column)
    for (int r = wave; r < 2 * (a.SC + 1); r += A_WAVES) {
        const int rr = r / (a.SC + 1), cc = r % (a.SC + 1);
        if (cc > ncs) continue;
        int jc = j0 + cc;
        if (jc >= a.n_phi) jc -= a.n_phi;
        const float* xr = x + ((int64_t)(i + rr) * a.n_phi + jc) * a.K + hlo;
        for (int h = lane; h < wst; h += WAVE) st[r * ws + h] = xr[h];
    }
    __syncthreads();
    float* zs = lds_dyn + 2 * (a.SC + 1) * ws + wave * NB * ZS;
    for (int rb = r_begin + wave * NB; rb < r_end; rb += A_WAVES * NB) {
        // the previous round's output phase may still be reading this wave's z rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float th0[NB];
        int row[NB];
        bool on[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int ri = rb + j;
            const FwdRec rc = load_const_rec(a.rec + (ri < r_end ? ri : r_end - 1));
            on[j] = ri < r_end && ((a.mask >> rc.order) & 1u);
            th0[j] = rc.th0;
            row[j] = rc.row;
            const int jc = rc.cell - cbase;             // local base column, 0 .. ncs-1
            const float* r00 = st + jc * ws - hlo;      // corner rows indexed by hat k
            const float* r01 = r00 + ws;
            const float* r10 = r00 + (a.SC + 1) * ws;
            const float* r11 = r10 + ws;
            const int klo = rc.k0 + f0 / Q;
#pragma unroll
            for (int it = 0; it < ZI; ++it) {
                const int h = lane + it * WAVE;
                const int k = klo + h;
                const bool ok = on[j] && k >= hlo && k < hhi;
                const int kk = ok ? k : hlo;
                const float z = rc.b00 * r00[kk] + rc.b10 * r10[kk] + rc.b01 * r01[kk] + rc.b11 * r11[kk];
                if (h < W) zs[j * ZS + h] = ok ? z : 0.f;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        lean_emit<Q, NB, VEC4>(zs, th0, row, on, f0, fend, a.F, y);
    }
}

template <int Q, int NB, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_strip(StripArgs a)
{
    strip_body<Q, NB, VEC4>(a, a.x + (int64_t)blockIdx.y * a.x_stride, a.y + (int64_t)blockIdx.y * a.y_stride,
                            xcd_remap(blockIdx.x, gridDim.x), blockIdx.z);
}

// --------------------------------------------------------------------------------------------
// A, register form for dt_obs/dt_src = 1/Q (Q = 1, 2).  Lanes run over frames, four consecutive
// frames per lane: a ray's frame chunk of 4 LPR frames is covered by LPR lanes and 64/LPR rays
// share a wave pass.  Each lane reads the hats its four frames need straight into registers,
// one 16-byte load per stencil corner (plus one 4-byte load for the fifth hat when Q = 1),
// combines the corners, interpolates and writes its frames with one 16-byte store: no LDS, and
// about a third of the memory instructions of the staged form.  A lane whose window would leave
// the x vector (corners in the first or last cells only) reads its hats one by one with offsets
// clamped into the vector.  Hats outside [0, K) contribute zero.  Records are scalar loads of
// the pass's rays, picked per lane.
// --------------------------------------------------------------------------------------------
struct RegArgs {
    const FwdRec* rec;
    int64_t n_rays;
    int K, F, nk, x_bytes;   // nk = n_phi * K: element step to the radial neighbour corner
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
    uint32_t mask;
};

template <int Q, int LPR, int NI, bool VEC4>
__device__ __forceinline__ void reg_body(const RegArgs& a, const float* __restrict__ x, float* __restrict__ y,
                                         int64_t blk, int chunk)
{
    constexpr int R = WAVE / LPR;           // rays side by side in a pass
    constexpr int FC = 4 * LPR;             // frames per chunk
    constexpr int NH = Q == 1 ? 5 : 4;      // hats per lane
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar record loads
    const int sub = lane / LPR;             // ray of this lane inside a pass
    const int li = lane % LPR;              // lane inside the ray
    const int64_t rb = (blk * A_WAVES + wave) * (int64_t)(R * NI);
    if (rb >= a.n_rays) return;
    const int f = chunk * FC + 4 * li;      // first frame of this lane (a multiple of 4)
    const int hoff = f / Q;                 // its hat offset from k0 (exact: Q divides 4)
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, a.x_bytes, 0x00020000);
    const int lim = a.x_bytes - 4 * NH;     // largest start (bytes) of a window inside x
    const int last = a.x_bytes / 4 - 1;     // last element of x

    int o[NI][4], kb[NI], row[NI];
    float bw[NI][4], th[NI];
    bool on[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        FwdRec rj[R];
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) {
            const int64_t ri = rb + (int64_t)j * R + s2;
            rj[s2] = load_const_rec(a.rec + (ri < a.n_rays ? ri : a.n_rays - 1));
        }
        FwdRec mine = rj[0];
#pragma unroll
        for (int s2 = 1; s2 < R; ++s2)
            if (sub == s2) mine = rj[s2];
        const int64_t ri = rb + (int64_t)j * R + sub;
        on[j] = ri < a.n_rays && ((a.mask >> mine.order) & 1u) && f < a.F;
        kb[j] = mine.k0 + hoff;
        o[j][0] = mine.c00k + kb[j];          // corner (i, j0)
        o[j][1] = o[j][0] + a.nk;             // corner (i+1, j0)
        o[j][2] = o[j][0] + mine.d01k;        // corner (i, j0+1), periodic
        o[j][3] = o[j][2] + a.nk;             // corner (i+1, j0+1)
        bw[j][0] = mine.b00;
        bw[j][1] = mine.b10;
        bw[j][2] = mine.b01;
        bw[j][3] = mine.b11;
        th[j] = mine.th0;
        row[j] = mine.row;
    }
    float xv[NI][4][NH];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        bool fast = lim >= 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) fast = fast && (unsigned)(o[j][c] * 4) <= (unsigned)lim;
        if (fast) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const f4 w = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(xr, o[j][c] * 4, 0, 0));
                xv[j][c][0] = w[0];
                xv[j][c][1] = w[1];
                xv[j][c][2] = w[2];
                xv[j][c][3] = w[3];
                if constexpr (Q == 1)
                    xv[j][c][4] = __builtin_bit_cast(float,
                                                     __builtin_amdgcn_raw_buffer_load_b32(xr, o[j][c] * 4 + 16, 0, 0));
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    const int e = min(max(o[j][c] + h, 0), last);
                    xv[j][c][h] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xr, e * 4, 0, 0));
                }
        }
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        if (!on[j]) continue;
        float z[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const float zz = bw[j][0] * xv[j][0][h] + bw[j][1] * xv[j][1][h] + bw[j][2] * xv[j][2][h] +
                             bw[j][3] * xv[j][3][h];
            z[h] = (unsigned)(kb[j] + h) < (unsigned)a.K ? zz : 0.f;
        }
        const float t = th[j];
        f4 v;
        if constexpr (Q == 1) {
            v[0] = z[0] + t * (z[1] - z[0]);
            v[1] = z[1] + t * (z[2] - z[1]);
            v[2] = z[2] + t * (z[3] - z[2]);
            v[3] = z[3] + t * (z[4] - z[3]);
        } else {
            const bool c1 = t >= 0.5f;
            const float t1 = c1 ? t - 0.5f : t + 0.5f;
            const float a1 = c1 ? z[1] : z[0], b1 = c1 ? z[2] : z[1];
            const float a3 = c1 ? z[2] : z[1], b3 = c1 ? z[3] : z[2];
            v[0] = z[0] + t * (z[1] - z[0]);
            v[1] = a1 + t1 * (b1 - a1);
            v[2] = z[1] + t * (z[2] - z[1]);
            v[3] = a3 + t1 * (b3 - a3);
        }
        float* yr = y + (int64_t)row[j] * a.F + f;
        if (VEC4) {
            __builtin_nontemporal_store(v, (f4*)yr);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (f + m < a.F) __builtin_nontemporal_store(v[m], yr + m);
        }
    }
}

template <int Q, int LPR, int NI, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_reg(RegArgs a)
{
    reg_body<Q, LPR, NI, VEC4>(a, a.x + (int64_t)blockIdx.y * a.x_stride, a.y + (int64_t)blockIdx.y * a.y_stride,
                               xcd_remap(blockIdx.x, gridDim.x), blockIdx.z);
}

// Every member in one launch (tasks numbered as in k_apply_lean_multi).
struct RegMember {
    const FwdRec* rec;
    int64_t n_rays;
    int64_t x_off, y_off;
    uint32_t blk_begin, nrb;
    int K, F, nk, x_bytes;
    uint32_t mask;
};
struct RegMulti {
    RegMember m[MULTI_MAX];
    int G;
    uint32_t per_vec, total;
    const float* x;
    float* y;
    int64_t x_stride, y_stride;
};

template <int Q, int LPR, int NI, bool VEC4>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_reg_multi(RegMulti a)
{
    for (uint32_t t = blockIdx.x; t < a.total; t += gridDim.x) {
        const uint32_t lt = xcd_remap32(t, a.total);
        const uint32_t v = lt / a.per_vec;
        uint32_t b = lt - v * a.per_vec;
        int g = 0;
        while (g + 1 < a.G && b >= a.m[g + 1].blk_begin) ++g;
        const RegMember& mm = a.m[g];
        b -= mm.blk_begin;
        RegArgs ra;
        ra.rec = mm.rec;
        ra.n_rays = mm.n_rays;
        ra.K = mm.K;
        ra.F = mm.F;
        ra.nk = mm.nk;
        ra.x_bytes = mm.x_bytes;
        ra.mask = mm.mask;
        const uint32_t chunk = b / mm.nrb;
        reg_body<Q, LPR, NI, VEC4>(ra, a.x + (int64_t)v * a.x_stride + mm.x_off,
                                   a.y + (int64_t)v * a.y_stride + mm.y_off, (int64_t)(b - chunk * mm.nrb),
                                   (int)chunk);
    }
}

// --------------------------------------------------------------------------------------------
// A^T, visit-list form (dt_obs/dt_src = 1/Q).  A wave owns cell row ci, a segment of vseg
// columns and a chunk of hats (V per lane).  Its visit list (built at load time) holds, in
// sweep order, every ray that touches the row inside the segment with the row's weights
// already folded in.  The wave reads NB visit records with scalar loads, applies each ray's
// fixed 2Q-tap hat filter (frame f = Q (k - k0) + m, weight 1 - |th0 + m/Q|) to its data row
// and accumulates into two sliding register accumulators (target columns u and u+1).  A
// finished column is written once.
//
// Memory access: one buffer descriptor spans the wave's data vectors and one its output
// vectors.  The uniform part of an address (row or column start, vector) goes into the scalar
// offset; the per-lane part is checked against the row (frames outside [0, F), hats outside
// [0, K), switched-off visits) and replaced by an offset past every range when it fails, so
// such lanes read 0 or drop their store without touching memory.
// --------------------------------------------------------------------------------------------
struct VisitArgs {
    const Visit* visits;
    const int64_t* vtask;
    int n_r, n_phi, K, F, nseg, vseg;
    int kchunks;        // hat chunks per cell row (visit_chunk hats each, one per wave)
    int nvec;           // vectors of the launch (a workgroup takes NVW of them)
    const float* y;
    float* x;
    int64_t y_stride, x_stride;
    uint32_t mask;
    uint32_t y_bytes, x_bytes;   // the member's data and output block of one vector (bytes)
    int64_t ntask;               // base-row form: tasks of the launch (vtask: offsets, then descriptors)
};

// Offset past every buffer range used here (ranges stay below 2^31 - 256, so adding a scalar
// offset below that cannot wrap).
constexpr unsigned VISIT_SENT = 0x7FFFFFF0u;
// Lane-shifted taps with halo lanes: the first H lanes of a chunk load the frames of the H hats
// before it and only feed their neighbours (no extra loads for lane 0).
template <int Q, bool DPP, bool HALO>
struct VisitHalo {
    static constexpr int H = (DPP && HALO) ? (Q == 1 ? 1 : 2) : 0;
};
template <int Q, int V, bool DPP, bool HALO>
constexpr int visit_chunk() { return WAVE * V - VisitHalo<Q, DPP, HALO>::H; }

// Tap weights of one visit: frame f = Q (k - k0) + MLO + t feeds hat k with weight
// 1 - |th0 + (MLO + t)/Q| (zero outside the hat).  Q = 1: taps m = -1, 0.  Q = 2: taps
// m = -4 .. 1 (six, the first always zero) so that frames come in aligned pairs.
template <int Q>
struct Taps {
    static constexpr int MLO = Q == 1 ? -1 : -4;
    static constexpr int T = Q == 1 ? 2 : 6;
    __device__ __forceinline__ static void weights(float th0, float* w)
    {
        if (Q == 1) {
            w[0] = th0;
            w[1] = 1.0f - th0;
        } else {
            const bool hi = th0 >= 0.5f;
            w[0] = 0.f;                                   // m = -4
            w[1] = hi ? th0 - 0.5f : 0.f;                 // m = -3
            w[2] = th0;                                   // m = -2
            w[3] = hi ? 1.5f - th0 : 0.5f + th0;          // m = -1
            w[4] = 1.0f - th0;                            // m =  0
            w[5] = hi ? 0.f : 0.5f - th0;                 // m =  1
        }
    }
};

// One block of the visit-list adjoint: task `lin` = (row group, segment, hat chunk) of one member
// for NVW consecutive vectors (y0, x0: the first of them, already offset to the member's blocks;
// nv of them exist).
// BR = 0: the wave owns RR rows (RR * t .. RR * t + RR - 1).  BR = 1, 2 (base-row form, RR = 2, visit
// set 3): the wave sweeps the rays of base row ci = 2 t + BR - 1 only and writes their sums into
// rows ci and ci + 1; the launch of the even base rows (BR = 1) stores, the following launch of the
// odd base rows (BR = 2) adds to what is there, so each row's value is (even contribution) + (odd
// contribution) in that fixed order and the two launches never touch a row at the same time.
template <int Q, int V, int NB, bool PAIR, int NVW, bool DPP, bool HALO, int RR = 1, int BR = 0>
__device__ __forceinline__ void visit_body(const VisitArgs& a, const float* __restrict__ y0, float* __restrict__ x0,
                                           int nv, int64_t lin)
{
    static_assert(BR == 0 || RR == 2, "the base-row form writes two rows");
    static_assert(!DPP || (Q == 1 && !PAIR) || (Q == 2 && PAIR), "lane-shifted taps: Q = 1, or Q = 2 with frame pairs");
    static_assert(DPP || !HALO, "halo lanes serve the lane-shifted taps");
    typedef Taps<Q> TP_;
    constexpr int T = TP_::T;
    constexpr int H = VisitHalo<Q, DPP, HALO>::H;
    constexpr int C = visit_chunk<Q, V, DPP, HALO>();
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(4))) int64_t* ci64p;
    typedef const __attribute__((address_space(4))) i4v* cvisp;
    const int lane = threadIdx.x & (WAVE - 1);
    // wave index in a scalar register: everything a wave reads from the task and visit
    // tables then comes through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int kch = (int)(lin % a.kchunks);
    const int64_t l2 = lin / a.kchunks;
    const int sg = (int)(l2 % a.nseg), rg = (int)(l2 / a.nseg);
    // RR consecutive rows ci .. ci + RR - 1 whose visits carry weights for each of them
    static_assert(RR == 1 || RR == 2, "rows per wave: 1 or 2");
    const int ti = rg * T_WAVES + wave;
    int ci, jlo, jhi;
    int64_t task;
    if constexpr (BR == 0) {
        if (ti >= (a.n_r + RR - 1) / RR) return;
        ci = RR * ti;
        task = (int64_t)ti * a.nseg + sg;
        jlo = sg * a.vseg;
        jhi = min(jlo + a.vseg, a.n_phi);
    } else {
        // a task of the launch's list (nseg = 1): its base row and columns from its descriptor
        task = ti;
        if (task >= a.ntask) return;
        const int64_t d = ((ci64p)a.vtask)[a.ntask + 1 + task];
        const int cell = (int)(d & 0xFFFFFFFF);
        ci = cell / a.n_phi;
        jlo = cell - ci * a.n_phi;
        jhi = jlo + (int)(d >> 32);
    }
    const int64_t vbeg = ((ci64p)a.vtask)[task], vend = ((ci64p)a.vtask)[task + 1];
    const int ncol = jhi - jlo + 1;
    const int kc = kch * C;              // first output hat of this wave's chunk
    const unsigned rowbytes = (unsigned)a.F * 4u;
    const int lane_off = Q * lane * 4;   // per-lane part of every frame offset

    // descriptors over the wave's vectors: the range ends with the last vector that exists
    auto span = [](const float* p, int64_t stride, uint32_t bytes, int n) {
        const uint64_t base = (uint64_t)p;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        const int nrec = __builtin_amdgcn_readfirstlane((int)((uint32_t)(n - 1) * (uint32_t)stride * 4u + bytes));
        return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0, nrec, 0x00020000);
    };
    const __amdgpu_buffer_rsrc_t ry = span(y0, a.y_stride, a.y_bytes, nv);
    const __amdgpu_buffer_rsrc_t rx = span(x0, a.x_stride, a.x_bytes, nv);
    // scalar offsets of the vectors; missing vectors re-read the first one (their sums are
    // never stored)
    int soy[NVW], sox[NVW];
#pragma unroll
    for (int u = 0; u < NVW; ++u) {
        soy[u] = u < nv ? (int)((uint32_t)u * (uint32_t)a.y_stride * 4u) : 0;
        sox[u] = (int)((uint32_t)u * (uint32_t)a.x_stride * 4u);
    }
    // hats of this lane: kc - H + lane + 64 v.  Frames are fetched for hats below K (halo lanes
    // included); sums are stored for the chunk's own hats below K.
    bool hat_in[V];
    unsigned st_off[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int k = kc - H + lane + WAVE * v;
        hat_in[v] = k < a.K;
        st_off[v] = (k >= kc && k < a.K) ? (unsigned)k * 4u : VISIT_SENT;
    }

    float acc_a[RR][NVW][V], acc_b[RR][NVW][V];   // row ci + r: columns u, u+1 of the sweep
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int u = 0; u < NVW; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) acc_a[r][u][v] = acc_b[r][u][v] = 0.f;
    int col = 0;
    auto emit = [&]() {
        if (col >= 1) {
            const int xo = (ci * a.n_phi + (jlo - 1 + col)) * a.K * 4;   // column start (bytes)
#pragma unroll
            for (int u = 0; u < NVW; ++u) {
                if (u >= nv) break;
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    if (r > 0 && ci + r >= a.n_r) break;
                    const int xr = xo + r * a.n_phi * a.K * 4;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        float val = acc_a[r][u][v];
                        if constexpr (BR == 2)
                            val = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                                rx, (int)st_off[v], sox[u] + xr, 0)) + val;
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, val), rx, (int)st_off[v],
                                                              sox[u] + xr, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int u = 0; u < NVW; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    acc_a[r][u][v] = acc_b[r][u][v];
                    acc_b[r][u][v] = 0.f;
                }
        ++col;
    };
    // byte offset of a frame of the row, or the sentinel when the frame or hat is out of range
    auto frame_off = [&](int fb, bool ok) -> int {
        return (ok && (unsigned)fb < rowbytes) ? fb : (int)VISIT_SENT;
    };

    for (int64_t e0 = vbeg; e0 < vend; e0 += NB) {
        // the batch's visit records, scalar loads (the last batch re-reads its last record for
        // the missing ones, which are then switched off)
        // RR = 1: (row, k0, th0, wa | wb, col, order, -); RR = 2: (row, k0, th0,
        // col | order << 16 | wa0, wb0, wa1, wb1)
        i4v r0[NB], r1[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const cvisp q = (cvisp)(a.visits + min(e0 + j, vend - 1));
            r0[j] = q[0];
            r1[j] = q[1];
        }
        float yv[NB][NVW][V][T], tw[NB][T], wa[NB][RR], wb[NB][RR];
        int vcol[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const bool valid = e0 + j < vend;
            // a vector element is copied to a plain int before its bits are reinterpreted
            // (bit_cast applied to the element expression itself reads element 0)
            const int row = r0[j].x, k0 = r0[j].y, th0_b = r0[j].z;
            int col_j, order;
            if constexpr (RR == 1) {
                const int wa_b = r0[j].w, wb_b = r1[j].x;
                wa[j][0] = __builtin_bit_cast(float, wa_b);
                wb[j][0] = __builtin_bit_cast(float, wb_b);
                col_j = r1[j].y;
                order = r1[j].z;
            } else {
                const int co = r0[j].w;
                const int e0b = r1[j].x, e1b = r1[j].y, e2b = r1[j].z, e3b = r1[j].w;
                col_j = co & 0xFFFF;
                order = co >> 16;
                wa[j][0] = __builtin_bit_cast(float, e0b);
                wb[j][0] = __builtin_bit_cast(float, e1b);
                wa[j][1] = __builtin_bit_cast(float, e2b);
                wb[j][1] = __builtin_bit_cast(float, e3b);
            }
            vcol[j] = valid ? col_j : ncol;
            const bool on = valid && ((a.mask >> order) & 1u);
            TP_::weights(__builtin_bit_cast(float, th0_b), tw[j]);
            const int rowoff = row * a.F * 4;   // start of the data row in the vector (bytes)
            // frame offsets of this visit within the row, identical for every vector
            int off[V][T];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int ub = (Q * (kc - H + WAVE * v - k0) + TP_::MLO) * 4;   // uniform part
#pragma unroll
                for (int t = 0; t < T; ++t) off[v][t] = frame_off(lane_off + ub + 4 * t, on && hat_in[v]);
            }
            // lane 0 of a chunk without halo lanes loads the earlier taps of its hat itself
            int off0[T];
            if constexpr (DPP && !HALO) {
                const int ub0 = (Q * (kc - k0) + TP_::MLO) * 4;
#pragma unroll
                for (int t = 0; t < T; ++t) off0[t] = frame_off(ub0 + 4 * t, on);
            }
#pragma unroll
            for (int u = 0; u < NVW; ++u) {
                const int so = soy[u] + rowoff;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if constexpr (DPP && Q == 1) {
                        // tap m = 0 (frame k - k0) loaded once per lane; tap m = -1 is the previous
                        // lane's, formed in the accumulation
                        yv[j][u][v][1] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(ry, off[v][1], so, 0));
                        if (!HALO && v == 0) {
                            yv[j][u][0][0] = 0.f;
                            if (lane == 0)
                                yv[j][u][0][0] = __builtin_bit_cast(
                                    float, __builtin_amdgcn_raw_buffer_load_b32(ry, off0[0], so, 0));
                        }
                    } else if constexpr (DPP && Q == 2) {
                        // frame pair m = (0, 1) loaded once per lane; pairs (-2, -1) and (-4, -3) are the
                        // pairs (0, 1) of the previous two lanes, formed in the accumulation
                        const f2 p2 = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(ry, off[v][4], so, 0));
                        yv[j][u][v][4] = p2[0];
                        yv[j][u][v][5] = p2[1];
                        if (!HALO && v == 0) {
                            yv[j][u][0][0] = yv[j][u][0][1] = yv[j][u][0][2] = yv[j][u][0][3] = 0.f;
                            if (lane == 0) {
                                const f2 pa = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(ry, off0[2], so, 0));
                                const f2 pb = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(ry, off0[0], so, 0));
                                yv[j][u][0][2] = pa[0];
                                yv[j][u][0][3] = pa[1];
                                yv[j][u][0][0] = pb[0];
                                yv[j][u][0][1] = pb[1];
                            }
                        }
                    } else if (PAIR) {
                        // aligned frame pairs (even F): a pair is inside the row or outside it
#pragma unroll
                        for (int t = 0; t < T; t += 2) {
                            const f2 p2 = __builtin_bit_cast(
                                f2, __builtin_amdgcn_raw_buffer_load_b64(ry, off[v][t], so, 0));
                            yv[j][u][v][t] = p2[0];
                            yv[j][u][v][t + 1] = p2[1];
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < T; ++t)
                            yv[j][u][v][t] = __builtin_bit_cast(
                                float, __builtin_amdgcn_raw_buffer_load_b32(ry, off[v][t], so, 0));
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            while (col < vcol[j]) emit();
            if constexpr (DPP) {
                // earlier taps of lane i are later taps of lanes i - 1 (and i - 2): wave shifts right by
                // one lane.  Lane 0 of a slot takes the previous slot's last lane through a rotation of
                // that slot (the shift's fill value); in the first slot it takes its own extra loads,
                // or, with halo lanes, the rotation itself (halo sums are not stored).
                auto shr1 = [](float old, float src) {
                    return __builtin_bit_cast(
                        float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, src),
                                                           0x138 /* wave_shr:1 */, 0xf, 0xf, false));
                };
                auto ror1 = [](float src) {
                    return __builtin_bit_cast(
                        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, src), 0x13C /* wave_ror:1 */, 0xf, 0xf, false));
                };
#pragma unroll
                for (int u = 0; u < NVW; ++u) {
                    if constexpr (Q == 1) {
                        float o = 0.f;   // fill of the next slot: this slot rotated by one lane
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            float* t = yv[j][u][v];
                            if (v == 0 && HALO) {
                                t[0] = ror1(t[1]);
                                o = t[0];
                            } else {
                                t[0] = shr1(v == 0 ? t[0] : o, t[1]);
                                if (v + 1 < V) o = ror1(t[1]);
                            }
                        }
                    } else {
                        float o4 = 0.f, o5 = 0.f, o2 = 0.f, o3 = 0.f;
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            float* t = yv[j][u][v];
                            if (v == 0 && HALO) {
                                t[2] = ror1(t[4]);
                                t[3] = ror1(t[5]);
                                t[0] = ror1(t[2]);
                                t[1] = ror1(t[3]);
                                o4 = t[2];
                                o5 = t[3];
                                o2 = t[0];
                                o3 = t[1];
                            } else {
                                // slot 0 without halo lanes: fill values are lane 0's own extra loads
                                t[2] = shr1(v == 0 ? t[2] : o4, t[4]);
                                t[3] = shr1(v == 0 ? t[3] : o5, t[5]);
                                t[0] = shr1(v == 0 ? t[0] : o2, t[2]);
                                t[1] = shr1(v == 0 ? t[1] : o3, t[3]);
                                if (v + 1 < V) {
                                    o4 = ror1(t[4]);
                                    o5 = ror1(t[5]);
                                    o2 = ror1(t[2]);
                                    o3 = ror1(t[3]);
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < NVW; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    float h = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t) h += tw[j][t] * yv[j][u][v][t];
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        acc_a[r][u][v] += wa[j][r] * h;
                        acc_b[r][u][v] += wb[j][r] * h;
                    }
                }
        }
    }
    while (col < ncol) emit();
}

// rows (or row pairs, or base rows of one parity) a launch of the visit kernel covers
// wave tasks of one (segment, hat chunk) in a launch of the visit kernel: rows, row pairs, or the
// base-row form's task list
template <int RR, int BR>
__host__ __device__ __forceinline__ int64_t visit_rows(const VisitArgs& a)
{
    return BR == 0 ? (a.n_r + RR - 1) / RR : a.ntask;
}

template <int Q, int V, int NB, bool PAIR, int NVW, bool DPP, bool HALO, int RR, int BR = 0>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint_visit(VisitArgs a)
{
    const int64_t rgroups = (visit_rows<RR, BR>(a) + T_WAVES - 1) / T_WAVES;
    const int v0 = blockIdx.y * NVW;
    visit_body<Q, V, NB, PAIR, NVW, DPP, HALO, RR, BR>(a, a.y + (int64_t)v0 * a.y_stride,
                                                       a.x + (int64_t)v0 * a.x_stride, min(NVW, a.nvec - v0),
                                                       xcd_remap(blockIdx.x, (int64_t)rgroups * a.nseg * a.kchunks));
}

// Every member of a handle (up to MULTI_MAX) in one launch; tasks numbered as in
// k_apply_lean_multi (vector, member, then the member's own task order).
struct VisitMember {
    const Visit* visits;
    const int64_t* vtask;
    int64_t y_off, x_off;
    uint32_t blk_begin;
    int n_r, n_phi, K, F, nseg, vseg, kchunks;
    uint32_t mask;
    uint32_t y_bytes, x_bytes;
};
struct VisitMulti {
    VisitMember m[MULTI_MAX];
    int G;
    int nvec;                    // vectors of the launch (a task takes NVW of them)
    uint32_t per_vec, total;
    const float* y;
    float* x;
    int64_t y_stride, x_stride;
};

template <int Q, int V, int NB, bool PAIR, bool DPP, bool HALO, int RR, int NVW = 1>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint_visit_multi(VisitMulti a)
{
    for (uint32_t t = blockIdx.x; t < a.total; t += gridDim.x) {
        const uint32_t lt = xcd_remap32(t, a.total);
        const uint32_t vg = lt / a.per_vec;          // vector group
        const uint32_t v = vg * NVW;                 // first of the group's NVW vectors
        const uint32_t b = lt - vg * a.per_vec;
        int g = 0;
        while (g + 1 < a.G && b >= a.m[g + 1].blk_begin) ++g;
        const VisitMember& mm = a.m[g];
        VisitArgs va;
        va.visits = mm.visits;
        va.vtask = mm.vtask;
        va.n_r = mm.n_r;
        va.n_phi = mm.n_phi;
        va.K = mm.K;
        va.F = mm.F;
        va.nseg = mm.nseg;
        va.vseg = mm.vseg;
        va.kchunks = mm.kchunks;
        va.mask = mm.mask;
        va.y_stride = a.y_stride;
        va.x_stride = a.x_stride;
        va.y_bytes = mm.y_bytes;
        va.x_bytes = mm.x_bytes;
        visit_body<Q, V, NB, PAIR, NVW, DPP, HALO, RR>(va, a.y + (int64_t)v * a.y_stride + mm.y_off,
                                                   a.x + (int64_t)v * a.x_stride + mm.x_off,
                                                   min(NVW, a.nvec - (int)v), (int64_t)(b - mm.blk_begin));
    }
}

// --------------------------------------------------------------------------------------------
// A^T, row-sweep form (dt_obs/dt_src = 1/Q) for launches over many vectors.  A wave owns a group
// of CW output cell columns and a band of output cell rows of one vector, lanes running over
// the hats (V per lane).  It sweeps the band's base rows in order; for every ray of base row i
// whose stencil reaches its columns (base columns cw0-1 .. cw0+CW-1: one contiguous run of the
// sorted rays, two at the periodic seam) it reads the ray's data row once, applies the ray's
// fixed 2Q-tap hat filter and adds the four bilinear shares into two wave-private LDS rows:
// output row i (top corners) and row i+1 (bottom corners).  Output row i is complete once base
// rows i-1 and i are done: it is written with coalesced stores and its LDS row is cleared for
// row i+2.  The rows are private to the wave and every lane owns its own hats, so plain
// read-add-write updates in program order give bitwise reproducible sums (LDS float atomics
// measured an order of magnitude slower).  A ray next to a column group or band edge is read by
// both neighbours (once per 1/CW and 1/band of the rays).
// --------------------------------------------------------------------------------------------
struct RowsArgs {
    const FwdRec* rec;       // the member's records, sorted by base cell
    const int32_t* cstart;   // the member's CSR over base cells
    int n_r, n_phi, K, F;
    int ngroups, nbands, rb; // column groups, row bands, output rows per band
    const float* y;
    float* x;
    int64_t y_stride, x_stride;
    uint32_t mask;
};

template <int Q, int V, int CW, int NB, bool PAIR>
__device__ __forceinline__ void rows_body(const RowsArgs& a, const float* __restrict__ y, float* __restrict__ x,
                                          int grp, int band)
{
    typedef Taps<Q> TP_;
    constexpr int T = TP_::T;
    constexpr int KP = V * WAVE;
    typedef float f2 __attribute__((ext_vector_type(2)));
    __shared__ float acc_all[T_WAVES][2][CW][KP];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float(*acc)[CW][KP] = acc_all[wave];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl)
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int v = 0; v < V; ++v) acc[sl][c][lane + WAVE * v] = 0.f;
    if (grp >= a.ngroups || band >= a.nbands) return;
    const int n_phi = a.n_phi;
    const int cw0 = grp * CW;
    const int cwe = min(CW, n_phi - cw0);            // columns owned
    const int o0 = band * a.rb, o1 = min(a.n_r, o0 + a.rb);
    const int ib = max(o0 - 1, 0), ie = min(o1, a.n_r - 1);
    const int rowbytes = a.F * 4;
    const int lane_off = Q * lane * 4;
    const int cleft = cw0 == 0 ? n_phi - 1 : cw0 - 1; // base column feeding column cw0 from the left

    // one run of rays [rb0, re0) of base row i; lfix >= -1: the run is base column cw0 + lfix
    // (only for the left neighbour run, lfix = -1), else the local column comes from the record
    auto run = [&](int i, int rb0, int re0, bool left) {
        const int slot = i & 1;
        const bool top = i >= o0, bot = i + 1 < o1;
        for (int e0 = rb0; e0 < re0; e0 += NB) {
            float yv[NB][V][T], tw[NB][T];
            FwdRec rc[NB];
            bool on[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int ri = e0 + j;
                rc[j] = load_const_rec(a.rec + (ri < re0 ? ri : re0 - 1));
                on[j] = ri < re0 && ((a.mask >> rc[j].order) & 1u);
                const uint64_t base = (uint64_t)(y + (int64_t)rc[j].row * a.F);
                const uint32_t blo = __builtin_amdgcn_readfirstlane((uint32_t)base);
                const uint32_t bhi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
                const int nrec = __builtin_amdgcn_readfirstlane(on[j] ? rowbytes : 0);
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(((uint64_t)bhi << 32) | blo), (short)0, nrec, 0x00020000);
                TP_::weights(rc[j].th0, tw[j]);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int ub = (Q * (WAVE * v - rc[j].k0) + TP_::MLO) * 4;
                    if (PAIR) {
#pragma unroll
                        for (int t = 0; t < T; t += 2) {
                            const unsigned off = min((unsigned)(lane_off + ub + 4 * t), 0x7FFFFFF0u);
                            const f2 p2 = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
                            yv[j][v][t] = p2[0];
                            yv[j][v][t + 1] = p2[1];
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < T; ++t) {
                            const unsigned off = min((unsigned)(lane_off + ub + 4 * t), 0x7FFFFFF0u);
                            yv[j][v][t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (!on[j]) continue;
                // local column of the ray's j0 corner; its j1 corner is column lc + 1
                const int lc = left ? -1 : rc[j].cell - (i * n_phi + cw0);
                const bool c0 = lc >= 0, c1 = lc + 1 < cwe;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    float g = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t) g += tw[j][t] * yv[j][v][t];
                    const int k = lane + WAVE * v;
                    if (top && c0) acc[slot][lc][k] += rc[j].b00 * g;
                    if (bot && c0) acc[slot ^ 1][lc][k] += rc[j].b10 * g;
                    if (top && c1) acc[slot][lc + 1][k] += rc[j].b01 * g;
                    if (bot && c1) acc[slot ^ 1][lc + 1][k] += rc[j].b11 * g;
                }
            }
        }
    };
    auto emit_row = [&](int o) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int sl = o & 1;
        for (int c = 0; c < cwe; ++c) {
            float* xr = x + ((int64_t)o * n_phi + cw0 + c) * a.K;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = lane + WAVE * v;
                if (k < a.K) xr[k] = acc[sl][c][k];
                acc[sl][c][k] = 0.f;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    for (int i = ib; i < ie; ++i) {
        const int cb = i * n_phi;
        run(i, a.cstart[cb + cleft], a.cstart[cb + cleft + 1], true);
        run(i, a.cstart[cb + cw0], a.cstart[cb + cw0 + cwe], false);
        if (i >= o0) emit_row(i);
    }
    if (o1 == a.n_r) emit_row(a.n_r - 1);
}

template <int Q, int V, int CW, int NB, bool PAIR>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint_rows(RowsArgs a)
{
    // waves of a workgroup: consecutive column groups of one band (neighbours share rays)
    const int64_t lin = xcd_remap(blockIdx.x, gridDim.x) * T_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = (int)(lin % a.ngroups), band = (int)(lin / a.ngroups);
    rows_body<Q, V, CW, NB, PAIR>(a, a.y + (int64_t)blockIdx.y * a.y_stride, a.x + (int64_t)blockIdx.y * a.x_stride,
                                  grp, band);
}

// --------------------------------------------------------------------------------------------
// A, persistent streaming form.  Work items are (vector, frame chunk, batch of NB rays); each
// XCD owns a contiguous range of items and its waves stride through that range.  Per item the
// wave forms z in LDS from the registers loaded for it, immediately issues the x gathers of its
// next item, and only then streams the current item's rows, so gather latency hides behind the
// stores.
// --------------------------------------------------------------------------------------------
template <int TP, int TQ, int NB, int ZI>
__global__ __launch_bounds__(A_WAVES * WAVE) void k_apply_stream(ApplyArgs a, int fc, int nch, int64_t nbatch,
                                                                 int64_t total)
{
    constexpr int ZW = ZI * WAVE + 4;
    __shared__ float zs_all[A_WAVES][NB][ZW];
    __shared__ int pi_all[A_WAVES][NB][4];
    __shared__ float pf_all[A_WAVES][NB][2];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    float (*zs)[ZW] = zs_all[wave];
    const int K = a.K, F = a.F;
    // XCD x (= blockIdx.x % 8) owns items [x*total/8, (x+1)*total/8)
    const int xcd = blockIdx.x & 7;
    const int64_t bpx = (gridDim.x + 7 - xcd) / 8;            // blocks on this XCD
    const int64_t lw = (int64_t)(blockIdx.x >> 3) * A_WAVES + wave;
    const int64_t nw = bpx * A_WAVES;
    const int64_t beg = total * xcd / 8, end = total * (xcd + 1) / 8;
    int64_t item = beg + lw;
    if (item >= end) return;

    float xv[NB][ZI][4];
    float bw[NB][4];
    int klo[NB], W[NB], k0s[NB], rows[NB];
    float th0s[NB], ws[NB];
    bool act[NB];
    int64_t vec = 0;
    int f0 = 0, fend = 0;

    auto load_item = [&](int64_t it) {
        const int64_t b = it % nbatch;
        const int64_t vc = it / nbatch;
        const int c = (int)(vc % nch);
        vec = vc / nch;
        f0 = c * fc;
        fend = min(F, f0 + fc);
        const float* __restrict__ x = a.x + vec * a.x_stride;
        const int64_t r0 = b * NB;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int64_t ri = r0 + j;
            act[j] = ri < a.n_rays;
            const RayRec rr = a.rays[__builtin_amdgcn_readfirstlane((int)(act[j] ? ri : r0))];
            act[j] = act[j] && ((a.mask >> rr.order) & 1u);
            const int i = rr.cell / a.n_phi;
            const int j0 = rr.cell - i * a.n_phi;
            const int j1 = (j0 + 1 == a.n_phi) ? 0 : j0 + 1;
            klo[j] = frame_step<TP, TQ>(f0, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf;
            W[j] = frame_step<TP, TQ>(fend - 1, rr.k0, rr.th0, a.P, a.Q, a.invQ).kf + 2 - klo[j];
            k0s[j] = rr.k0;
            th0s[j] = rr.th0;
            ws[j] = rr.w;
            rows[j] = rr.row;
            bw[j][0] = (1.0f - rr.fr) * (1.0f - rr.fphi);
            bw[j][1] = rr.fr * (1.0f - rr.fphi);
            bw[j][2] = (1.0f - rr.fr) * rr.fphi;
            bw[j][3] = rr.fr * rr.fphi;
            const int64_t c00 = (int64_t)(i * a.n_phi + j0) * K, c10 = (int64_t)((i + 1) * a.n_phi + j0) * K;
            const int64_t c01 = (int64_t)(i * a.n_phi + j1) * K, c11 = (int64_t)((i + 1) * a.n_phi + j1) * K;
#pragma unroll
            for (int q = 0; q < ZI; ++q) {
                const int jj = lane + q * WAVE;
                const int kk = min(max(klo[j] + jj, 0), K - 1);   // clamped: always a valid address
                xv[j][q][0] = x[c00 + kk];
                xv[j][q][1] = x[c10 + kk];
                xv[j][q][2] = x[c01 + kk];
                xv[j][q][3] = x[c11 + kk];
            }
        }
    };

    load_item(item);
    for (;;) {
        // z of the current item into LDS (zero outside the hat range and for inactive rays)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
#pragma unroll
            for (int q = 0; q < ZI; ++q) {
                const int jj = lane + q * WAVE;
                const int k = klo[j] + jj;
                const bool ok = act[j] && k >= 0 && k < K;
                if (jj < W[j])
                    zs[j][jj] = ok ? bw[j][0] * xv[j][q][0] + bw[j][1] * xv[j][q][1] + bw[j][2] * xv[j][q][2] +
                                         bw[j][3] * xv[j][q][3]
                                   : 0.f;
            }
            if (lane == 0) {
                pi_all[wave][j][0] = klo[j];
                pi_all[wave][j][1] = k0s[j];
                pi_all[wave][j][2] = rows[j];
                pi_all[wave][j][3] = act[j] ? 1 : 0;
                pf_all[wave][j][0] = th0s[j];
                pf_all[wave][j][1] = ws[j];
            }
        }
        const int64_t cur_vec = vec;
        const int cf0 = f0, cfend = fend;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t next = item + nw;
        const bool has_next = next < end;
        if (has_next) load_item(next);   // gathers of the next item fly while this one is stored
        float* __restrict__ y = a.y + cur_vec * a.y_stride;
        const bool vec4 = ((F & 3) == 0) && ((cfend - cf0) & 3) == 0 && ((((uintptr_t)y) & 15) == 0);
        if (vec4) {
            const int ng = (cfend - cf0) >> 2;
            for (int g = lane; g < NB * ng; g += WAVE) {
                const int j = g / ng, q = g - j * ng;
                if (!pi_all[wave][j][3]) continue;
                const int kl = pi_all[wave][j][0], k0 = pi_all[wave][j][1];
                const float th0 = pf_all[wave][j][0], w = pf_all[wave][j][1];
                const int f = cf0 + 4 * q;
                f4 v;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const FrameStep st = frame_step<TP, TQ>(f + t, k0, th0, a.P, a.Q, a.invQ);
                    const int jz = st.kf - kl;
                    v[t] = w * ((1.0f - st.th) * zs[j][jz] + st.th * zs[j][jz + 1]);
                }
                __builtin_nontemporal_store(v, (f4*)(y + (int64_t)pi_all[wave][j][2] * F + f));
            }
        } else {
            const int ng = cfend - cf0;
            for (int g = lane; g < NB * ng; g += WAVE) {
                const int j = g / ng, q = g - j * ng;
                if (!pi_all[wave][j][3]) continue;
                const int kl = pi_all[wave][j][0], k0 = pi_all[wave][j][1];
                const float th0 = pf_all[wave][j][0], w = pf_all[wave][j][1];
                const int f = cf0 + q;
                const FrameStep st = frame_step<TP, TQ>(f, k0, th0, a.P, a.Q, a.invQ);
                const int jz = st.kf - kl;
                __builtin_nontemporal_store(w * ((1.0f - st.th) * zs[j][jz] + st.th * zs[j][jz + 1]),
                                            y + (int64_t)pi_all[wave][j][2] * F + f);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (!has_next) break;
        item = next;
    }
}

// --------------------------------------------------------------------------------------------
// A^T, sweep form.  A wave owns one cell row ci, a column segment [jlo, jhi) and 64*V hats.
// The cells of row ci are corners of rays whose base row is ci-1 (their upper corners, radial
// weight fr) or ci (lower corners, weight 1-fr).  The wave sweeps the base columns
// u = jlo-1 .. jhi-1; the rays of base column u feed target columns u (azimuthal weight
// 1-fphi) and u+1 (weight fphi).  Two register accumulators per hat hold target columns u and
// u+1; when the sweep leaves base column u, column u is complete and written once.  Ray records
// and data loads are issued NB rays at a time.  No atomics, no LDS, deterministic.
// --------------------------------------------------------------------------------------------
template <int TP, int TQ, int TC, int V, int NB>
__global__ __launch_bounds__(T_WAVES * WAVE) void k_adjoint_sweep(AdjArgs a)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int segs = (a.n_phi + TC - 1) / TC;
    const int kchunks = (a.K + WAVE * V - 1) / (WAVE * V);
    const int rgroups = (a.n_r + T_WAVES - 1) / T_WAVES;
    const int64_t lin = xcd_remap(blockIdx.x, (int64_t)rgroups * segs * kchunks);
    const int kch = (int)(lin % kchunks);
    const int64_t t2 = lin / kchunks;
    const int seg = (int)(t2 % segs), rg = (int)(t2 / segs);
    const int ci = rg * T_WAVES + wave;
    if (ci >= a.n_r) return;
    const int jlo = seg * TC, jhi = min(jlo + TC, a.n_phi);
    const int ncol = jhi - jlo + 1;   // base columns jlo-1 .. jhi-1
    const int kc = kch * WAVE * V;
    const float* __restrict__ y = a.y + (int64_t)blockIdx.y * a.y_stride;
    float* __restrict__ x = a.x + (int64_t)blockIdx.y * a.x_stride;

    // per-lane column table: lane c describes base column u = jlo - 1 + c
    int st0 = 0, ln0 = 0, st1 = 0, ln1 = 0;
    if (lane < ncol) {
        const int u = jlo - 1 + lane;
        const int ub = (u + a.n_phi) % a.n_phi;
        if (ci >= 1) {
            const int c = (ci - 1) * a.n_phi + ub;
            st0 = a.cstart[c];
            ln0 = a.cstart[c + 1] - st0;
        }
        if (ci <= a.n_r - 2) {
            const int c = ci * a.n_phi + ub;
            st1 = a.cstart[c];
            ln1 = a.cstart[c + 1] - st1;
        }
    }
    const int cnt = ln0 + ln1;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int o = __shfl_up(incl, d, WAVE);
        if (lane >= d) incl += o;
    }
    const int total = __shfl(incl, WAVE - 1, WAVE);

    float acc_a[V], acc_b[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc_a[v] = acc_b[v] = 0.f;
    int col = 0;   // base column index whose target columns acc_a (u) and acc_b (u+1) hold

    auto emit = [&]() {
        // target column u = jlo - 1 + col is complete
        if (col >= 1) {
            const int u = jlo - 1 + col;
            float* xr = x + (int64_t)(ci * a.n_phi + u) * a.K;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = kc + lane + WAVE * v;
                if (k < a.K) xr[k] = acc_a[v];
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc_a[v] = acc_b[v];
            acc_b[v] = 0.f;
        }
        ++col;
    };

    for (int e0 = 0; e0 < total; e0 += NB) {
        int cj[NB];
        float hv[NB][V], wa[NB], wb[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int e = e0 + j;
            const bool valid = e < total;
            const int ee = valid ? e : total - 1;
            const int c = __popcll(__ballot(incl <= ee));
            const int inc_c = __shfl(incl, c, WAVE), cnt_c = __shfl(cnt, c, WAVE);
            const int l0c = __shfl(ln0, c, WAVE);
            const int o = ee - (inc_c - cnt_c);
            const bool upper = o < l0c;   // base row ci-1
            const int ri = upper ? __shfl(st0, c, WAVE) + o : __shfl(st1, c, WAVE) + (o - l0c);
            const RayRec rr = a.rays[__builtin_amdgcn_readfirstlane(ri)];
            const bool on = valid && ((a.mask >> rr.order) & 1u);
            cj[j] = valid ? c : ncol;
            const float wr = upper ? rr.fr : 1.0f - rr.fr;
            wa[j] = on ? rr.w * wr * (1.0f - rr.fphi) : 0.f;
            wb[j] = on ? rr.w * wr * rr.fphi : 0.f;
            const float* __restrict__ yrow = y + (int64_t)rr.row * a.F;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = kc + lane + WAVE * v;
                hv[j][v] = 0.f;
                if (TP == 1 && TQ == 1) {
                    const int f = k - rr.k0;
                    const bool ok1 = f >= 0 && f < a.F, ok2 = f >= 1 && f <= a.F;
                    const float y1 = yrow[min(max(f, 0), a.F - 1)];
                    const float y2 = yrow[min(max(f - 1, 0), a.F - 1)];
                    hv[j][v] = (ok1 ? (1.0f - rr.th0) * y1 : 0.f) + (ok2 ? rr.th0 * y2 : 0.f);
                } else {
                    hv[j][v] = hat_gather<TP, TQ>(yrow, k, rr.k0, rr.th0, a.F, a.P, a.Q, a.invQ);
                }
                if (k >= a.K) hv[j][v] = 0.f;
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            while (col < cj[j]) emit();
#pragma unroll
            for (int v = 0; v < V; ++v) {
                acc_a[v] += wa[j] * hv[j][v];
                acc_b[v] += wb[j] * hv[j][v];
            }
        }
    }
    while (col < ncol) emit();
}

// --------------------------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------------------------
// Adjoint variants: 0-2 LDS tile kernels, 3-6 sweep kernels (TC column segment, V hats per lane),
// 7-10 batched LDS tile kernels, 11 visit-list kernel (dt_obs/dt_src = 1 or 1/2).
struct AdjVariant {
    const char* name;
    int kind;   // 0 tile, 1 sweep, 2 batched tile, 3 visit list, 4 row sweep
    int a, b;   // tile: TR, TC; sweep: TC, V; visit list: vectors per wave, lane-shifted taps; row sweep: CW
};
static const AdjVariant kAdjVariants[] = {
    {"tile8x8", 0, 8, 8},    {"tile4x8", 0, 4, 8},    {"tile4x4", 0, 4, 4},    {"sweep32v1", 1, 32, 1},
    {"sweep32v2", 1, 32, 2}, {"sweep16v1", 1, 16, 1}, {"sweep16v2", 1, 16, 2}, {"tb8x8", 2, 8, 8},
    {"tb4x8", 2, 4, 8},      {"tb4x4", 2, 4, 4},      {"tb2x4", 2, 2, 4},      {"visit", 3, 0, 0},
    {"rows4", 4, 4, 0},      {"rows8", 4, 8, 0},      {"visit2v", 3, 2, 0},    {"visit4v", 3, 4, 0},
    {"visitd", 3, 1, 1},     {"visitd2v", 3, 2, 1},   {"visitd4v", 3, 4, 1},   {"visitp2v", 3, 2, 2},
    {"visitp4v", 3, 4, 2},   {"visitb", 3, 1, 3},     {"visitb2v", 3, 2, 3},
};
constexpr int kNumAdj = sizeof(kAdjVariants) / sizeof(kAdjVariants[0]);

int n_adjoint_variants() { return kNumAdj; }
const char* adjoint_variant_name(int v) { return kAdjVariants[v].name; }
int n_apply_variants() { return 15; }
const char* apply_variant_name(int v)
{
    static const char* names[] = {"rpw1", "rpw2", "batch", "stream", "lean4", "lean8", "reg1", "reg2", "strip16",
                                  "strip8", "lean4q", "abs4", "abs8", "lean4r", "abs4r"};
    return names[v];
}
bool lean_supported(const Member& m)
{
    return m.P == 1 && (m.Q == 1 || m.Q == 2) && (int64_t)m.grid.n_r * m.grid.n_phi * m.grid.n_hat < (1ll << 29);
}

bool visit_supported(const Member& m) { return m.P == 1 && (m.Q == 1 || m.Q == 2); }

bool adjoint_variant_ok(const Member& m, int v)
{
    if (v < 0 || v >= n_adjoint_variants()) return false;
    if ((v == 11 || v >= 14) && !visit_supported(m)) return false;
    if ((v == 12 || v == 13) && !(visit_supported(m) && m.grid.n_hat <= 4 * WAVE)) return false;   // rows: K <= 256
    return true;
}

// LDS bytes of the strip forward with strips of sc base cells (staged corner rows + z rows)
static int64_t strip_lds_bytes(const Member& m, int sc)
{
    const int fcq = 128;   // hats per frame chunk (128 Q frames at ratio 1/Q)
    const int64_t w = std::min<int64_t>(m.grid.n_hat, (int64_t)m.k0_max - m.k0_min + fcq + 2);
    const int64_t zs = (int64_t)A_WAVES * 4 * (((fcq + 4) + WAVE - 1) / WAVE * WAVE);
    return 4 * (2 * (int64_t)(sc + 1) * std::max<int64_t>(w, 1) + zs);
}

bool apply_variant_ok(const Member& m, int v)
{
    if (v < 0 || v >= n_apply_variants()) return false;
    if ((v == 2 || v == 3) && m.P > m.Q) return false;   // batch / stream need dt_obs <= dt_src
    if (v >= 4 && !lean_supported(m)) return false;      // lean / reg / strip need dt_obs/dt_src = 1 or 1/2
    if ((v == 8 || v == 9) && strip_lds_bytes(m, v == 8 ? 16 : 8) > 65536) return false;
    if (v == 10 && m.grid.n_hat % 4 != 0) return false;   // quad gathers need 16-byte aligned x rows
    if ((v == 11 || v == 12 || v == 14) && m.grid.n_hat > ABS_KMAX) return false;   // absolute hats: two gather passes
    return true;
}

// Lanes per ray of the register forward (frames per chunk = 4 * LPR) for rows of F frames: the
// chunk that wastes the fewest lanes, the longer one on ties.
static int reg_lpr(int64_t F)
{
    int best = 64;
    int64_t waste = INT64_MAX;
    for (int lpr : {64, 32, 16}) {
        const int64_t fc = 4 * lpr, w = (F + fc - 1) / fc * fc - F;
        if (w < waste) {
            waste = w;
            best = lpr;
        }
    }
    return best;
}

int default_adjoint_variant(const Member& m)
{
    if (visit_supported(m)) return 11;
    return 2;
}
int default_apply_variant(const Member& m) { return lean_supported(m) ? 4 : (m.P <= m.Q ? 2 : 1); }

template <int TP, int TQ, int NB, int ZI>
static void apply_batch_launch(const ApplyArgs& a, int nvec, hipStream_t s)
{
    // frames per chunk: the chunk's hat window (<= floor((fc-1)P/Q) + 4) must fit ZI*64
    const int P = a.P, Q = a.Q;
    int fc = a.F;
    const int64_t span = (int64_t)(fc - 1) * P / Q + 4;
    if (span > (int64_t)ZI * WAVE) {
        fc = (int)(((int64_t)ZI * WAVE - 4) * Q / P) + 1;
        fc &= ~3;
    }
    const int nch = (a.F + fc - 1) / fc;
    const int64_t rays_per_block = (int64_t)A_WAVES * NB;
    dim3 grid((unsigned)((a.n_rays + rays_per_block - 1) / rays_per_block), (unsigned)nvec, (unsigned)nch);
    hipLaunchKernelGGL((k_apply_batch<TP, TQ, NB, ZI>), grid, dim3(A_WAVES * WAVE), 0, s, a, fc);
}

template <int TP, int TQ, int NB, int ZI>
static void apply_stream_launch(const ApplyArgs& a, int nvec, hipStream_t s)
{
    const int P = a.P, Q = a.Q;
    int fc = a.F;
    const int64_t span = (int64_t)(fc - 1) * P / Q + 4;
    if (span > (int64_t)ZI * WAVE) {
        fc = (int)(((int64_t)ZI * WAVE - 4) * Q / P) + 1;
        fc &= ~3;
    }
    const int nch = (a.F + fc - 1) / fc;
    const int64_t nbatch = (a.n_rays + NB - 1) / NB;
    const int64_t total = nbatch * nch * nvec;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t blocks = std::min<int64_t>((int64_t)cus * 8, (total + A_WAVES - 1) / A_WAVES);
    blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((k_apply_stream<TP, TQ, NB, ZI>), dim3((unsigned)blocks), dim3(A_WAVES * WAVE), 0, s, a, fc,
                       nch, nbatch, total);
}

template <int TP, int TQ>
static void apply_dispatch(const ApplyArgs& a, int nvec, int variant, hipStream_t s)
{
    if (variant == 3 && a.P <= a.Q) {
        const int64_t span = (int64_t)(a.F - 1) * a.P / a.Q + 4;
        if (span <= 2 * WAVE) apply_stream_launch<TP, TQ, 4, 2>(a, nvec, s);
        else if (span <= 3 * WAVE) apply_stream_launch<TP, TQ, 4, 3>(a, nvec, s);
        else apply_stream_launch<TP, TQ, 2, 5>(a, nvec, s);
        return;
    }
    if (variant == 2 && a.P <= a.Q) {
        const int64_t span = (int64_t)(a.F - 1) * a.P / a.Q + 4;
        if (span <= 2 * WAVE) apply_batch_launch<TP, TQ, 4, 2>(a, nvec, s);
        else if (span <= 3 * WAVE) apply_batch_launch<TP, TQ, 4, 3>(a, nvec, s);
        else apply_batch_launch<TP, TQ, 2, 5>(a, nvec, s);
        return;
    }
    const int rpw = variant == 1 ? 2 : 1;
    const int64_t rays_per_block = (int64_t)A_WAVES * rpw;
    dim3 grid((unsigned)((a.n_rays + rays_per_block - 1) / rays_per_block), (unsigned)nvec);
    if (rpw == 2)
        hipLaunchKernelGGL((k_apply<TP, TQ, 2>), grid, dim3(A_WAVES * WAVE), 0, s, a);
    else
        hipLaunchKernelGGL((k_apply<TP, TQ, 1>), grid, dim3(A_WAVES * WAVE), 0, s, a);
}

// Frame chunks of the lean forward: the fewest chunks of at most lean_fcmax(Q) frames, of equal
// length rounded up to a multiple of 4 (chunk starts stay 16-byte aligned within a row).
static void lean_chunks(int F, int Q, int* nch, int* fc)
{
    const int mx = Q == 1 ? lean_fcmax(1) : lean_fcmax(2);
    *nch = std::max(1, (F + mx - 1) / mx);
    *fc = ((F + *nch - 1) / *nch + 3) / 4 * 4;
}

template <int Q, int NB, bool QUAD = false>
static void lean_launch(LeanArgs a, int nvec, bool vec4, hipStream_t s)
{
    const int64_t rays_per_block = (int64_t)A_WAVES * NB;
    int nch = (a.F + 128 * Q - 1) / (128 * Q);   // the quad-gather form keeps chunks of 128 Q frames
    if (!QUAD) lean_chunks(a.F, Q, &nch, &a.fc);
    dim3 grid((unsigned)((a.n_rays + rays_per_block - 1) / rays_per_block), (unsigned)nvec, (unsigned)nch);
    if (QUAD) {
        if (vec4) hipLaunchKernelGGL((k_apply_leanq<Q, NB, true>), grid, dim3(A_WAVES * WAVE), 0, s, a);
        else hipLaunchKernelGGL((k_apply_leanq<Q, NB, false>), grid, dim3(A_WAVES * WAVE), 0, s, a);
        return;
    }
    if (vec4) hipLaunchKernelGGL((k_apply_lean<Q, NB, true>), grid, dim3(A_WAVES * WAVE), 0, s, a);
    else hipLaunchKernelGGL((k_apply_lean<Q, NB, false>), grid, dim3(A_WAVES * WAVE), 0, s, a);
}

template <int Q, int LPR, int NI>
static void reg_launch(const RegArgs& a, int nvec, bool vec4, hipStream_t s)
{
    constexpr int64_t rays_per_block = (int64_t)A_WAVES * (WAVE / LPR) * NI;
    const int nch = (a.F + 4 * LPR - 1) / (4 * LPR);
    dim3 grid((unsigned)((a.n_rays + rays_per_block - 1) / rays_per_block), (unsigned)nvec, (unsigned)nch);
    if (vec4) hipLaunchKernelGGL((k_apply_reg<Q, LPR, NI, true>), grid, dim3(A_WAVES * WAVE), 0, s, a);
    else hipLaunchKernelGGL((k_apply_reg<Q, LPR, NI, false>), grid, dim3(A_WAVES * WAVE), 0, s, a);
}

template <int Q, int NI>
static void reg_dispatch(const RegArgs& a, int nvec, bool vec4, hipStream_t s)
{
    switch (reg_lpr(a.F)) {
    case 16: reg_launch<Q, 16, NI>(a, nvec, vec4, s); break;
    case 32: reg_launch<Q, 32, NI>(a, nvec, vec4, s); break;
    default: reg_launch<Q, 64, NI>(a, nvec, vec4, s); break;
    }
}

int launch_apply(const rtt_geometry* g, const Member& m, const float* x, float* y, int nvec,
                 int64_t x_stride, int64_t y_stride, uint32_t mask, hipStream_t s, int variant)
{
    if (m.n_rays == 0 || nvec == 0) return RTT_OK;
    if (variant < 0 || variant >= n_apply_variants()) variant = m.apply_variant;
    if (!apply_variant_ok(m, variant)) variant = m.P <= m.Q ? 2 : 1;
    if (variant == 8 || variant == 9) {
        StripArgs sa;
        sa.rec = g->d_fwd + m.ray_begin;
        sa.cstart = g->d_cell_start + m.cell_begin;
        sa.n_r = m.grid.n_r;
        sa.n_phi = m.grid.n_phi;
        sa.K = m.grid.n_hat;
        sa.F = m.grid.n_frames;
        sa.SC = variant == 8 ? 16 : 8;
        sa.nstrip = (sa.n_phi + sa.SC - 1) / sa.SC;
        sa.w_alloc = (int)std::max<int64_t>(1, std::min<int64_t>(sa.K, (int64_t)m.k0_max - m.k0_min + 130));
        sa.k0min = m.k0_min;
        sa.k0max = m.k0_max;
        sa.x = x;
        sa.y = y;
        sa.x_stride = x_stride;
        sa.y_stride = y_stride;
        sa.mask = mask;
        const bool vec4 = (sa.F % 4) == 0 && (((uintptr_t)y) & 15) == 0 && (nvec == 1 || (y_stride % 4) == 0);
        const int nch = (sa.F + 128 * m.Q - 1) / (128 * m.Q);
        const dim3 grid((unsigned)((int64_t)(sa.n_r - 1) * sa.nstrip), (unsigned)nvec, (unsigned)nch);
        const size_t lds = (size_t)strip_lds_bytes(m, sa.SC);
        if (m.Q == 1) {
            if (vec4) hipLaunchKernelGGL((k_apply_strip<1, 4, true>), grid, dim3(A_WAVES * WAVE), lds, s, sa);
            else hipLaunchKernelGGL((k_apply_strip<1, 4, false>), grid, dim3(A_WAVES * WAVE), lds, s, sa);
        } else {
            if (vec4) hipLaunchKernelGGL((k_apply_strip<2, 4, true>), grid, dim3(A_WAVES * WAVE), lds, s, sa);
            else hipLaunchKernelGGL((k_apply_strip<2, 4, false>), grid, dim3(A_WAVES * WAVE), lds, s, sa);
        }
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    if (variant == 6 || variant == 7) {
        RegArgs ra;
        ra.rec = g->d_fwd + m.ray_begin;
        ra.n_rays = m.n_rays;
        ra.K = m.grid.n_hat;
        ra.F = m.grid.n_frames;
        ra.nk = m.grid.n_phi * m.grid.n_hat;
        ra.x_bytes = (int)(m.n_cols * 4);
        ra.x = x;
        ra.y = y;
        ra.x_stride = x_stride;
        ra.y_stride = y_stride;
        ra.mask = mask;
        const bool vec4 = (ra.F % 4) == 0 && (((uintptr_t)y) & 15) == 0 && (nvec == 1 || (y_stride % 4) == 0);
        if (m.Q == 1) {
            if (variant == 6) reg_dispatch<1, 1>(ra, nvec, vec4, s);
            else reg_dispatch<1, 2>(ra, nvec, vec4, s);
        } else {
            if (variant == 6) reg_dispatch<2, 1>(ra, nvec, vec4, s);
            else reg_dispatch<2, 2>(ra, nvec, vec4, s);
        }
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    if (variant == 11 || variant == 12 || variant == 14) {
        if (m.grid.n_hat > ABS_KMAX) return fail(RTT_EINVAL, "absolute-hat forward needs n_hat <= 128");
        LeanArgs la;
        // abs4r: the records in data-row order, consecutive rows staged (Q = 1)
        la.rec = (variant == 14 ? g->d_fwd_row : g->d_fwd) + m.ray_begin;
        la.n_rays = m.n_rays;
        la.K = m.grid.n_hat;
        la.F = m.grid.n_frames;
        la.nk = m.grid.n_phi * m.grid.n_hat;
        la.x = x;
        la.y = y;
        la.x_stride = x_stride;
        la.y_stride = y_stride;
        la.x_bytes = (int)(m.n_cols * 4);
        la.mask = mask;
        la.fc = m.grid.n_frames;
        const int wa = m.Q == 1 ? 2 : 4;
        const bool vec4 = (la.F % wa) == 0 && (((uintptr_t)y) & (4 * wa - 1)) == 0 && (nvec == 1 || (y_stride % wa) == 0);
        const int nb = variant == 12 ? 8 : 4;
        const dim3 grid((unsigned)((la.n_rays + (int64_t)A_WAVES * nb - 1) / ((int64_t)A_WAVES * nb)), (unsigned)nvec);
        const dim3 blk(A_WAVES * WAVE);
#define RTT_ABS(Q_, NB_)                                                                      \
    do {                                                                                      \
        if (vec4) hipLaunchKernelGGL((k_apply_abs<Q_, NB_, true>), grid, blk, 0, s, la);      \
        else hipLaunchKernelGGL((k_apply_abs<Q_, NB_, false>), grid, blk, 0, s, la);          \
    } while (0)
        if (variant == 14 && m.Q == 1) {
            if (vec4) hipLaunchKernelGGL((k_apply_abs<1, 4, true, true>), grid, blk, 0, s, la);
            else hipLaunchKernelGGL((k_apply_abs<1, 4, false, true>), grid, blk, 0, s, la);
        } else if (m.Q == 1) {
            if (nb == 4) RTT_ABS(1, 4);
            else RTT_ABS(1, 8);
        } else {
            if (nb == 4) RTT_ABS(2, 4);
            else RTT_ABS(2, 8);
        }
#undef RTT_ABS
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    // quad gathers read 16-byte words: they need 16-byte aligned coefficient vectors
    if (variant == 10 && ((((uintptr_t)x) & 15) != 0 || (nvec > 1 && (x_stride % 4) != 0))) variant = 4;
    // lean4r: the lean forward over the records in data-row order
    if (variant == 4 || variant == 5 || variant == 10 || variant == 13) {
        LeanArgs la;
        la.rec = (variant == 13 ? g->d_fwd_row : g->d_fwd) + m.ray_begin;
        la.n_rays = m.n_rays;
        la.K = m.grid.n_hat;
        la.F = m.grid.n_frames;
        la.nk = m.grid.n_phi * m.grid.n_hat;
        la.x = x;
        la.y = y;
        la.x_stride = x_stride;
        la.y_stride = y_stride;
        la.x_bytes = (int)(m.n_cols * 4);
        la.mask = mask;
        la.fc = 128 * m.Q;
        // wide output stores: 8-byte aligned rows at Q = 1 (F even), 16-byte at Q = 2 (F % 4 == 0)
        const int wa = m.Q == 1 ? 2 : 4;
        const bool vec4 = (la.F % wa) == 0 && (((uintptr_t)y) & (4 * wa - 1)) == 0 && (nvec == 1 || (y_stride % wa) == 0);
        if (m.Q == 1) {
            if (variant == 10) lean_launch<1, 4, true>(la, nvec, vec4, s);
            else if (variant == 4 || variant == 13) lean_launch<1, 4>(la, nvec, vec4, s);
            else lean_launch<1, 8>(la, nvec, vec4, s);
        } else {
            if (variant == 10) lean_launch<2, 4, true>(la, nvec, vec4, s);
            else if (variant == 4 || variant == 13) lean_launch<2, 4>(la, nvec, vec4, s);
            else lean_launch<2, 8>(la, nvec, vec4, s);
        }
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
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

template <int TR, int TC>
static void adjoint_dispatch_tb(const AdjArgs& a, int P, int Q, int nvec, hipStream_t s)
{
    constexpr int NB = 8;
    const int64_t tiles = (int64_t)((a.n_r + TR - 1) / TR) * ((a.n_phi + TC - 1) / TC) * ((a.K + KC - 1) / KC);
    dim3 grid((unsigned)tiles, (unsigned)nvec);
    if (P == 1 && Q == 1)
        hipLaunchKernelGGL((k_adjoint_tb<TR, TC, 1, 1, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else if (P == 1 && Q == 2)
        hipLaunchKernelGGL((k_adjoint_tb<TR, TC, 1, 2, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint_tb<TR, TC, 0, 0, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
}

template <int TC, int V>
static void adjoint_dispatch_sweep(const AdjArgs& a, int P, int Q, int nvec, hipStream_t s)
{
    constexpr int NB = 8;
    const int64_t work = (int64_t)((a.n_r + T_WAVES - 1) / T_WAVES) * ((a.n_phi + TC - 1) / TC) *
                         ((a.K + WAVE * V - 1) / (WAVE * V));
    dim3 grid((unsigned)work, (unsigned)nvec);
    if (P == 1 && Q == 1)
        hipLaunchKernelGGL((k_adjoint_sweep<1, 1, TC, V, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else if (P == 1 && Q == 2)
        hipLaunchKernelGGL((k_adjoint_sweep<1, 2, TC, V, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint_sweep<0, 0, TC, V, NB>), grid, dim3(T_WAVES * WAVE), 0, s, a);
}

// The visit kernel addresses the data and output vectors of a wave through one buffer range
// each: nvw vectors (stride in floats) of a member's n_rows data and n_cols output floats must
// span less than 2^31 - 256 bytes.
static bool visit_fits(int64_t n_rows, int64_t n_cols, int64_t y_stride, int64_t x_stride, int nvw)
{
    const int64_t lim = (int64_t)VISIT_SENT - 240;
    return (int64_t)(nvw - 1) * y_stride * 4 + n_rows * 4 <= lim && (int64_t)(nvw - 1) * x_stride * 4 + n_cols * 4 <= lim;
}

// Halo lanes (lane-shifted taps) when they cost no extra hat chunk: K hats in as many chunks of
// 64 V - H hats as of 64 V.
template <int Q, int V>
static bool visit_halo_fits(int K)
{
    constexpr int C = visit_chunk<Q, V, true, true>();
    return (K + C - 1) / C == (K + WAVE * V - 1) / (WAVE * V);
}

template <int Q, int V, int NB, bool PAIR, int NVW, bool DPP = false, bool HALO = false, int RR = 1, int BR = 0>
static void visit_launch(VisitArgs a, int nvec, hipStream_t s)
{
    if constexpr (DPP && !HALO) {
        if (visit_halo_fits<Q, V>(a.K)) {
            visit_launch<Q, V, NB, PAIR, NVW, true, true, RR, BR>(a, nvec, s);
            return;
        }
    }
    constexpr int C = visit_chunk<Q, V, DPP, HALO>();
    a.kchunks = (a.K + C - 1) / C;
    a.nvec = nvec;
    const int64_t rows = visit_rows<RR, BR>(a);
    if (rows <= 0) return;
    const int64_t blocks = ((rows + T_WAVES - 1) / T_WAVES) * a.nseg * a.kchunks;
    hipLaunchKernelGGL((k_adjoint_visit<Q, V, NB, PAIR, NVW, DPP, HALO, RR, BR>),
                       dim3((unsigned)blocks, (unsigned)((nvec + NVW - 1) / NVW)), dim3(T_WAVES * WAVE), 0, s, a);
}

// Base-row form (visit set 3, lane-shifted taps): the tasks of the even base rows store, then
// those of the odd base rows add (two launches on one stream).  vpw vectors per wave; one hat slot
// per lane unless the launch has enough waves without splitting the hats.
template <int Q, int V, int NB, int NVW>
static void visitb_pass(VisitArgs a, const int64_t* vtask0, int64_t ntask0, const int64_t* vtask1, int64_t ntask1,
                        int nvec, hipStream_t s)
{
    constexpr bool P = Q == 2;
    a.nseg = 1;
    a.vtask = vtask0;
    a.ntask = ntask0;
    visit_launch<Q, V, NB, P, NVW, true, false, 2, 1>(a, nvec, s);
    a.vtask = vtask1;
    a.ntask = ntask1;
    visit_launch<Q, V, NB, P, NVW, true, false, 2, 2>(a, nvec, s);
}

template <int Q>
static void visitb_dispatch(const VisitArgs& a, const int64_t* vtask0, int64_t ntask0, const int64_t* vtask1,
                            int64_t ntask1, int nvec, int vpw, hipStream_t s)
{
    const int64_t waves = ntask0 * ((nvec + vpw - 1) / vpw);
#define RTT_VISITB(V_, NB_, NVW_) visitb_pass<Q, V_, NB_, NVW_>(a, vtask0, ntask0, vtask1, ntask1, nvec, s)
    if (vpw == 2) {
        if (a.K <= 64 || waves < 16384) RTT_VISITB(1, 4, 2);
        else if (a.K <= 128) RTT_VISITB(2, 4, 2);
        else RTT_VISITB(4, 2, 2);
        return;
    }
    // at half-step frames (Q = 2) a visit feeds two frames per hat, and four hats per lane pay for
    // the visit's set-up even when the launch has few waves (512^2 geometry, one vector: 0.204 ->
    // 0.147 ms); at Q = 1 one hat per lane stays faster there (256^2: 0.078 against 0.14 ms)
    if (Q == 2 && a.K > 128) RTT_VISITB(4, 2, 1);
    else if (a.K <= 64 || waves < 16384) RTT_VISITB(1, 4, 1);
    else if (a.K <= 128) RTT_VISITB(2, 4, 1);
    else RTT_VISITB(4, 2, 1);
#undef RTT_VISITB
}

// lane-shifted taps (Q = 1, or Q = 2 with frame pairs); vpw vectors per wave
template <int Q>
static void visitd_dispatch(const VisitArgs& a, int nvec, int vpw, hipStream_t s)
{
    constexpr bool P = Q == 2;
    const int64_t waves = (int64_t)a.n_r * a.nseg * ((nvec + vpw - 1) / vpw);
    if (vpw == 4) {
        if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 2, P, 4, true>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, 2, P, 4, true>(a, nvec, s);
        else visit_launch<Q, 4, 1, P, 4, true>(a, nvec, s);
        return;
    }
    if (vpw == 2) {
        if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 4, P, 2, true>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, 4, P, 2, true>(a, nvec, s);
        else visit_launch<Q, 4, 2, P, 2, true>(a, nvec, s);
        return;
    }
    if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 8, P, 1, true>(a, nvec, s);
    else if (a.K <= 128) visit_launch<Q, 2, 8, P, 1, true>(a, nvec, s);
    else if (a.K <= 256) visit_launch<Q, 4, 4, P, 1, true>(a, nvec, s);
    else visit_launch<Q, 8, 2, P, 1, true>(a, nvec, s);
}

// lane-shifted taps over row pairs (visit set 2); vpw vectors per wave
template <int Q, int RR>
static void visitg_dispatch(const VisitArgs& a, int nvec, int vpw, hipStream_t s)
{
    constexpr bool P = Q == 2;
    if (vpw == 4) {
        if (a.K <= 64) visit_launch<Q, 1, 2, P, 4, true, false, RR>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, 2, P, 4, true, false, RR>(a, nvec, s);
        else visit_launch<Q, 4, 1, P, 4, true, false, RR>(a, nvec, s);
        return;
    }
    if (vpw == 2) {
        if (a.K <= 64) visit_launch<Q, 1, 4, P, 2, true, false, RR>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, 4, P, 2, true, false, RR>(a, nvec, s);
        else visit_launch<Q, 4, 2, P, 2, true, false, RR>(a, nvec, s);
        return;
    }
    if (a.K <= 64) visit_launch<Q, 1, 4, P, 1, true, false, RR>(a, nvec, s);
    else if (a.K <= 128) visit_launch<Q, 2, 4, P, 1, true, false, RR>(a, nvec, s);
    else visit_launch<Q, 4, 2, P, 1, true, false, RR>(a, nvec, s);
}

// vpw: vectors per wave (1, 2 or 4).  Loads in flight per lane stay near NB * V * T / 8.
template <int Q, bool PAIR>
static void visit_dispatch(const VisitArgs& a, int nvec, int vpw, hipStream_t s)
{
    constexpr int NB1 = Q == 1 ? 8 : 4;
    // enough waves to fill the chip with one wave per (row, segment): cover all hats per wave;
    // otherwise split the hats into 64-hat chunks, one per wave
    const int64_t waves = (int64_t)a.n_r * a.nseg * ((nvec + vpw - 1) / vpw);
    if (vpw == 4) {
        if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 2, PAIR, 4>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, Q == 1 ? 2 : 1, PAIR, 4>(a, nvec, s);
        else visit_launch<Q, 4, 1, PAIR, 4>(a, nvec, s);
        return;
    }
    if (vpw == 2) {
        if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 4, PAIR, 2>(a, nvec, s);
        else if (a.K <= 128) visit_launch<Q, 2, Q == 1 ? 4 : 2, PAIR, 2>(a, nvec, s);
        else visit_launch<Q, 4, Q == 1 ? 2 : 1, PAIR, 2>(a, nvec, s);
        return;
    }
    if (a.K <= 64 || waves < 16384) visit_launch<Q, 1, 8, PAIR, 1>(a, nvec, s);
    else if (a.K <= 128) visit_launch<Q, 2, NB1, PAIR, 1>(a, nvec, s);
    else if (a.K <= 256) visit_launch<Q, 4, Q == 1 ? 4 : 2, PAIR, 1>(a, nvec, s);
    else visit_launch<Q, 8, 2, PAIR, 1>(a, nvec, s);
}

// ------------------------------------------------------------------ one launch for many members
// Resident blocks of a persistent launch: 256 CUs x 8 (a multiple of 8, see k_apply_lean_multi).
constexpr int64_t PERSIST_BLOCKS = 2048;

static unsigned multi_grid(int64_t total, bool persist)
{
    return (unsigned)(persist ? std::min<int64_t>(total, PERSIST_BLOCKS) : total);
}

// Forward of members [b, e) in one launch; false if they do not fit the lean multi kernel.
template <int Q, int LPR, int NI>
static void reg_multi_launch(RegMulti& a, bool vec4, bool persist, hipStream_t s)
{
    const dim3 grid(multi_grid(a.total, persist)), blk(A_WAVES * WAVE);
    if (vec4) hipLaunchKernelGGL((k_apply_reg_multi<Q, LPR, NI, true>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((k_apply_reg_multi<Q, LPR, NI, false>), grid, blk, 0, s, a);
}

template <int Q, int NI>
static void reg_multi_dispatch(RegMulti& a, int lpr, bool vec4, bool persist, hipStream_t s)
{
    switch (lpr) {
    case 16: reg_multi_launch<Q, 16, NI>(a, vec4, persist, s); break;
    case 32: reg_multi_launch<Q, 32, NI>(a, vec4, persist, s); break;
    default: reg_multi_launch<Q, 64, NI>(a, vec4, persist, s); break;
    }
}

// Register forward of members [b, e) in one launch (all members on reg1 or all on reg2).
static bool apply_multi_reg(const rtt_geometry* g, int b, int e, const float* x, float* y, int nvec, uint32_t mask,
                            hipStream_t s, bool persist, bool shared, int* rc, bool probe = false)
{
    const Member& m0 = g->members[b];
    const int v0 = m0.apply_variant;
    bool vec4 = (((uintptr_t)y) & 15) == 0 && (nvec == 1 || (g->n_rows % 4) == 0);
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        if (!lean_supported(m) || m.Q != m0.Q || m.apply_variant != v0) return false;
        vec4 = vec4 && (m.grid.n_frames % 4) == 0 && (m.row_offset % 4) == 0;
    }
    const int NI = v0 == 6 ? 1 : 2;
    // one chunk length for the launch: the fewest idle lanes over all rows
    int lpr = 64;
    int64_t best = INT64_MAX;
    for (int c : {64, 32, 16}) {
        int64_t w = 0;
        for (int i = b; i < e; ++i) {
            const int64_t F = g->members[i].grid.n_frames, fc = 4 * c;
            w += g->members[i].n_rays * ((F + fc - 1) / fc * fc - F);
        }
        if (w < best) {
            best = w;
            lpr = c;
        }
    }
    RegMulti a;
    a.G = e - b;
    int64_t nb = 0;
    const int64_t rays_per_block = (int64_t)A_WAVES * (WAVE / lpr) * NI;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        RegMember& d = a.m[i - b];
        d.rec = g->d_fwd + m.ray_begin;
        d.n_rays = m.n_rays;
        d.x_off = shared ? 0 : m.col_offset;
        d.y_off = m.row_offset;
        d.K = m.grid.n_hat;
        d.F = m.grid.n_frames;
        d.nk = m.grid.n_phi * m.grid.n_hat;
        d.x_bytes = (int)(m.n_cols * 4);
        d.mask = effective_mask(m, mask);
        d.blk_begin = (uint32_t)nb;
        d.nrb = (uint32_t)((m.n_rays + rays_per_block - 1) / rays_per_block);
        const int64_t nch = (m.grid.n_frames + 4 * lpr - 1) / (4 * lpr);
        nb += m.n_rays > 0 ? (int64_t)d.nrb * nch : 0;
    }
    if (nb * nvec >= (1ll << 31)) return false;
    if (probe) return true;
    a.per_vec = (uint32_t)nb;
    a.total = (uint32_t)(nb * nvec);
    a.x = x;
    a.y = y;
    a.x_stride = shared ? m0.n_cols : g->n_cols;
    a.y_stride = g->n_rows;
    *rc = RTT_OK;
    if (a.total == 0) return true;
    if (m0.Q == 1) {
        if (NI == 1) reg_multi_dispatch<1, 1>(a, lpr, vec4, persist, s);
        else reg_multi_dispatch<1, 2>(a, lpr, vec4, persist, s);
    } else {
        if (NI == 1) reg_multi_dispatch<2, 1>(a, lpr, vec4, persist, s);
        else reg_multi_dispatch<2, 2>(a, lpr, vec4, persist, s);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) *rc = hip_fail(err, "k_apply_reg_multi");
    return true;
}

// probe: report whether the members would run in one launch, without launching
static bool apply_multi(const rtt_geometry* g, int b, int e, const float* x, float* y, int nvec, uint32_t mask,
                        hipStream_t s, bool persist, bool shared, int* rc, bool probe = false)
{
    const Member& m0 = g->members[b];
    if (m0.apply_variant == 6 || m0.apply_variant == 7)
        return apply_multi_reg(g, b, e, x, y, nvec, mask, s, persist, shared, rc, probe);
    // wide output stores (8-byte aligned rows at Q = 1, 16-byte at Q = 2), decided per member
    const int wa = m0.Q == 1 ? 2 : 4;
    const bool vec4 = (((uintptr_t)y) & (4 * wa - 1)) == 0 && (nvec == 1 || (g->n_rows % wa) == 0);
    bool all8 = true, use_abs = m0.apply_variant == 11;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        if (use_abs) {
            if (!apply_variant_ok(m, 11) || m.Q != m0.Q || m.apply_variant != 11) return false;
            continue;
        }
        if (!lean_supported(m) || m.Q != m0.Q) return false;
        if (m0.apply_variant == 13 ? m.apply_variant != 13 : (m.apply_variant != 4 && m.apply_variant != 5)) return false;
        all8 = all8 && m.apply_variant == 5;
    }
    const FwdRec* recs = m0.apply_variant == 13 ? g->d_fwd_row : g->d_fwd;
    const int NB = all8 && !use_abs ? 8 : 4;
    LeanMulti a;
    a.G = e - b;
    int64_t nb = 0;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        LeanMember& d = a.m[i - b];
        d.rec = (use_abs ? g->d_fwd : recs) + m.ray_begin;
        d.n_rays = m.n_rays;
        d.blk_begin = (uint32_t)nb;
        d.x_off = shared ? 0 : m.col_offset;
        d.y_off = m.row_offset;
        d.K = m.grid.n_hat;
        d.F = m.grid.n_frames;
        d.nk = m.grid.n_phi * m.grid.n_hat;
        d.x_bytes = (int)(m.n_cols * 4);
        d.nrb = (uint32_t)((m.n_rays + (int64_t)A_WAVES * NB - 1) / ((int64_t)A_WAVES * NB));
        d.mask = effective_mask(m, mask);
        int nch = 1;
        if (use_abs) d.fc = m.grid.n_frames;   // one task covers every frame
        else lean_chunks(m.grid.n_frames, m.Q, &nch, &d.fc);
        d.wide = (m.grid.n_frames % wa) == 0 && (m.row_offset % wa) == 0;
        nb += m.n_rays > 0 ? (int64_t)d.nrb * nch : 0;
    }
    if (nb * nvec >= (1ll << 31)) return false;
    if (probe) return true;
    a.per_vec = (uint32_t)nb;
    a.total = (uint32_t)(nb * nvec);
    a.x = x;
    a.y = y;
    a.x_stride = shared ? m0.n_cols : g->n_cols;
    a.y_stride = g->n_rows;
    *rc = RTT_OK;
    if (a.total == 0) return true;
    const dim3 grid(multi_grid(a.total, persist)), blk(A_WAVES * WAVE);
    if (use_abs) {
        if (m0.Q == 1) {
            if (vec4) hipLaunchKernelGGL((k_apply_abs_multi<1, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_abs_multi<1, false>), grid, blk, 0, s, a);
        } else {
            if (vec4) hipLaunchKernelGGL((k_apply_abs_multi<2, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_abs_multi<2, false>), grid, blk, 0, s, a);
        }
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) *rc = hip_fail(err, "k_apply_abs_multi");
        return true;
    }
    if (m0.Q == 1) {
        if (NB == 4) {
            if (vec4) hipLaunchKernelGGL((k_apply_lean_multi<1, 4, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_lean_multi<1, 4, false>), grid, blk, 0, s, a);
        } else {
            if (vec4) hipLaunchKernelGGL((k_apply_lean_multi<1, 8, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_lean_multi<1, 8, false>), grid, blk, 0, s, a);
        }
    } else {
        if (NB == 4) {
            if (vec4) hipLaunchKernelGGL((k_apply_lean_multi<2, 4, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_lean_multi<2, 4, false>), grid, blk, 0, s, a);
        } else {
            if (vec4) hipLaunchKernelGGL((k_apply_lean_multi<2, 8, true>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_apply_lean_multi<2, 8, false>), grid, blk, 0, s, a);
        }
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) *rc = hip_fail(err, "k_apply_lean_multi");
    return true;
}

template <int Q, int V, int NB, bool PAIR, bool DPP, bool HALO = false, int RR = 1, int NVW = 1>
static void visit_multi_launch(VisitMulti& a, const rtt_geometry* g, int b, int e, int set, int nvec, bool persist,
                               hipStream_t s)
{
    if constexpr (DPP && !HALO) {
        bool fits = true;
        for (int i = b; i < e; ++i) fits = fits && visit_halo_fits<Q, V>(g->members[i].grid.n_hat);
        if (fits) {
            visit_multi_launch<Q, V, NB, PAIR, true, true, RR, NVW>(a, g, b, e, set, nvec, persist, s);
            return;
        }
    }
    constexpr int C = visit_chunk<Q, V, DPP, HALO>();
    int64_t nb = 0;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        VisitMember& d = a.m[i - b];
        d.kchunks = (m.grid.n_hat + C - 1) / C;
        d.blk_begin = (uint32_t)nb;
        nb += (int64_t)(((m.grid.n_r + RR - 1) / RR + T_WAVES - 1) / T_WAVES) * d.nseg * d.kchunks;
    }
    a.per_vec = (uint32_t)nb;
    a.nvec = nvec;
    a.total = (uint32_t)(nb * ((nvec + NVW - 1) / NVW));   // below 2^31: checked by adjoint_multi
    if (a.total == 0) return;
    hipLaunchKernelGGL((k_adjoint_visit_multi<Q, V, NB, PAIR, DPP, HALO, RR, NVW>), dim3(multi_grid(a.total, persist)),
                       dim3(T_WAVES * WAVE), 0, s, a);
}

template <int Q, bool PAIR, bool DPP = false, int RR = 1>
static void visit_multi_dispatch(VisitMulti& a, const rtt_geometry* g, int b, int e, int set, int nvec,
                                 bool persist, hipStream_t s, int vpw = 1)
{
    constexpr int NB1 = Q == 1 ? 8 : 4;
    int64_t waves = 0;
    int K = 0;
    for (int i = b; i < e; ++i) {
        waves += (int64_t)g->members[i].grid.n_r * g->members[i].nseg[set] * nvec;
        K = std::max(K, g->members[i].grid.n_hat);
    }
    if (RR == 2 && vpw == 4) {
        // row pairs, four vectors per wave
        if (K <= 64) visit_multi_launch<Q, 1, 2, PAIR, DPP, false, RR, 4>(a, g, b, e, set, nvec, persist, s);
        else if (K <= 128) visit_multi_launch<Q, 2, 2, PAIR, DPP, false, RR, 4>(a, g, b, e, set, nvec, persist, s);
        else visit_multi_launch<Q, 4, 1, PAIR, DPP, false, RR, 4>(a, g, b, e, set, nvec, persist, s);
        return;
    }
    if (RR == 2 && vpw == 2) {
        // row pairs, two vectors per wave (record decode and tap weights shared)
        if (K <= 64) visit_multi_launch<Q, 1, 4, PAIR, DPP, false, RR, 2>(a, g, b, e, set, nvec, persist, s);
        else if (K <= 128) visit_multi_launch<Q, 2, 4, PAIR, DPP, false, RR, 2>(a, g, b, e, set, nvec, persist, s);
        else visit_multi_launch<Q, 4, 2, PAIR, DPP, false, RR, 2>(a, g, b, e, set, nvec, persist, s);
        return;
    }
    if (RR == 2) {
        // row pairs: half the (row, segment) tasks; batches as in the single-geometry pair form
        if (K <= 64) visit_multi_launch<Q, 1, 4, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
        else if (K <= 128) visit_multi_launch<Q, 2, 4, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
        else visit_multi_launch<Q, 4, 2, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
        return;
    }
    if (K <= 64 || waves < 16384) visit_multi_launch<Q, 1, 8, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
    else if (K <= 128) visit_multi_launch<Q, 2, NB1, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
    else if (K <= 256) visit_multi_launch<Q, 4, Q == 1 ? 4 : 2, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
    else visit_multi_launch<Q, 8, 2, PAIR, DPP, false, RR>(a, g, b, e, set, nvec, persist, s);
}

// Adjoint of members [b, e) in one launch; false if they do not fit the visit multi kernel.
static bool adjoint_multi(const rtt_geometry* g, int b, int e, const float* y, float* x, int nvec, uint32_t mask,
                          hipStream_t s, bool persist, int* rc, bool probe = false)
{
    const Member& m0 = g->members[b];
    bool pair = (((uintptr_t)y) & 7) == 0 && (nvec == 1 || (g->n_rows % 2) == 0);
    int64_t wide = 0;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        if (!visit_supported(m) || m.Q != m0.Q || m.adj_variant != m0.adj_variant ||
            (m0.adj_variant != 11 && m0.adj_variant != 16 && m0.adj_variant != 19 && m0.adj_variant != 20))
            return false;
        pair = pair && (m.grid.n_frames % 2) == 0 && (m.row_offset % 2) == 0;
        wide += (int64_t)m.grid.n_r * m.nseg[0] * nvec;
    }
    // row pairs (lane-shifted taps; frame pairs at Q = 2) read visit set 2
    const bool rp = (m0.adj_variant == 19 || m0.adj_variant == 20) && (m0.Q == 1 || pair);
    if (m0.adj_variant == 20 && !rp) return false;
    const int set = rp ? 2 : wide >= 16384 ? 0 : 1;
    // task count with the narrowest hat chunk (62 hats, the largest count any V gives); every
    // member's blocks must fit the visit kernel's 31-bit buffer ranges
    int64_t most = 0;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        if (!visit_fits(m.n_rows, m.n_cols, 0, 0, 1)) return false;
        most += (int64_t)((m.grid.n_r + T_WAVES - 1) / T_WAVES) * m.nseg[set] * ((m.grid.n_hat + WAVE - 3) / (WAVE - 2));
    }
    if (most * nvec >= (1ll << 31)) return false;
    if (probe) return true;
    VisitMulti a;
    a.G = e - b;
    for (int i = b; i < e; ++i) {
        const Member& m = g->members[i];
        VisitMember& d = a.m[i - b];
        d.visits = g->d_visits + m.visit_begin[set];
        d.vtask = g->d_vtask + m.vtask_begin[set];
        d.y_off = m.row_offset;
        d.x_off = m.col_offset;
        d.n_r = m.grid.n_r;
        d.n_phi = m.grid.n_phi;
        d.K = m.grid.n_hat;
        d.F = m.grid.n_frames;
        d.nseg = m.nseg[set];
        d.vseg = m.vseg[set];
        d.mask = effective_mask(m, mask);
        d.y_bytes = (uint32_t)(m.n_rows * 4);
        d.x_bytes = (uint32_t)(m.n_cols * 4);
    }
    a.y = y;
    a.x = x;
    a.y_stride = g->n_rows;
    a.x_stride = g->n_cols;
    // row pairs: two (visitp2v) or four (visitp4v) vectors per wave, as in the single-geometry
    // launch, when the launch has that many and every member's group of vectors fits the buffer
    // ranges
    int vpw = std::min(m0.adj_variant == 20 ? 4 : 2, nvec);
    if (vpw == 3) vpw = 2;
    for (int i = b; i < e; ++i)
        while (vpw > 1 && !visit_fits(g->members[i].n_rows, g->members[i].n_cols, g->n_rows, g->n_cols, vpw)) vpw /= 2;
    if (rp && m0.Q == 1) visit_multi_dispatch<1, false, true, 2>(a, g, b, e, set, nvec, persist, s, vpw);
    else if (rp) visit_multi_dispatch<2, true, true, 2>(a, g, b, e, set, nvec, persist, s, vpw);
    else if (m0.Q == 1 && (m0.adj_variant == 16 || m0.adj_variant == 19))
        visit_multi_dispatch<1, false, true>(a, g, b, e, set, nvec, persist, s);
    else if (m0.Q == 1) visit_multi_dispatch<1, false>(a, g, b, e, set, nvec, persist, s);
    else if (pair && (m0.adj_variant == 16 || m0.adj_variant == 19))
        visit_multi_dispatch<2, true, true>(a, g, b, e, set, nvec, persist, s);
    else if (pair) visit_multi_dispatch<2, true>(a, g, b, e, set, nvec, persist, s);
    else visit_multi_dispatch<2, false>(a, g, b, e, set, nvec, persist, s);
    hipError_t err = hipGetLastError();
    *rc = err == hipSuccess ? RTT_OK : hip_fail(err, "k_adjoint_visit_multi");
    return true;
}

template <int Q, int V, int CW, bool PAIR>
static void rows_launch(const RowsArgs& a, int nvec, hipStream_t s)
{
    constexpr int NB = Q == 1 ? (V <= 2 ? 8 : 4) : (V <= 2 ? 4 : 2);
    const int64_t waves = (int64_t)a.ngroups * a.nbands;
    const dim3 grid((unsigned)((waves + T_WAVES - 1) / T_WAVES), (unsigned)nvec);
    hipLaunchKernelGGL((k_adjoint_rows<Q, V, CW, NB, PAIR>), grid, dim3(T_WAVES * WAVE), 0, s, a);
}

template <int Q, int CW, bool PAIR>
static void rows_dispatch(const RowsArgs& a, int nvec, hipStream_t s)
{
    switch ((a.K + WAVE - 1) / WAVE) {
    case 1: rows_launch<Q, 1, CW, PAIR>(a, nvec, s); break;
    case 2: rows_launch<Q, 2, CW, PAIR>(a, nvec, s); break;
    case 3: rows_launch<Q, 3, CW, PAIR>(a, nvec, s); break;
    default: rows_launch<Q, 4, CW, PAIR>(a, nvec, s); break;
    }
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
    if (!adjoint_variant_ok(m, variant)) variant = 2;
    if (variant == 12 || variant == 13) {
        RowsArgs ra;
        ra.rec = g->d_fwd + m.ray_begin;
        ra.cstart = g->d_cell_start + m.cell_begin;
        ra.n_r = m.grid.n_r;
        ra.n_phi = m.grid.n_phi;
        ra.K = m.grid.n_hat;
        ra.F = m.grid.n_frames;
        const int CW = variant == 12 ? 4 : 8;
        ra.ngroups = (ra.n_phi + CW - 1) / CW;
        // enough waves to hide memory latency: split the rows into bands when the groups and
        // vectors alone give fewer than 65536 waves (bands of at least 4 rows)
        const int64_t base = (int64_t)ra.ngroups * nvec;
        const int64_t want = std::max<int64_t>(1, (65536 + base - 1) / base);
        const int nb = (int)std::min<int64_t>(want, (ra.n_r + 3) / 4);
        ra.rb = (ra.n_r + nb - 1) / nb;
        ra.nbands = (ra.n_r + ra.rb - 1) / ra.rb;
        ra.y = y;
        ra.x = x;
        ra.y_stride = y_stride;
        ra.x_stride = x_stride;
        ra.mask = mask;
        const bool pair = (ra.F % 2) == 0 && (((uintptr_t)y) & 7) == 0 && (nvec == 1 || (y_stride % 2) == 0);
        if (m.Q == 1) {
            if (CW == 4) rows_dispatch<1, 4, false>(ra, nvec, s);
            else rows_dispatch<1, 8, false>(ra, nvec, s);
        } else if (pair) {
            if (CW == 4) rows_dispatch<2, 4, true>(ra, nvec, s);
            else rows_dispatch<2, 8, true>(ra, nvec, s);
        } else {
            if (CW == 4) rows_dispatch<2, 4, false>(ra, nvec, s);
            else rows_dispatch<2, 8, false>(ra, nvec, s);
        }
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    if ((variant == 11 || variant >= 14) && !visit_fits(m.n_rows, m.n_cols, y_stride, x_stride, 1)) variant = 2;
    // base rows (visit set 3): frame pairs at Q = 2; else the single-row lane-shifted form
    if (variant == 21 || variant == 22) {
        const bool fpair = m.Q == 1 || ((m.grid.n_frames % 2) == 0 && (((uintptr_t)y) & 7) == 0 && (nvec == 1 || (y_stride % 2) == 0));
        int vpw = std::min(variant == 22 ? 2 : 1, nvec);
        if (!visit_fits(m.n_rows, m.n_cols, y_stride, x_stride, vpw)) vpw = 1;
        if (fpair) {
            VisitArgs va;
            va.visits = g->d_visits + m.visit_begin[3];
            va.n_r = m.grid.n_r;
            va.n_phi = m.grid.n_phi;
            va.K = m.grid.n_hat;
            va.F = m.grid.n_frames;
            va.vseg = VISIT_SEG_MAX;
            va.y = y;
            va.x = x;
            va.y_stride = y_stride;
            va.x_stride = x_stride;
            va.mask = mask;
            va.y_bytes = (uint32_t)(m.n_rows * 4);
            va.x_bytes = (uint32_t)(m.n_cols * 4);
            const int64_t* t0 = g->d_vtask + m.br_task_begin[0];
            const int64_t* t1 = g->d_vtask + m.br_task_begin[1];
            if (m.Q == 1) visitb_dispatch<1>(va, t0, m.br_ntask[0], t1, m.br_ntask[1], nvec, vpw, s);
            else visitb_dispatch<2>(va, t0, m.br_ntask[0], t1, m.br_ntask[1], nvec, vpw, s);
            RTT_HIP(hipGetLastError());
            return RTT_OK;
        }
        variant = nvec >= 2 ? 17 : 16;
    }
    // row pairs: frame pairs at Q = 2, and enough (pair, segment, vector group) tasks to fill the
    // chip once; else the single-row form, which narrows its segments for small launches
    if (variant == 19 || variant == 20) {
        const bool fpair = m.Q == 1 || ((m.grid.n_frames % 2) == 0 && (((uintptr_t)y) & 7) == 0 && (nvec == 1 || (y_stride % 2) == 0));
        const int pvw = std::min(variant == 19 ? 2 : 4, nvec);
        const int64_t waves = (int64_t)((m.grid.n_r + 1) / 2) * m.nseg[2] * ((nvec + pvw - 1) / pvw);
        if (!fpair || waves < 8192) variant = nvec >= 2 ? 17 : 16;
    }
    if (variant == 11 || variant >= 14) {
        // the wide segment set when the vectors alone give enough waves, else the narrow one
        // rows per wave: 2 for the row-pair forms (visit set 2)
        const int rr = (variant == 19 || variant == 20) ? 2 : 1;
        int vpw = (variant == 14 || variant == 17 || variant == 19) ? 2 : (variant == 15 || variant == 18 || variant == 20) ? 4 : 1;
        // no more vectors per wave than the launch has (a missing vector costs a full one)
        while (vpw > 1 && vpw > nvec) vpw /= 2;
        if (!visit_fits(m.n_rows, m.n_cols, y_stride, x_stride, vpw)) vpw = 1;
        const int set = rr == 2 ? 2 : ((int64_t)m.grid.n_r * m.nseg[0] * ((nvec + vpw - 1) / vpw) >= 16384) ? 0 : 1;
        VisitArgs va;
        va.visits = g->d_visits + m.visit_begin[set];
        va.vtask = g->d_vtask + m.vtask_begin[set];
        va.n_r = m.grid.n_r;
        va.n_phi = m.grid.n_phi;
        va.K = m.grid.n_hat;
        va.F = m.grid.n_frames;
        va.nseg = m.nseg[set];
        va.vseg = m.vseg[set];
        va.y = y;
        va.x = x;
        va.y_stride = y_stride;
        va.x_stride = x_stride;
        va.mask = mask;
        va.y_bytes = (uint32_t)(m.n_rows * 4);
        va.x_bytes = (uint32_t)(m.n_cols * 4);
        // frame pairs need 8-byte aligned rows: even n_frames and aligned data vectors
        const bool pair = (va.F % 2) == 0 && (((uintptr_t)y) & 7) == 0 && (nvec == 1 || (y_stride % 2) == 0);
        if (rr == 2 && m.Q == 1) visitg_dispatch<1, 2>(va, nvec, vpw, s);
        else if (rr == 2) visitg_dispatch<2, 2>(va, nvec, vpw, s);
        else if (variant >= 16 && m.Q == 1) visitd_dispatch<1>(va, nvec, vpw, s);
        else if (variant >= 16 && pair) visitd_dispatch<2>(va, nvec, vpw, s);
        else if (m.Q == 1) visit_dispatch<1, false>(va, nvec, vpw, s);
        else if (pair) visit_dispatch<2, true>(va, nvec, vpw, s);
        else visit_dispatch<2, false>(va, nvec, vpw, s);
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    switch (variant) {
    case 0: adjoint_dispatch_tile<8, 8>(a, m.P, m.Q, nvec, s); break;
    case 1: adjoint_dispatch_tile<4, 8>(a, m.P, m.Q, nvec, s); break;
    case 2: adjoint_dispatch_tile<4, 4>(a, m.P, m.Q, nvec, s); break;
    case 3: adjoint_dispatch_sweep<32, 1>(a, m.P, m.Q, nvec, s); break;
    case 4: adjoint_dispatch_sweep<32, 2>(a, m.P, m.Q, nvec, s); break;
    case 5: adjoint_dispatch_sweep<16, 1>(a, m.P, m.Q, nvec, s); break;
    case 6: adjoint_dispatch_sweep<16, 2>(a, m.P, m.Q, nvec, s); break;
    case 7: adjoint_dispatch_tb<8, 8>(a, m.P, m.Q, nvec, s); break;
    case 8: adjoint_dispatch_tb<4, 8>(a, m.P, m.Q, nvec, s); break;
    case 9: adjoint_dispatch_tb<4, 4>(a, m.P, m.Q, nvec, s); break;
    default: adjoint_dispatch_tb<2, 4>(a, m.P, m.Q, nvec, s); break;
    }
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

}  // namespace rtt

namespace rtt {

int apply_op(const rtt_geometry* g, int member, bool adjoint, const float* in, float* out, int nvec,
             uint32_t mask, hipStream_t s, bool shared_x)
{
    // shared_x (forward only): every member reads its columns from the one block `in`
    // ([nvec][member columns]) instead of its own block of a [nvec][n_cols] vector
    if (member >= 0) {
        const Member& m = g->members[member];
        const uint32_t em = effective_mask(m, mask);
        return adjoint ? launch_adjoint(g, m, in, out, nvec, m.n_rows, m.n_cols, em, s, -1)
                       : launch_apply(g, m, in, out, nvec, m.n_cols, m.n_rows, em, s, -1);
    }
    if (nvec == 0) return RTT_OK;
    const int G = (int)g->members.size();
    const int mode = adjoint ? g->batch_adjoint_mode : g->batch_apply_mode;
    for (int b = 0; b < G; b += MULTI_MAX) {
        const int e = std::min(G, b + MULTI_MAX);
        if (G > 1 && mode != 0) {
            int rc = RTT_OK;
            const bool done = adjoint ? adjoint_multi(g, b, e, in, out, nvec, mask, s, mode == 2, &rc)
                                      : apply_multi(g, b, e, in, out, nvec, mask, s, mode == 2, shared_x, &rc);
            if (rc) return rc;
            if (done) continue;
        }
        for (int i = b; i < e; ++i) {
            const Member& m = g->members[i];
            const uint32_t em = effective_mask(m, mask);
            int rc = adjoint ? launch_adjoint(g, m, in + m.row_offset, out + m.col_offset, nvec, g->n_rows,
                                              g->n_cols, em, s, -1)
                             : launch_apply(g, m, in + (shared_x ? 0 : m.col_offset), out + m.row_offset, nvec,
                                            shared_x ? m.n_cols : g->n_cols, g->n_rows, em, s, -1);
            if (rc) return rc;
        }
    }
    return RTT_OK;
}

int whole_operator_launches(const rtt_geometry* g, bool adjoint)
{
    const int G = (int)g->members.size();
    const int mode = adjoint ? g->batch_adjoint_mode : g->batch_apply_mode;
    int n = 0;
    for (int b = 0; b < G; b += MULTI_MAX) {
        const int e = std::min(G, b + MULTI_MAX);
        if (G > 1 && mode != 0) {
            int rc = RTT_OK;
            const bool one = adjoint ? adjoint_multi(g, b, e, nullptr, nullptr, 1, 0u, nullptr, mode == 2, &rc, true)
                                     : apply_multi(g, b, e, nullptr, nullptr, 1, 0u, nullptr, mode == 2, false, &rc, true);
            if (one) {
                ++n;
                continue;
            }
        }
        for (int i = b; i < e; ++i) {
            const Member& m = g->members[i];
            if (m.n_rays == 0) continue;
            // the base-row adjoint makes two passes (frame pairs at Q = 2; else the single-row form)
            const bool br = adjoint && (m.adj_variant == 21 || m.adj_variant == 22) &&
                            (m.Q == 1 || (m.grid.n_frames % 2) == 0);
            n += br ? 2 : 1;
        }
    }
    return n;
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

extern "C" int op_apply_shared(const rtt_geometry* g, const float* x, float* y, int32_t nvec, uint32_t order_mask,
                               void* stream)
{
    int rc = check_call(g, x, y, nvec);
    if (rc) return rc;
    const rtt_grid& g0 = g->members[0].grid;
    for (const Member& m : g->members) {
        const rtt_grid& q = m.grid;
        if (q.n_r != g0.n_r || q.n_phi != g0.n_phi || q.n_hat != g0.n_hat || q.r_in != g0.r_in ||
            q.r_out != g0.r_out || q.s0 != g0.s0 || q.dt_src != g0.dt_src)
            return fail(RTT_EINVAL, "op_apply_shared: the geometries do not share one source grid");
    }
    return apply_op(g, -1, false, x, y, nvec, order_mask, (hipStream_t)stream, true);
}

extern "C" int op_apply_adjoint(const rtt_geometry* g, const float* y, float* x, int32_t nvec,
                                uint32_t order_mask, void* stream)
{
    int rc = check_call(g, y, x, nvec);
    if (rc) return rc;
    return apply_op(g, -1, true, y, x, nvec, order_mask, (hipStream_t)stream);
}
