// Dense kernels of the spectral drivers on gfx950: FP32 MFMA Gram and block
// combination, deterministic FP64 reductions, and normal draws.
//
// Blocks of vectors are stored vector-major: V[i][0..L) with row stride ld.
//
//  gram:    G[i][j] = sum_l A[i][l] B[j][l]        (M x N, L long; e.g. Y^T Y)
//           split over L into independent slices; each workgroup computes a
//           64x64 output block of one slice with v_mfma_f32_32x32x2f32 (one
//           32x32 tile per wave) and writes an FP32 partial; a second kernel
//           sums the partials of every entry in FP64 in slice order, so the
//           result does not depend on scheduling.  The output blocks of one
//           slice run on one XCD; for G = A A^T only the 32x32 tiles on and
//           above the diagonal are computed and the rest is mirrored.
//  combine: Out[m][l] = sum_k C[k][m] Y[k][l]      (Out = C^T Y; e.g. Q = Y R^-1)
//           C (K x M, small) and the matching rows of Y are staged in LDS 16
//           rows at a time, double buffered with the next chunk's loads in
//           flight; each wave owns 32 columns l and up to MG 32-row blocks of
//           Out, so every element of Y is read once per pass.
//
//  skinny forms (N <= 32 for gram, M <= 32 for combine; 16-byte aligned rows):
//           no LDS staging.  gram: a wave owns a 32-row tile of A against all
//           of B over part of an L slice; each lane feeds 16 consecutive l of
//           its row per chunk (the contraction order is free, so lane (r, h)
//           gives the MFMA k-pair member h the l values 16h .. 16h+15 of the
//           chunk, one per step).  combine: a wave owns 128 columns l as four
//           32-column tiles interleaved by 4, so every lane reads 4 adjacent
//           columns of a row of Y with one 16-byte load and writes 4 adjacent
//           outputs with one 16-byte store.
//
// MFMA operand layout used (32x32x2 f32): lane t supplies A[t%32][t/32] and
// B[t/32][t%32]; accumulator register r of lane t holds
// C[8(r/4) + 4(t/32) + r%4][t%32].
#include "rtt_internal.h"
#include "dense.h"

namespace rtt {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int GB = 64;   // gram output block
constexpr int GK = 32;   // k-chunk staged in LDS

template <bool VL, int PF = 4>
__global__ __launch_bounds__(256) void k_gram_partial(const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ B, int64_t ldb, int M, int N,
                                                      int64_t L, int64_t slice, int nsplit, int nbn, int sym,
                                                      float* __restrict__ part, const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    // 64 x 64 output block of one L slice; the slice runs in chunks of GK columns staged in LDS
    // (double buffered), and the global loads (16-byte when VL) of the chunk PF ahead are issued
    // into registers before the current chunk's MFMAs, so PF chunks are in flight per workgroup
    // (PF = 4: 0.77 -> 0.62 ms for the 288 x 288 Gram of 1.55M-long rows against one ahead, still
    // four waves per SIMD; the products and their order do not depend on PF).
    __shared__ float As[2][GB][GK + 1];
    __shared__ float Bs[2][GB][GK + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // One workgroup per (slice, output block), output blocks on and above the diagonal only when
    // sym.  The hardware deals workgroups round robin over the 8 XCDs; workgroup b takes output
    // block (b / 8) % nact of slice 8 ((b / 8) / nact) + b % 8, so all blocks of a slice run one
    // after another on one XCD and the slice's rows come into that XCD's L2 once.
    const int nact = sym ? nbn * (nbn + 1) / 2 : (((M + GB - 1) / GB) * nbn);
    const int kx = (int)(blockIdx.x >> 3);
    const int s = (kx / nact) * 8 + (int)(blockIdx.x & 7);
    if (s >= nsplit) return;
    int bm, bn;
    {
        int t = kx % nact;
        if (sym) {
            bm = 0;
            while (t >= nbn - bm) {
                t -= nbn - bm;
                ++bm;
            }
            bn = bm + t;
        } else {
            bm = t / nbn;
            bn = t % nbn;
        }
    }
    float* __restrict__ out = part + (int64_t)s * M * N;
    const int64_t l0 = (int64_t)s * slice;
    const int64_t l1 = min(L, l0 + slice);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    // a wave whose 32 x 32 tile lies past the last row or column, or below the diagonal of a
    // diagonal block (mirrored when the partials are summed), only helps stage the chunks
    const bool live = bm * GB + wm < M && bn * GB + wn < N && !(sym && bm == bn && wm > wn);
    // element group e: row e / CPR, columns 4 (e % CPR) .. +3 of the chunk
    constexpr int NQ = GB * GK / 4 / 256;   // 16-byte groups per thread per operand
    constexpr int CPR = GK / 4;             // groups per row
    f4v ra[PF][NQ], rb[PF][NQ];
    auto load = [&](int64_t lc, f4v* xa, f4v* xb) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256;
            const int r = e / CPR, c = (e % CPR) * 4;
            const int64_t l = lc + c;
            const int ia = bm * GB + r, ib = bn * GB + r;
            if (VL && ia < M && l + 3 < l1) {
                xa[q] = *(const f4v*)(A + (int64_t)ia * lda + l);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) xa[q][t] = (ia < M && l + t < l1) ? A[(int64_t)ia * lda + l + t] : 0.f;
            }
            if (VL && ib < N && l + 3 < l1) {
                xb[q] = *(const f4v*)(B + (int64_t)ib * ldb + l);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) xb[q][t] = (ib < N && l + t < l1) ? B[(int64_t)ib * ldb + l + t] : 0.f;
            }
        }
    };
    auto store = [&](int buf, const f4v* xa, const f4v* xb) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256;
            const int r = e / CPR, c = (e % CPR) * 4;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                As[buf][r][c + t] = xa[q][t];
                Bs[buf][r][c + t] = xb[q][t];
            }
        }
    };
    f16v acc = {};
    const int half = lane >> 5, row = lane & 31;
    auto mfma = [&](int buf) {
        if (live) {
#pragma unroll
            for (int j = 0; j < GK / 2; ++j) {
                // step j covers k = j and k = j + GK / 2 (half selects which)
                const float a = As[buf][wm + row][(GK / 2) * half + j];
                const float b = Bs[buf][wn + row][(GK / 2) * half + j];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
            }
        }
    };
    // chunk c sits in LDS buffer c % 2; register set c % PF receives chunk c + PF while chunk c is
    // multiplied (sets hold the PF - 1 chunks after c, issued earlier)
    constexpr int NS = PF % 2 == 0 ? PF : 2 * PF;   // steps per unrolled round: lcm(2, PF)
#pragma unroll
    for (int j = 0; j < PF; ++j)
        if (l0 + (int64_t)j * GK < l1) load(l0 + (int64_t)j * GK, ra[j], rb[j]);
    if (l0 < l1) store(0, ra[0], rb[0]);
    __syncthreads();
    for (int64_t base = l0; base < l1; base += (int64_t)NS * GK) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int64_t lc = base + (int64_t)i * GK;
            if (lc < l1) {
                if (lc + (int64_t)PF * GK < l1) load(lc + (int64_t)PF * GK, ra[i % PF], rb[i % PF]);
                mfma(i % 2);
                if (lc + GK < l1) store((i + 1) % 2, ra[(i + 1) % PF], rb[(i + 1) % PF]);
                __syncthreads();
            }
        }
    }
    if (!live) return;
    const int col = lane & 31, hi = lane >> 5;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = bm * GB + wm + 8 * (r >> 2) + 4 * hi + (r & 3);
        const int j = bn * GB + wn + col;
        if (i < M && j < N) out[(int64_t)i * N + j] = acc[r];
    }
}

__global__ void k_gram_reduce(const float* __restrict__ part, int nsplit, int M, int N, int sym,
                              double* __restrict__ G, const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    int i = (int)(e / N), j = (int)(e % N);
    int si = i, sj = j;
    if (sym && (j >> 5) < (i >> 5)) { si = j; sj = i; }   // below the diagonal 32 x 32 tiles: mirror
    double s = 0.0;
#pragma unroll 8
    for (int t = 0; t < nsplit; ++t) s += (double)part[(int64_t)t * M * N + (int64_t)si * N + sj];
    G[e] = s;
}

template <int MG, bool VY>
__global__ __launch_bounds__(256, 2) void k_combine(const float* __restrict__ C, int K, int M, int m0,
                                                 const float* __restrict__ Y, int64_t ldy,
                                                 float* __restrict__ Out, int64_t ldo, int64_t L, float beta,
                                                 int upper, const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    // The block owns 128 columns l (32 per wave) and MG 32-row blocks of Out.  k runs in chunks of
    // CK: the chunk's rows of C and Y are staged in LDS (double buffered), and the next chunk's global
    // loads are issued into registers before the current chunk's MFMAs, so they overlap.  upper:
    // C[k][m] = 0 for k > m, so the row blocks that end at or before a chunk's first k are skipped
    // (their products are exact zeros).
    constexpr int CK = 16;
    constexpr int MW = MG * 32;
    constexpr int NC = (CK * MW + 255) / 256;     // C elements per thread per chunk
    __shared__ float Cs[2][CK][MW + 1];
    __shared__ __attribute__((aligned(16))) float Ys[2][CK][128 + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t lb = (int64_t)blockIdx.x * 128;
    const int col = lane & 31, half = lane >> 5;
    float cr[NC];
    f4v yr[2];
    auto load = [&](int kc) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int e = tid + q * 256;
            const int kr = e / MW, mc = e % MW;
            const int k = kc + kr, m = m0 + mc;
            cr[q] = (e < CK * MW && k < K && m < M) ? C[(int64_t)k * M + m] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * 256;          // 512 four-column groups: 16 rows x 32 groups
            const int kr = e >> 5, c4 = (e & 31) * 4;
            const int k = kc + kr;
            const int64_t l = lb + c4;
            if (VY && k < K && l + 3 < L) {
                yr[q] = *(const f4v*)(Y + (int64_t)k * ldy + l);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) yr[q][t] = (k < K && l + t < L) ? Y[(int64_t)k * ldy + l + t] : 0.f;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int e = tid + q * 256;
            if (e < CK * MW) Cs[buf][e / MW][e % MW] = cr[q];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * 256;
            *(f4v*)&Ys[buf][e >> 5][(e & 31) * 4] = yr[q];
        }
    };
    f16v acc[MG];
#pragma unroll
    for (int g = 0; g < MG; ++g) acc[g] = (f16v){};
    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    const int kend = upper ? min(K, m0 + MW) : K;
    for (int kc = 0; kc < kend; kc += CK) {
        const bool more = kc + CK < kend;
        if (more) load(kc + CK);
        const int gmin = (upper && kc > m0) ? (kc - m0) >> 5 : 0;   // first row block reached
#pragma unroll
        for (int j = 0; j < CK / 2; ++j) {
            const int kr = 2 * j + half;
            const float bv = Ys[buf][kr][wave * 32 + col];
#pragma unroll
            for (int g = 0; g < MG; ++g)
                if (g >= gmin)
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(Cs[buf][kr][g * 32 + col], bv, acc[g], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    const int64_t l = lb + wave * 32 + col;
    if (l >= L) return;
#pragma unroll
    for (int g = 0; g < MG; ++g) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = m0 + g * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (m < M) {
                float* o = Out + (int64_t)m * ldo + l;
                *o = (beta == 0.f) ? acc[g][r] : beta * (*o) + acc[g][r];
            }
        }
    }
}

// G partials for N <= 32: block (tile group, slice) with four waves taking every fourth 32-column
// chunk of the slice; a wave owns TM consecutive 32-row tiles of A, so each chunk of B is read once
// for all of them.  The waves' sums are added in wave order and written as the block's partial.
template <int TM>
__global__ __launch_bounds__(256) void k_gram_skinny(const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ B, int64_t ldb, int M, int N,
                                                     int64_t L, int64_t slice, float* __restrict__ part,
                                                     const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    __shared__ float red[3][64][17];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = blockIdx.y;
    const int64_t l0 = (int64_t)s * slice, l1 = min(L, l0 + slice);
    const int r = lane & 31, h = lane >> 5;
    const bool vb = r < N;
    const float* __restrict__ pb = B + (int64_t)(vb ? r : 0) * ldb;    // rows past the end read row 0,
    bool va[TM];                                                       // and their values are zeroed
    const float* __restrict__ pa[TM];
#pragma unroll
    for (int u = 0; u < TM; ++u) {
        const int ia = (blockIdx.x * TM + u) * 32 + r;
        va[u] = ia < M;
        pa[u] = A + (int64_t)(va[u] ? ia : 0) * lda;
    }
    f16v acc[TM];
#pragma unroll
    for (int u = 0; u < TM; ++u) acc[u] = (f16v){};
    for (int64_t lc = l0 + (int64_t)wave * 32; lc < l1; lc += 128) {
        const int64_t l = lc + 16 * h;
        float av[TM][16], bv[16];
        if (l + 16 <= l1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f4v xb = *(const f4v*)(pb + l + 4 * q);
#pragma unroll
                for (int t = 0; t < 4; ++t) bv[4 * q + t] = vb ? xb[t] : 0.f;
#pragma unroll
                for (int u = 0; u < TM; ++u) {
                    const f4v xa = *(const f4v*)(pa[u] + l + 4 * q);
#pragma unroll
                    for (int t = 0; t < 4; ++t) av[u][4 * q + t] = va[u] ? xa[t] : 0.f;
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const bool in = l + t < l1;
                bv[t] = (vb && in) ? pb[l + t] : 0.f;
#pragma unroll
                for (int u = 0; u < TM; ++u) av[u][t] = (va[u] && in) ? pa[u][l + t] : 0.f;
            }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t)
#pragma unroll
            for (int u = 0; u < TM; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u][t], bv[t], acc[u], 0, 0, 0);
    }
    float* __restrict__ out = part + (int64_t)s * M * N;
#pragma unroll
    for (int u = 0; u < TM; ++u) {
        if (wave > 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) red[wave - 1][lane][q] = acc[u][q];
        __syncthreads();
        if (wave == 0) {
            f16v sum = acc[u];
#pragma unroll
            for (int w = 0; w < 3; ++w)
#pragma unroll
                for (int q = 0; q < 16; ++q) sum[q] += red[w][lane][q];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = (blockIdx.x * TM + u) * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
                if (i < M && r < N) out[(int64_t)i * N + r] = sum[q];
            }
        }
        __syncthreads();
    }
}

// Sum of the slice partials of the skinny Gram in FP64: a block takes 64 entries; thread group g
// (of 16) sums, in slice order, the g-th of 16 contiguous ranges of slices; the 16 group sums are
// added in group order.  Deterministic; many slices are summed in parallel.
__global__ __launch_bounds__(1024) void k_gram_reduce_wide(const float* __restrict__ part, int nsplit, int64_t MN,
                                                           double* __restrict__ G, const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    __shared__ double sum[16][64];
    const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + e;
    const int t0 = (int)((int64_t)nsplit * g / 16), t1 = (int)((int64_t)nsplit * (g + 1) / 16);
    double acc = 0.0;
    if (i < MN) {
#pragma unroll 8
        for (int t = t0; t < t1; ++t) acc += (double)part[(int64_t)t * MN + i];
    }
    sum[g][e] = acc;
    __syncthreads();
    if (g != 0 || i >= MN) return;
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) tot += sum[q][e];
    G[i] = tot;
}

// Out = beta Out + C^T Y for M <= 32: a wave owns columns l0 .. l0 + 127; lane (j, h) reads
// Y[k][l0 + 4j .. 4j + 3] for k = 2 s + h and feeds tile q (columns l0 + 4j + q) with element q.
__global__ __launch_bounds__(256) void k_combine_skinny(const float* __restrict__ C, int K, int M,
                                                        const float* __restrict__ Y, int64_t ldy,
                                                        float* __restrict__ Out, int64_t ldo, int64_t L, float beta,
                                                        const int* __restrict__ run_if)
{
    if (run_if && !*run_if) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 31, h = lane >> 5;
    const int64_t l0 = ((int64_t)blockIdx.x * 4 + wave) * 128;
    if (l0 >= L) return;
    const int64_t lj = l0 + 4 * j;
    const bool full = lj + 3 < L;
    const bool vm = j < M;
    f16v acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (f16v){};
#pragma unroll 8
    for (int kc = 0; kc < K; kc += 2) {
        const int k = kc + h;
        float a = 0.f;
        f4v y = {0.f, 0.f, 0.f, 0.f};
        if (k < K) {
            a = vm ? C[(int64_t)k * M + j] : 0.f;
            const float* __restrict__ py = Y + (int64_t)k * ldy + lj;
            if (full) {
                y = *(const f4v*)py;
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) y[t] = lj + t < L ? py[t] : 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, y[q], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int m = 8 * (q >> 2) + 4 * h + (q & 3);
        if (m >= M) continue;
        float* __restrict__ o = Out + (int64_t)m * ldo + lj;
        f4v v = {acc[0][q], acc[1][q], acc[2][q], acc[3][q]};
        if (full) {
            if (beta != 0.f) v += beta * *(const f4v*)o;
            *(f4v*)o = v;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (lj + t < L) o[t] = (beta == 0.f) ? v[t] : beta * o[t] + v[t];
        }
    }
}

// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) and Box-Muller normals.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0; c[1] = (uint32_t)p1; c[2] = n2; c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
}

__global__ void k_normal(float* __restrict__ out, int64_t n, uint64_t seed, uint64_t offset)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t base = 4 * i;
    if (base >= n) return;
    uint32_t c[4] = {(uint32_t)(i + offset), (uint32_t)((i + offset) >> 32), 0u, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float two_pi = 6.2831853071795864769f;
    const float inv = 2.3283064365386963e-10f;   // 2^-32
    float u0 = ((float)c[0] + 0.5f) * inv, u1 = ((float)c[1] + 0.5f) * inv;
    float u2 = ((float)c[2] + 0.5f) * inv, u3 = ((float)c[3] + 0.5f) * inv;
    float r0 = sqrtf(-2.0f * logf(u0)), r1 = sqrtf(-2.0f * logf(u2));
    float v[4] = {r0 * cosf(two_pi * u1), r0 * sinf(two_pi * u1), r1 * cosf(two_pi * u3), r1 * sinf(two_pi * u3)};
    for (int t = 0; t < 4 && base + t < n; ++t) out[base + t] = v[t];
}

// y[i] += sigma * z_i with z the draws of k_normal (same counters, same mapping)
__global__ void k_normal_add(float* __restrict__ y, int64_t n, uint64_t seed, float sigma)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t base = 4 * i;
    if (base >= n) return;
    uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float two_pi = 6.2831853071795864769f;
    const float inv = 2.3283064365386963e-10f;   // 2^-32
    float u0 = ((float)c[0] + 0.5f) * inv, u1 = ((float)c[1] + 0.5f) * inv;
    float u2 = ((float)c[2] + 0.5f) * inv, u3 = ((float)c[3] + 0.5f) * inv;
    float r0 = sqrtf(-2.0f * logf(u0)), r1 = sqrtf(-2.0f * logf(u2));
    float v[4] = {r0 * cosf(two_pi * u1), r0 * sinf(two_pi * u1), r1 * cosf(two_pi * u3), r1 * sinf(two_pi * u3)};
    for (int t = 0; t < 4 && base + t < n; ++t) y[base + t] += sigma * v[t];
}

// per-vector dot products in FP64, deterministic: partials of fixed slices, then a fixed-order sum
__global__ void k_dot_partial(const float* __restrict__ a, int64_t lda, const float* __restrict__ b,
                              int64_t ldb, int64_t n, int64_t slice, double* __restrict__ part)
{
    __shared__ double red[256];
    const int v = blockIdx.y, s = blockIdx.x;
    const float* av = a + (int64_t)v * lda;
    const float* bv = b + (int64_t)v * ldb;
    const int64_t l0 = (int64_t)s * slice, l1 = min(n, l0 + slice);
    double acc = 0.0;
    for (int64_t l = l0 + threadIdx.x; l < l1; l += blockDim.x) acc += (double)av[l] * (double)bv[l];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + s] = red[0];
}

__global__ void k_dot_final(const double* __restrict__ part, int nsplit, int nvec, double* __restrict__ out)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvec) return;
    double s = 0.0;
    for (int t = 0; t < nsplit; ++t) s += part[(int64_t)v * nsplit + t];
    out[v] = s;
}

// Segmented variant: segment g of vector v is [seg[2g], seg[2g] + seg[2g+1]) and its dot product
// goes to out[v * G + g]; slices of one segment are summed in a fixed order as above.
__global__ void k_dot_partial_seg(const float* __restrict__ a, int64_t lda, const float* __restrict__ b,
                                  int64_t ldb, const int64_t* __restrict__ seg, int G, double* __restrict__ part)
{
    __shared__ double red[256];
    const int s = blockIdx.x, v = blockIdx.y, g = blockIdx.z;
    const int nsplit = gridDim.x;
    const int64_t off = seg[2 * g], len = seg[2 * g + 1];
    const int64_t slice = (len + nsplit - 1) / nsplit;
    const float* av = a + (int64_t)v * lda + off;
    const float* bv = b + (int64_t)v * ldb + off;
    const int64_t l0 = (int64_t)s * slice, l1 = min(len, l0 + slice);
    double acc = 0.0;
    for (int64_t l = l0 + threadIdx.x; l < l1; l += blockDim.x) acc += (double)av[l] * (double)bv[l];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)v * G + g) * nsplit + s] = red[0];
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// C[set][i][r] = Cd[set][i][r] / sigma[set][i]^2 when sigma[set][i] >= sigma_min and > 0, else 0
__global__ void k_scale_inv_sq(const double* __restrict__ Cd, const double* __restrict__ sigma, int sets, int t,
                               int k, int nrhs, double sigma_min, float* __restrict__ C)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)sets * t * nrhs) return;
    const int set = (int)(e / ((int64_t)t * nrhs));
    const int i = (int)((e / nrhs) % t);
    const double sg = sigma[(int64_t)set * k + i];
    C[e] = (sg >= sigma_min && sg > 0.0) ? (float)(Cd[e] / (sg * sg)) : 0.f;
}

// --------------------------------------------------------------------------------- host side
Workspace::~Workspace() { release(); }
void Workspace::release()
{
    for (auto& kv : bufs) hipFree(kv.second.first);
    bufs.clear();
}
void* Workspace::get(const char* name, size_t bytes)
{
    auto it = bufs.find(name);
    if (it != bufs.end() && it->second.second >= bytes) return it->second.first;
    if (it != bufs.end()) {
        hipFree(it->second.first);
        bufs.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
    bufs[name] = {p, bytes};
    return p;
}

int gram(Workspace& ws, const float* A, int64_t lda, const float* B, int64_t ldb, int M, int N, int64_t L,
         double* G_dev, hipStream_t s, const int* run_if)
{
    if (M <= 0 || N <= 0) return RTT_OK;
    const bool aligned = (((uintptr_t)A) & 15) == 0 && (((uintptr_t)B) & 15) == 0 && (lda % 4) == 0 && (ldb % 4) == 0;
    if (N <= 32 && aligned) {
        // skinny form: slices of whole 128-column steps, about 4096 blocks in all
        const int tm = M > 96 ? 4 : 1;                       // 32-row tiles per wave
        const int tiles = (M + 32 * tm - 1) / (32 * tm);      // tile groups
        int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(1, 4096 / tiles), L / 1024));
        int64_t slice = (L + nsplit - 1) / nsplit;
        slice = std::max<int64_t>(128, ((slice + 127) / 128) * 128);
        nsplit = (int)std::max<int64_t>(1, (L + slice - 1) / slice);   // L = 0: one empty slice
        float* part = (float*)ws.get("gram_part", sizeof(float) * (size_t)nsplit * M * N);
        if (!part) return fail(RTT_ENOMEM, "gram workspace");
        if (tm == 4)
            hipLaunchKernelGGL(k_gram_skinny<4>, dim3((unsigned)tiles, (unsigned)nsplit), dim3(256), 0, s, A, lda, B, ldb,
                               M, N, L, slice, part, run_if);
        else
            hipLaunchKernelGGL(k_gram_skinny<1>, dim3((unsigned)tiles, (unsigned)nsplit), dim3(256), 0, s, A, lda, B, ldb,
                               M, N, L, slice, part, run_if);
        const int64_t tot = (int64_t)M * N;
        hipLaunchKernelGGL(k_gram_reduce_wide, dim3((unsigned)((tot + 63) / 64)), dim3(1024), 0, s, part, nsplit, tot,
                           G_dev, run_if);
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    const int nbm = (M + GB - 1) / GB, nbn = (N + GB - 1) / GB;
    const int sym = (A == B && lda == ldb && M == N) ? 1 : 0;
    int nsplit = (int)std::min<int64_t>(std::max<int64_t>(1, L / 2048), 512);
    const int64_t blocks_per_split = (int64_t)nbm * nbn;
    if (blocks_per_split * nsplit > 8192) nsplit = (int)std::max<int64_t>(1, 8192 / blocks_per_split);
    int64_t slice = (L + nsplit - 1) / nsplit;
    slice = ((slice + GK - 1) / GK) * GK;
    nsplit = (int)((L + slice - 1) / slice);
    if (nsplit < 1) nsplit = 1;
    float* part = (float*)ws.get("gram_part", sizeof(float) * (size_t)nsplit * M * N);
    if (!part) return fail(RTT_ENOMEM, "gram workspace");
    // output blocks per slice (upper ones only when sym), slices rounded up to whole groups of 8
    const int64_t nact = sym ? (int64_t)nbn * (nbn + 1) / 2 : (int64_t)nbm * nbn;
    dim3 grid((unsigned)(nact * (((int64_t)nsplit + 7) / 8) * 8));
    // 16-byte loads need 16-byte aligned rows (slice starts are multiples of GK)
    const bool vl = (((uintptr_t)A) & 15) == 0 && (((uintptr_t)B) & 15) == 0 && (lda % 4) == 0 && (ldb % 4) == 0;
    if (vl)
        hipLaunchKernelGGL(k_gram_partial<true>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, L, slice, nsplit, nbn,
                           sym, part, run_if);
    else
        hipLaunchKernelGGL(k_gram_partial<false>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, L, slice, nsplit, nbn,
                           sym, part, run_if);
    const int64_t tot = (int64_t)M * N;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part, nsplit, M, N,
                       sym, G_dev, run_if);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

template <int MG>
static void combine_launch(const float* C, int K, int M, int m0, const float* Y, int64_t ldy, float* Out,
                           int64_t ldo, int64_t L, float beta, int upper, hipStream_t s, const int* run_if)
{
    dim3 grid((unsigned)((L + 127) / 128));
    // 16-byte loads of Y need 16-byte aligned rows
    const bool vy = (((uintptr_t)Y) & 15) == 0 && (ldy % 4) == 0;
    if (vy)
        hipLaunchKernelGGL((k_combine<MG, true>), grid, dim3(256), 0, s, C, K, M, m0, Y, ldy, Out, ldo, L, beta, upper,
                           run_if);
    else
        hipLaunchKernelGGL((k_combine<MG, false>), grid, dim3(256), 0, s, C, K, M, m0, Y, ldy, Out, ldo, L, beta, upper,
                           run_if);
}

int combine(const float* C, int K, int M, const float* Y, int64_t ldy, float* Out, int64_t ldo, int64_t L,
            float beta, hipStream_t s, bool upper, const int* run_if)
{
    const int up = upper ? 1 : 0;
    if (M <= 0 || L <= 0) return RTT_OK;
    if (M <= 32 && (((uintptr_t)Y) & 15) == 0 && (ldy % 4) == 0 && (((uintptr_t)Out) & 15) == 0 && (ldo % 4) == 0) {
        const int64_t waves = (L + 127) / 128;
        hipLaunchKernelGGL(k_combine_skinny, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, C, K, M, Y, ldy, Out,
                           ldo, L, beta, run_if);
        RTT_HIP(hipGetLastError());
        return RTT_OK;
    }
    // at most COMBINE_ROW_BLOCKS row blocks of 32 per launch: their accumulators leave room for
    // three waves per SIMD, which cover a chunk's loads
    constexpr int COMBINE_ROW_BLOCKS = 4;
    auto launch = [&](int m0, int mg) {
        static_assert(COMBINE_ROW_BLOCKS == 4, "one case per row-block count below");
        switch (mg) {
        case 1: combine_launch<1>(C, K, M, m0, Y, ldy, Out, ldo, L, beta, up, s, run_if); break;
        case 2: combine_launch<2>(C, K, M, m0, Y, ldy, Out, ldo, L, beta, up, s, run_if); break;
        case 3: combine_launch<3>(C, K, M, m0, Y, ldy, Out, ldo, L, beta, up, s, run_if); break;
        default: combine_launch<4>(C, K, M, m0, Y, ldy, Out, ldo, L, beta, up, s, run_if); break;
        }
    };
    // upper: a launch reads the rows of Y up to its last output row, so the launch with fewer row
    // blocks takes the top rows (a 288-row C: 32 + 160 + 288 rows of Y read, not 128 + 256 + 288).
    // A tile's products and their order depend only on its rows, not on the launch it falls in.
    const int nblk = (M + 31) / 32, head = upper ? nblk % COMBINE_ROW_BLOCKS : 0;
    if (head) launch(0, head);
    for (int m0 = head * 32; m0 < M; m0 += COMBINE_ROW_BLOCKS * 32)
        launch(m0, std::min(COMBINE_ROW_BLOCKS, (M - m0 + 31) / 32));
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int normal_add(float* y, int64_t n, uint64_t seed, float sigma, hipStream_t s)
{
    if (n <= 0) return RTT_OK;
    const int64_t q = (n + 3) / 4;
    hipLaunchKernelGGL(k_normal_add, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, y, n, seed, sigma);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int normal_fill(float* out, int64_t n, uint64_t seed, hipStream_t s)
{
    const int64_t q = (n + 3) / 4;
    hipLaunchKernelGGL(k_normal, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, out, n, seed, (uint64_t)0);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int dots_seg(Workspace& ws, const float* a, int64_t lda, const float* b, int64_t ldb, const int64_t* seg_dev,
             int G, int64_t max_len, int nvec, double* out_dev, hipStream_t s)
{
    if (nvec <= 0 || G <= 0) return RTT_OK;
    const int nsplit = (int)std::min<int64_t>(std::max<int64_t>(1, max_len / 4096), 256);
    double* part = (double*)ws.get("dotseg_part", sizeof(double) * (size_t)nsplit * nvec * G);
    if (!part) return fail(RTT_ENOMEM, "dot workspace");
    hipLaunchKernelGGL(k_dot_partial_seg, dim3((unsigned)nsplit, (unsigned)nvec, (unsigned)G), dim3(256), 0, s, a,
                       lda, b, ldb, seg_dev, G, part);
    const int tot = nvec * G;
    hipLaunchKernelGGL(k_dot_final, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, s, part, nsplit, tot, out_dev);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return RTT_OK;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int scale_inv_sq(const double* Cd, const double* sigma_dev, int sets, int t, int k, int nrhs, double sigma_min,
                 float* C, hipStream_t s)
{
    const int64_t n = (int64_t)sets * t * nrhs;
    if (n <= 0) return RTT_OK;
    hipLaunchKernelGGL(k_scale_inv_sq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Cd, sigma_dev, sets, t, k,
                       nrhs, sigma_min, C);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

int dots(Workspace& ws, const float* a, int64_t lda, const float* b, int64_t ldb, int64_t n, int nvec,
         double* out_dev, hipStream_t s)
{
    const int nsplit = (int)std::min<int64_t>(std::max<int64_t>(1, n / 4096), 256);
    const int64_t slice = (n + nsplit - 1) / nsplit;
    double* part = (double*)ws.get("dot_part", sizeof(double) * (size_t)nsplit * nvec);
    if (!part) return fail(RTT_ENOMEM, "dot workspace");
    hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)nsplit, (unsigned)nvec), dim3(256), 0, s, a, lda, b, ldb, n,
                       slice, part);
    hipLaunchKernelGGL(k_dot_final, dim3((unsigned)((nvec + 127) / 128)), dim3(128), 0, s, part, nsplit, nvec,
                       out_dev);
    RTT_HIP(hipGetLastError());
    return RTT_OK;
}

}  // namespace rtt
