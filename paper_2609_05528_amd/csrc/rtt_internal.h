// Internal declarations of the retarded-time tomography library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rtt.h"

namespace rtt {

// Device record of one retained ray (32 bytes), built in FP64 on the host from
// (r, phi, delay, weight) and cast once (the row data of eq. (47)).
struct alignas(16) RayRec {
    int32_t cell;   // base cell s = i*n_phi + j0 of the 2x2 bilinear stencil
    float fr;       // radial fraction: weights (1-fr) on row i, fr on row i+1
    float fphi;     // azimuthal fraction: (1-fphi) on column j0, fphi on j0+1 (periodic)
    float w;        // transfer weight (chi * w * optional whitening)
    int32_t k0;     // floor(u0), u0 = (t0 - delay - s0)/dt_src
    float th0;      // u0 - k0 in [0, 1)
    int32_t row;    // caller ray index inside the geometry (row block row*n_frames)
    int32_t order;  // image order n
};
static_assert(sizeof(RayRec) == 32, "RayRec must be 32 bytes");

// One visit of a ray by the wave that owns one cell row: the ray feeds two
// cells of that row (target columns col-1 and col of the row's sweep, in the
// segment's local numbering) with weights wa and wb (transfer weight x radial
// weight of this row x azimuthal weights).  32 bytes.
struct alignas(16) Visit {
    int32_t row;    // caller ray index (data row block row * n_frames)
    int32_t k0;     // hat origin of frame 0
    float th0;      // fraction of frame 0
    float wa;       // weight into target column (col - 1 + segment start)
    float wb;       // weight into target column (col + segment start)
    int32_t col;    // sweep position 0 .. ncol-1 (base column segment_start - 1 + col)
    int32_t order;  // image order (for order masks)
    int32_t pad;
};
static_assert(sizeof(Visit) == 32, "Visit must be 32 bytes");
// One visit of a ray by the wave that owns a pair of cell rows (2p, 2p+1): this header, then
// the weights (wa0, wb0, wa1, wb1) into the target columns col-1 and col of both rows (zero for
// a row the ray does not touch).  32 bytes.
struct alignas(16) VisitHead {
    int32_t row;        // caller ray index
    int32_t k0;         // hat origin of frame 0
    float th0;          // fraction of frame 0
    int32_t col_order;  // sweep position (low 16 bits) | image order << 16
};
static_assert(sizeof(VisitHead) == 16, "VisitHead must be 16 bytes");
constexpr int VISIT_SEG_MAX = 16;   // widest sweep segment (columns)

// Forward record of one ray (48 bytes): corner offsets and weights precomputed so
// the forward kernel does no integer division and no weight arithmetic.
struct alignas(16) FwdRec {
    int32_t c00k;   // (i*n_phi + j0) * n_hat: start of the x row of corner (i, j0)
    int32_t d01k;   // (cell(i, j0+1) - cell(i, j0)) * n_hat (periodic wrap folded in)
    float b00, b10, b01, b11;   // bilinear weights times the transfer weight
    int32_t k0;     // hat origin of frame 0
    float th0;      // fraction of frame 0
    int32_t row;    // caller ray index
    int32_t order;  // image order
    int32_t cell;   // base cell s = i*n_phi + j0
    int32_t pad1;
};
static_assert(sizeof(FwdRec) == 48, "FwdRec must be 48 bytes");

// One geometry of a handle, as the kernels see it.
struct Member {
    rtt_grid grid;
    int32_t P, Q;          // dt_obs/dt_src = P/Q exactly (1/1 when n_frames == 1)
    int64_t ray_begin;     // first record of this geometry in the sorted ray array
    int64_t n_rays;
    int64_t row_offset, n_rows;
    int64_t col_offset, n_cols;
    int64_t cell_begin;    // first CSR entry (n_cells + 1 entries)
    int64_t rays_per_order[8];
    int32_t adj_variant;   // adjoint kernel variant (default heuristic or autotuner)
    int32_t apply_variant; // forward kernel variant
    uint64_t digest;       // FNV-1a of the grid and this member's device records
    // visit-list sets: [0] single rows, 16-column segments (many vectors per call); [1] single
    // rows, narrower segments chosen so one vector alone gives enough (row, segment) tasks;
    // [2] row pairs (VisitHead + weights, 16-column segments, ceil(n_r / 2) * nseg tasks);
    // [3] base rows (VisitHead + weights into the base row and the next one; the rays of one base
    // row only, in tasks of a few columns cut to about equal visit counts, one task list per
    // parity of the base row: br_ntask[p] + 1 visit offsets, then br_ntask[p] descriptors
    // (base row * n_phi + first column) | columns << 32, from d_vtask + br_task_begin[p])
    int64_t visit_begin[4];  // first visit record of each set
    int64_t vtask_begin[3];  // first entry of each set's task offsets (rows or pairs * nseg + 1 entries)
    int32_t nseg[3];         // sweep segments per cell row
    int32_t vseg[3];         // columns per sweep segment
    int64_t br_task_begin[2], br_ntask[2];
    int32_t k0_min, k0_max;  // range of the hat origins k0 of the member's rays
    // per order: smallest and largest delay of the rays with non-zero weight (+inf / -inf if none)
    double delay_min[8], delay_max[8];
};

struct Workspace;

}  // namespace rtt

struct rtt_geometry {
    std::vector<rtt::Member> members;
    rtt::RayRec* d_rays = nullptr;      // all members, each sorted by base cell
    int32_t* d_cell_start = nullptr;    // per member CSR over base cells (relative to ray_begin)
    rtt::Visit* d_visits = nullptr;     // per member visit lists (cell row x segment tasks)
    rtt::FwdRec* d_fwd = nullptr;       // forward records, same order as d_rays
    rtt::FwdRec* d_fwd_row = nullptr;   // the same records of each member in data-row order
    int64_t* d_vtask = nullptr;         // per member task offsets into the visit lists
    int64_t* d_seg = nullptr;           // [G] (col_offset, n_cols) then [G] (row_offset, n_rows)
    // grow-only scratch of the stream-ordered (graph-capturable) solver mode, kept across calls
    mutable rtt::Workspace* solve_ws = nullptr;
    int64_t n_rows = 0, n_cols = 0, n_rays = 0;
    int64_t table_bytes = 0;
    // whole-operator calls on G > 1 members: 0 = one launch per member, 1 = one launch for
    // up to 16 members, 2 = the same as a persistent launch (one block per resident slot)
    int32_t batch_apply_mode = 1, batch_adjoint_mode = 1;
    int device = 0;
    // per member: delays and |weights| of the order-0 rays with non-zero weight (host copies for the
    // direct throughput age boundary)
    std::vector<std::vector<double>> dir_delay, dir_weight;
    uint32_t magic = 0x52545447u;
};

namespace rtt {

// thread-local error reporting ---------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define RTT_HIP(call)                                            \
    do {                                                         \
        hipError_t e__ = (call);                                 \
        if (e__ != hipSuccess) return ::rtt::hip_fail(e__, #call); \
    } while (0)

bool valid_handle(const rtt_geometry* g);
uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull);

// launchers (operator.hip) ---------------------------------------------------------------------
int launch_apply(const rtt_geometry* g, const Member& m, const float* x, float* y, int nvec,
                 int64_t x_stride, int64_t y_stride, uint32_t mask, hipStream_t s, int variant);
int launch_adjoint(const rtt_geometry* g, const Member& m, const float* y, float* x, int nvec,
                   int64_t y_stride, int64_t x_stride, uint32_t mask, hipStream_t s, int variant);
int n_adjoint_variants();
int n_apply_variants();
const char* adjoint_variant_name(int v);
const char* apply_variant_name(int v);
int default_adjoint_variant(const Member& m);
int default_apply_variant(const Member& m);
bool visit_supported(const Member& m);
bool lean_supported(const Member& m);
// forward / adjoint variant v can run on member m (ratio and size limits)
bool apply_variant_ok(const Member& m, int v);
bool adjoint_variant_ok(const Member& m, int v);

uint32_t effective_mask(const Member& m, uint32_t mask);

// A (adjoint = false) or A^T on one member (member-compact vectors of length
// n_cols / n_rows of that member) or, with member = -1, on the whole
// block-diagonal operator (full-length vectors).
int apply_op(const rtt_geometry* g, int member, bool adjoint, const float* in, float* out, int nvec,
             uint32_t mask, hipStream_t s, bool shared_x = false);
// kernel launches one whole-operator op_apply (or op_apply_adjoint) call makes with the current
// variants and launch modes (for one vector)
int whole_operator_launches(const rtt_geometry* g, bool adjoint);

// order mixers (mixer.hip) ---------------------------------------------------------------------
bool mixer_ok(const rtt_mixer* m);
int64_t mixer_rows(const rtt_mixer* m);       // rows of a mixed data vector
int64_t mixer_src_rows(const rtt_mixer* m);   // rows of the order-resolved vectors it reads
// (offset, length) of every geometry's mixed rows, appended to seg
void mixer_segments(const rtt_mixer* m, std::vector<int64_t>& seg);
// d = (L kron I) y on nvec vectors (strides in floats), stream-ordered
int mix_forward(const rtt_mixer* m, const float* y, int64_t y_stride, float* d, int64_t d_stride, int nvec,
                hipStream_t s);

}  // namespace rtt
