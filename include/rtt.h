/*
 * rtt.h -- C ABI of the MI355X retarded-time tomography library.
 *
 * The library evaluates the order-resolved retarded-time imaging operator of
 * "Photon-Ring Retarded-Time Tomography" (Sec. 3.1, eq. (2)-(3); App. A.2,
 * eq. (47)) and its transpose on one GPU, and builds the spectral quantities
 * and estimators on top of it: randomized SVD / block Lanczos singular values
 * (Sec. 3.6 eq. (19), Sec. 4.4 eq. (31)), the TSVD and ridge estimates of
 * Sec. 9, and the order mixers of Sec. 3.1 eq. (4) (unresolved image, total
 * flux) with their covariance propagation.
 *
 * Discretisation.  A source history is a coefficient vector x[s][k] over
 * n_r x n_phi polar cells (s = i*n_phi + j; nodal bilinear basis on the cell
 * centres, uniform in r over [r_in, r_out], periodic in phi, constant over the
 * half cells next to r_in and r_out) times n_hat degree-one B-spline hats
 * centred at s_k = s0 + k*dt_src with half-width dt_src (Sec. 7).  A datum is
 * indexed by (order n, ray p, frame f) with t_f = t0 + f*dt_obs and equals
 *     w_{n,p} * sum_s psi_s(r_{n,p}, phi_{n,p}) * sum_k tau_k(t_f - Delta_{n,p}) * x[s][k].
 *
 * Conventions shared by every entry point:
 *  - All float arrays passed to compute calls are DEVICE pointers to FP32,
 *    contiguous and 4-byte aligned (16-byte alignment of data rows lets the
 *    forward kernel use vector stores); they stay owned by the caller.
 *  - A coefficient block is [nvec][n_cols] with n_cols = n_r*n_phi*n_hat
 *    (k fastest).  A data block is [nvec][n_rows] with rows ordered
 *    (order n, caller ray p, frame f), frames fastest.  For a handle holding
 *    G > 1 geometries the operator is block diagonal: columns and rows are the
 *    per-geometry blocks concatenated in geometry order (offsets from
 *    geometry_info).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Compute calls are
 *    asynchronous on it unless stated otherwise.
 *  - Return value 0 (RTT_OK) or a negative RTT_E* code; on error nothing has
 *    been launched and last_error() holds a message for the calling thread.
 *    No C++ exception crosses this boundary.
 *  - The ratio dt_obs/dt_src must be a rational P/Q with Q <= 64, P <= 4096.
 */
#ifndef RTT_H
#define RTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RTT_OK = 0,
    RTT_EINVAL = -1,   /* bad argument, shape or value                         */
    RTT_ENOMEM = -2,   /* device or host allocation failed                     */
    RTT_EDEVICE = -3,  /* a HIP runtime call failed                             */
    RTT_ENOCONV = -4,  /* an iteration stopped before reaching its tolerance    */
    RTT_ESTATE = -5    /* object in the wrong state (e.g. freed, no factors)    */
};

typedef struct rtt_geometry rtt_geometry; /* opaque; owns the device ray tables */
typedef struct rtt_svd rtt_svd;           /* opaque; owns device singular factors */

/* Observer frames, polar source cells and source-time hats of one geometry. */
typedef struct {
    int32_t n_orders;  /* image orders 0..n_orders-1 (1..8)                    */
    int32_t n_frames;  /* observer frames, t_f = t0 + f*dt_obs                  */
    double t0, dt_obs;
    int32_t n_r, n_phi;/* polar cells, n_r >= 2, n_phi >= 1                      */
    double r_in, r_out;
    int32_t n_hat;     /* hats at s_k = s0 + k*dt_src, n_hat >= 2                */
    double s0, dt_src;
} rtt_grid;

/* Retained rays of one order (Sec. 3.1: chi = 1 rays only).  Host FP64
 * arrays, caller-owned, copied by geometry_load. */
typedef struct {
    int64_t n_rays;
    const double* r_src;      /* source radius r_{n,p}                            */
    const double* phi_src;    /* source azimuth phi_{n,p} (any real; folded mod 2 pi) */
    const double* delay;      /* coordinate-time delay Delta_{n,p}                 */
    const double* weight;     /* transfer weight w_{n,p} (incl. order weight, g^3) */
    const double* pixel_area; /* nullable: solid angle dOmega_p for whitening     */
} rtt_raymap;

typedef struct {
    double sigma_omega;   /* noise density of eq. (15); with pixel_area set, rows
                             are whitened by sqrt(dOmega_p)/sigma_omega (eq. (16));
                             0 means 1                                            */
    int32_t drop_invalid; /* 1: rays with r_src outside [r_in, r_out] get chi = 0
                             (their rows are written as zeros); 0: RTT_EINVAL     */
    int32_t reserved[5];
} rtt_load_opts;

typedef struct {
    int32_t n_geometries;
    int64_t n_rows;        /* total rows (all geometries, all orders)          */
    int64_t n_cols;        /* total columns                                    */
    int64_t n_rays;        /* total retained rays                              */
    int64_t table_bytes;   /* device bytes held by the handle                  */
    int32_t batch_apply_mode;   /* launch mode of whole-operator op_apply (below)  */
    int32_t batch_adjoint_mode; /* launch mode of whole-operator op_apply_adjoint  */
    int32_t apply_launches;     /* kernel launches of one whole-operator op_apply /  */
    int32_t adjoint_launches;   /* op_apply_adjoint call with the current variants   */
} rtt_geometry_info;

/* Per-geometry layout inside a handle (geometry g of geometry_info). */
typedef struct {
    rtt_grid grid;
    int64_t row_offset, n_rows;  /* rows of this geometry inside a data vector */
    int64_t col_offset, n_cols;  /* columns inside a coefficient vector       */
    int64_t rays_per_order[8];
    int32_t apply_variant;       /* kernel variant used by op_apply            */
    int32_t adjoint_variant;     /* kernel variant used by op_apply_adjoint    */
    uint64_t digest;             /* FNV-1a hash of the grid and device tables  */
} rtt_member_info;

/*
 * geometry_load -- validate ray maps, build the device ray tables.
 * grids[G], maps[sum_g grids[g].n_orders] (maps of geometry 0 first, by order).
 * Per ray, in FP64 on the host: the bilinear stencil of (r, phi) and the hat
 * index/fraction of t0 - Delta; rays are then sorted by base cell and cast to
 * a 32-byte device record (eq. (47) row data).  Blocking: ends with the tables
 * resident on the current device.  opts may be NULL.  *out receives a handle
 * to release with geometry_free.
 * Errors: RTT_EINVAL (sizes, NaN/Inf, r outside range without drop_invalid,
 * unsupported dt_obs/dt_src ratio), RTT_ENOMEM, RTT_EDEVICE.
 */
int geometry_load(const rtt_grid* grids, const rtt_raymap* maps, int32_t n_geometries,
                  const rtt_load_opts* opts, rtt_geometry** out);
int geometry_free(rtt_geometry* geom);
int geometry_info(const rtt_geometry* geom, rtt_geometry_info* info);
int geometry_member(const rtt_geometry* geom, int32_t g, rtt_member_info* info);

/*
 * geometry_set_variant -- pin the kernel variant of op_apply / op_apply_adjoint
 * for member g (-1: every member); -1 leaves a variant unchanged.  Variants
 * compute the same operator with different tilings; names via
 * variant_name().  Errors: RTT_EINVAL for an unknown index.
 */
int geometry_set_variant(rtt_geometry* geom, int32_t g, int32_t apply_variant, int32_t adjoint_variant);
/*
 * geometry_set_batch_mode -- how op_apply / op_apply_adjoint (and the drivers
 * built on them) launch a handle with G > 1 geometries: 0 = one launch per
 * geometry; 1 (default) = one launch for up to 16 geometries, their blocks
 * numbered consecutively; 2 = the same launch made persistent (2048 blocks
 * that stride over the work).  Modes 1 and 2 apply when every geometry of the
 * group uses one lean, absolute-hat (abs4) or register forward variant and a
 * visit-list adjoint variant, with one common dt_obs/dt_src; otherwise the
 * call falls back to one launch per geometry.
 * -1 leaves a mode unchanged.  geometry_tune picks the fastest.  All modes give
 * bitwise identical results.  Errors: RTT_EINVAL for other values.
 */
int geometry_set_batch_mode(rtt_geometry* geom, int32_t apply_mode, int32_t adjoint_mode);

/* Name of variant v of the forward (adjoint = 0) or adjoint (1) kernel, NULL if out of range. */
const char* variant_name(int32_t adjoint, int32_t v);

/*
 * geometry_tune -- autotuner: times every applicable variant of both kernels
 * on nvec random vectors (HIP events on `stream`, median of `reps`) for each
 * member at its place in the handle's [nvec][n_rows] data layout (the 128-byte
 * phase of its rows, which row stores are sensitive to; member cache keys
 * combine the member's content digest with that phase), keeps the fastest,
 * then (G > 1) times the whole operator with those
 * choices launched per member against one variant shared by every member in
 * one launch (launch modes of geometry_set_batch_mode), keeps the fastest, and
 * records the choices in the text cache at cache_path (nullable; one "digest
 * nvec apply adjoint" line per member, one "multi digest nvec apply_mode
 * adjoint_mode apply_shared adjoint_shared" line per handle).  When every
 * member images one source grid, the whole-operator forward is timed as
 * op_apply_shared, the form a batch of histories uses.  A cache hit skips the
 * timing.  Blocking; allocates scratch vectors.
 */
int geometry_tune(rtt_geometry* geom, int32_t nvec, int32_t reps, const char* cache_path, void* stream);

/*
 * op_apply -- y = A x (Sec. 3.1 eq. (2)-(3), App. A.2 eq. (47)).
 * x: device [nvec][n_cols]; y: device [nvec][n_rows].  Rows of orders whose
 * bit is clear in order_mask (bit n = order n) are neither written nor read;
 * order_mask = 0 selects all orders.  Deterministic.
 */
int op_apply(const rtt_geometry* geom, const float* x, float* y, int32_t nvec,
             uint32_t order_mask, void* stream);

/*
 * op_apply_shared -- y = A x for a handle whose G geometries share one source
 * grid (equal n_r, n_phi, n_hat, r_in, r_out, s0, dt_src): every geometry
 * images the same coefficient vector, as when one source history is seen
 * through several spin/inclination geometries.  x: device [nvec][n_cols / G]
 * (one member's columns); y: device [nvec][n_rows] (every member's rows).
 * The result is op_apply applied to x repeated in every member's column block,
 * bit for bit, but each coefficient block is read once per vector instead of
 * once per geometry.  Its transpose with respect to x is the sum over members
 * of the column blocks op_apply_adjoint returns.  Rows of orders outside
 * order_mask are neither written nor read.  Errors: RTT_EINVAL when the
 * members' source grids differ, as op_apply otherwise.
 */
int op_apply_shared(const rtt_geometry* geom, const float* x, float* y, int32_t nvec,
                    uint32_t order_mask, void* stream);

/*
 * op_apply_adjoint -- x = A^T y, the exact transpose of op_apply (the
 * transposed action whose consistency Sec. 5 validates), computed
 * owner-by-owner without atomics; x is overwritten.  Bitwise reproducible
 * for fixed inputs.
 */
int op_apply_adjoint(const rtt_geometry* geom, const float* y, float* x, int32_t nvec,
                     uint32_t order_mask, void* stream);

/* ------------------------------------------------------------------ spectra */
enum { RTT_SVD_RSVD = 0, RTT_SVD_BLOCK_LANCZOS = 1 };
/* rtt_svd_opts.geometry: factorise every geometry of the handle on its own (rSVD only). */
enum { RTT_EACH_GEOMETRY = -2 };

typedef struct {
    int32_t method;     /* RTT_SVD_RSVD or RTT_SVD_BLOCK_LANCZOS                 */
    int32_t k;          /* wanted singular triplets                              */
    int32_t p;          /* oversampling (rSVD): block l = k + p                   */
    int32_t q;          /* power iterations (rSVD)                                */
    int32_t block;      /* Lanczos block size b                                   */
    int32_t steps;      /* Lanczos steps (b*steps right vectors)                  */
    uint32_t order_mask;/* rows used (0 = all)                                    */
    int32_t geometry;   /* member geometry g (vectors of that geometry alone), -1 =
                           the whole operator, RTT_EACH_GEOMETRY = every geometry
                           separately in one call (full-length vectors)           */
    uint64_t seed;      /* used when omega == NULL (counter-based normal draws)   */
    int32_t keep_u;     /* 1: also store left vectors (rSVD)                       */
    int32_t reserved[3];
} rtt_svd_opts;

/*
 * rsvd -- leading singular triplets of A (Sec. 3.6 eq. (19) with C = I).
 * rSVD: randomized subspace iteration (Halko, Martinsson & Tropp 2011,
 * Alg. 4.4) with block l = k + p, q power iterations, orthonormalisation by
 * Cholesky QR (FP32 MFMA Gram, FP64 factor and inverse on the device, no host
 * round trip) after every application, and the FP64 SVD of the projected
 * l x l factor on the host (one download).  Block Lanczos: block Golub-Kahan
 * with one-sided FP64 reorthogonalisation.  omega: device FP32 [l][n_cols]
 * start block (NULL: drawn from seed).  Blocking (returns after the small SVD);
 * not capturable into a graph as a whole.
 * With geometry = RTT_EACH_GEOMETRY the G geometries of the handle are
 * factorised independently in one run: every application of A or A^T is one
 * batched call on the whole handle, every orthonormalisation and small SVD is
 * done per geometry block; row i of V then holds the i-th right singular
 * vector of every geometry in that geometry's column block.
 */
int rsvd(const rtt_geometry* geom, const rtt_svd_opts* opts, const float* omega,
         rtt_svd** out, void* stream);
int svd_free(rtt_svd* s);
/* sigma_host[k] (FP64 host, descending), *V_dev = device [k][n_cols] FP32
 * right vectors, *U_dev = device [k][n_rows] left vectors or NULL,
 * resid_host[k] = ||A v_i - sigma_i u_i|| (rSVD with keep_u) or the Ritz
 * residual estimate (Lanczos).  For RTT_EACH_GEOMETRY factors sigma_host and
 * resid_host receive [G][k] values.  Any output pointer may be NULL.  *k_out
 * receives k.  Pointers stay owned by s. */
int svd_get(const rtt_svd* s, int32_t* k_out, double* sigma_host, const float** V_dev,
            const float** U_dev, double* resid_host);

/*
 * svd_converged -- how many singular values of the factors count as converged:
 * count[q] = #{ i : resid_i <= rel_tol * sigma_1 } for each factorisation q
 * (one, or G for RTT_EACH_GEOMETRY factors; count has room for as many), with
 * resid_i the residual svd_get reports (block Lanczos: the Ritz residual
 * estimate ||A^T u_i - theta_i v_i|| of the recurrence; rSVD with keep_u:
 * ||A v_i - sigma_i u_i||).  The operational rank of Sec. 4.4 eq. (31) counts
 * singular values above a threshold, so only converged values should enter it
 * (rel_tol = 1e-6 is the usual choice).  Host arithmetic on the stored values.
 * Errors: RTT_EINVAL (bad handle, NULL count, rel_tol < 0); RTT_ESTATE when
 * the factors carry no residuals (rSVD without keep_u).
 */
int svd_converged(const rtt_svd* s, double rel_tol, int32_t* count);

/*
 * tsvd_solve -- TSVD estimate of Sec. 9: x = V_t diag(sigma_t^-2) V_t^T A^T y
 * (= sum_{i<t} v_i (u_i . y)/sigma_i for an exact factorisation).
 * y: device [nrhs][n_rows]; x: device [nrhs][n_cols], with the lengths of the
 * factorised operator (one geometry's for factors of a member g, the handle's
 * otherwise; RTT_EACH_GEOMETRY factors solve every geometry with its own
 * factors).  t <= k keeps the t leading components; t <= 0 keeps those with
 * sigma_i >= sigma_min (per geometry).  Zero singular values are never kept.
 * Stream-ordered (no host synchronisation).  Scratch memory is kept by s and
 * only grows, so a call with no more right-hand sides than an earlier one
 * allocates nothing and may be captured into a hipGraph; calls on one s must
 * not overlap in time.
 */
int tsvd_solve(const rtt_geometry* geom, const rtt_svd* s, const float* y, int32_t nrhs,
               int32_t t, double sigma_min, float* x, void* stream);

enum { RTT_SOLVE_ASYNC = 1, RTT_SOLVE_NORMAL_RHS = 2 };

typedef struct {
    float tol;          /* stop when ||r|| <= tol ||A^T y|| (per right-hand side
                           and geometry)                                         */
    int32_t maxit;      /* iteration cap (RTT_SOLVE_ASYNC: iteration count)      */
    uint32_t order_mask;
    int32_t flags;      /* RTT_SOLVE_ASYNC: stream-ordered, see ridge_solve;     */
                        /* RTT_SOLVE_NORMAL_RHS: y is a right-hand side b        */
    float* resid_dev;   /* nullable device FP32 [nrhs][G]: final ||r||/||A^T y||  */
    int32_t reserved[2];
} rtt_cg_opts;

typedef struct {
    int32_t iterations;  /* largest iteration count over right-hand sides        */
    int32_t converged;   /* number of right-hand sides that met tol               */
    float rel_residual;  /* largest final ||r||/||A^T y||                         */
    int32_t reserved;
} rtt_solve_info;

/*
 * ridge_solve -- ridge (Tikhonov) estimate of Sec. 9:
 * argmin 1/2||A x - y||^2 + lambda/2 ||x||^2, by conjugate gradients on
 * (A^T A + lambda I) x = A^T y.  Every (right-hand side, geometry) pair of
 * the block-diagonal operator runs its own CG (own step lengths, own stop
 * test), so a handle of G geometries solves G x nrhs independent problems in
 * one call.  y: device [nrhs][n_rows]; x: device [nrhs][n_cols] (overwritten;
 * the start is x = 0).  info may be NULL.
 * Default mode: blocking; returns RTT_ENOCONV if some pair did not reach tol
 * within maxit (x still holds the iterate; info counts pairs).
 * flags & RTT_SOLVE_ASYNC: stream-ordered, no host synchronisation: exactly
 * maxit iterations are enqueued (a pair that meets tol stops changing), the
 * final relative residuals go to opts->resid_dev when given, info (if any)
 * gets iterations = maxit and converged = -1.  Scratch memory is kept by the
 * handle and only grows, so a call that needs no more than an earlier one
 * allocates nothing and may be captured into a hipGraph.  Asynchronous solves
 * on one handle must not overlap in time (they share that scratch).
 */
int ridge_solve(const rtt_geometry* geom, const float* y, int32_t nrhs, float lambda,
                const rtt_cg_opts* opts, float* x, rtt_solve_info* info, void* stream);
/* With flags & RTT_SOLVE_NORMAL_RHS, ridge_solve solves (A^T A + lambda I) x = b
 * for a coefficient block b passed in place of y (device [nrhs][n_cols]); the
 * relative residual is then ||r|| / ||b||.  This is the one extra solve that
 * the derivative of the ridge estimate with respect to the data needs:
 * d<g, x_hat(y)>/dy = A (A^T A + lambda I)^{-1} g (the normal matrix is
 * symmetric). */

/*
 * tsvd_project -- x = V_t diag(sigma_t^-2) V_t^T b for a coefficient block b
 * (device [nrhs][n_cols]; must not overlap x), the map that tsvd_solve applies
 * after A^T (Sec. 9): tsvd_solve(y) = tsvd_project(A^T y), and the derivative
 * of <g, tsvd_solve(y)> with respect to y is A tsvd_project(g).  Arguments,
 * truncation and stream behaviour as tsvd_solve.
 */
int tsvd_project(const rtt_geometry* geom, const rtt_svd* s, const float* b, int32_t nrhs, int32_t t,
                 double sigma_min, float* x, void* stream);

/*
 * noise_add -- y[i] += sigma * z_i, i < n, with seeded N(0, 1) draws z (white
 * data noise; at a sweep point sigma = sigma_Omega = s_ref / SNR0 of
 * eq. (18) for whitened rows).  Draws: group i of four takes the
 * Philox-4x32-10 block (Salmon et al., SC'11) of counter (i mod 2^32,
 * i >> 32, 0, 0) and key (seed mod 2^32, seed >> 32); words w map to uniforms
 * (w + 1/2) 2^-32 and the pairs (u0, u1), (u2, u3) to Box-Muller normals
 * r cos(2 pi u'), r sin(2 pi u'), r = sqrt(-2 ln u), in FP32.  The same seed
 * gives the same draws for any n.  Stream-ordered.  Errors: RTT_EINVAL.
 */
int noise_add(float* y, int64_t n, uint64_t seed, float sigma, void* stream);

/* -------------------------------------------------------------- order mixer */
/*
 * Order mixers L of Sec. 3.1 eq. (4): d_L = (L kron I) d_R collapses the
 * order-resolved rows of a handle (eq. (3)) into a coarser observation, and
 * its noise follows through C_L = (L kron I) C_R (L^T kron I).  Two kinds:
 *  - RTT_MIX_UNRESOLVED: the unresolved spatial image.  Each ray carries the
 *    index of the image pixel it lands on; the rays of every order that share
 *    a pixel are added.  A geometry's mixed rows are its distinct pixels in
 *    ascending index order, each a row of n_frames frames.
 *  - RTT_MIX_TOTAL_FLUX: the total-flux readout, one row (n_frames frames)
 *    per geometry adding every ray of every order.
 * A mixed data block is [nvec][n_rows] (mixer_info), geometries concatenated
 * in handle order (offsets from mixer_member).  Every sum runs in a fixed
 * order (source rays in data-row order, in chunks of 64 whose partial rows are
 * then added in chunk order), so results are bitwise reproducible.
 */
typedef struct rtt_mixer rtt_mixer; /* opaque; owns the device gather tables */
enum { RTT_MIX_UNRESOLVED = 0, RTT_MIX_TOTAL_FLUX = 1 };

typedef struct {
    int32_t kind;          /* RTT_MIX_*                                          */
    int32_t n_geometries;
    int64_t n_rows;        /* rows of a mixed data vector (all geometries)       */
    int64_t n_src_rows;    /* rows of the handle's order-resolved data vectors   */
    int32_t reserved[4];
} rtt_mixer_info;

/*
 * mixer_create -- build the mixer of kind `kind` for every geometry of geom.
 * pixels (RTT_MIX_UNRESOLVED only, else may be NULL): host arrays in the
 * order of geometry_load's ray maps (geometry 0's orders first), pixels[i]
 * holding one int64 pixel index >= 0 per ray of ray map i (NULL allowed for
 * an empty map); caller-owned, copied.  Pixel indices are local to a
 * geometry.  Blocking; *out receives a handle to release with mixer_free.
 * The mixer does not keep geom.  Errors: RTT_EINVAL (bad kind, handle, NULL
 * or negative pixels), RTT_ENOMEM, RTT_EDEVICE.
 */
int mixer_create(const rtt_geometry* geom, int32_t kind, const int64_t* const* pixels, rtt_mixer** out);
int mixer_free(rtt_mixer* mixer);
int mixer_info(const rtt_mixer* mixer, rtt_mixer_info* info);
/* Mixed rows of geometry g: offset and length inside a mixed data vector, and
 * the number of mixed rows (pixels, or 1 for the total flux).  Any output
 * pointer may be NULL.  Errors: RTT_EINVAL for a bad handle or index. */
int mixer_member(const rtt_mixer* mixer, int32_t g, int64_t* row_offset, int64_t* n_rows, int64_t* n_out);

/*
 * mixer_set_variant -- pin how many vectors of a block one wave of mix_apply /
 * mix_covariance (apply_vectors) or of mix_adjoint (adjoint_vectors) handles:
 * 1, 2, 4 or 8; 0 = chosen per call (forward: 1 when mixed rows average 16 or
 * more source rays, else 8; transpose: 4; either halved while the launch
 * would have fewer than 32768 waves); -1 leaves a choice unchanged.  Every
 * choice gives bitwise identical results.
 * Errors: RTT_EINVAL for other values or a bad handle.
 */
int mixer_set_variant(rtt_mixer* mixer, int32_t apply_vectors, int32_t adjoint_vectors);

/*
 * mix_apply -- d = (L kron I) y (eq. (4)).  y: device [nvec][n_src_rows]
 * order-resolved data; d: device [nvec][n_rows], overwritten.  A mixer with
 * rows of more than 64 rays keeps a partial-row scratch buffer of
 * (number of chunks) x (largest n_frames) x nvec floats, allocated on the
 * first call that needs more and reused after; calls on one mixer must not
 * overlap in time.  0 <= nvec <= 65535.  Errors: RTT_EINVAL, RTT_ENOMEM,
 * RTT_EDEVICE.
 */
int mix_apply(const rtt_mixer* mixer, const float* y, float* d, int32_t nvec, void* stream);

/*
 * mix_apply_noalloc -- mix_apply for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same bits as mix_apply, with the
 * partial rows of multi-chunk mixed rows (the total flux) in a library-static
 * device array of RTT_MIX_NOALLOC_SCRATCH_BYTES per GPU (held by every GPU the
 * library runs on until the process ends) instead of a buffer owned by the
 * mixer.  Calls no allocating routine.  A call needs
 * (number of chunks) x (largest n_frames rounded up to 4) x nvec x 4 bytes of
 * it; larger calls are rejected with RTT_EINVAL (nothing launched) and the
 * message names the vector limit.  Every call on one GPU shares that GPU's
 * array (each call writes what it reads), so calls that overlap in time on
 * one GPU -- on different streams or threads -- race; serialise them.
 * Errors: as mix_apply, RTT_EDEVICE when the array's address cannot be taken.
 */
#define RTT_MIX_NOALLOC_SCRATCH_BYTES (16u << 20)
int mix_apply_noalloc(const rtt_mixer* mixer, const float* y, float* d, int32_t nvec, void* stream);

/*
 * mix_adjoint -- y = (L^T kron I) d: every order-resolved row receives the
 * mixed row its ray feeds.  d: device [nvec][n_rows]; y: device
 * [nvec][n_src_rows], every row overwritten.  Allocates nothing.
 */
int mix_adjoint(const rtt_mixer* mixer, const float* d, float* y, int32_t nvec, void* stream);

/*
 * mix_covariance -- C_L of eq. (4) for a diagonal C_R = diag(var).  Each
 * order-resolved row feeds exactly one mixed row, so C_L is diagonal too and
 * its diagonal is the mixed sum of the variances: var: device [n_src_rows];
 * var_out: device [n_rows] (the diagonal of C_L).  Same scratch rule as
 * mix_apply.
 */
int mix_covariance(const rtt_mixer* mixer, const float* var, float* var_out, void* stream);

/* ------------------------------------------------------- age information */
/*
 * reference_response -- s_ref of Sec. 3.5 eq. (17) for every geometry g of
 * the handle: sqrt(||A_{g,0} j_ref||^2 / m_0) with the constant reference
 * emissivity j_ref = 1 on every coefficient (the bilinear cells and the hats
 * both reproduce constants) and m_0 the direct-order rows of g.  The noise
 * density of a sweep point is sigma_Omega = s_ref / SNR0 (eq. (18)).
 * s_ref: host double[G].  Blocking.  Errors: RTT_EINVAL, RTT_ENOMEM,
 * RTT_EDEVICE.
 */
int reference_response(const rtt_geometry* geom, double* s_ref, void* stream);

/*
 * age_information -- the squared responses of eq. (12) / (29) to the
 * age-localised probes of Sec. 3.3 eq. (10)-(11): for every age a the probe
 * q_a, flat over the annulus and exp(-(t + a)^2 / (2 h^2)) / N_h in source
 * time, N_h^2 = pi (r_out^2 - r_in^2) h sqrt(pi), is set on the coefficient
 * nodes (every cell, hat k at s_k) and A is applied to it.
 * mixer == NULL: energy (host double [n_ages][G][8]) receives ||A_{g,n} q_a||^2
 * for every geometry g and order n (0 for n >= n_orders): the direct arm is
 * n = 0, the resolved stack the sum over n.  mixer != NULL (built on this
 * geometry): energy (host double [n_ages][G]) receives
 * ||C_L^{-1/2} (L kron I) A_g q_a||^2 with C_L = diag((L kron I) var), the
 * covariance of eq. (4) propagated from per-datum variances var (device FP32
 * [n_rows]; NULL = 1, i.e. whitened rows).  Rows are as loaded (whitened by
 * eq. (16) when pixel areas were given).  Multiply by SNR0^2 / s_ref^2 for the
 * information at a sweep point.  ages: host double[n_ages]; h > 0 (the paper
 * uses 3M).  Blocking; scratch of at most about 1 GiB is allocated per call.
 * Errors: RTT_EINVAL, RTT_ENOMEM, RTT_EDEVICE.
 */
int age_information(const rtt_geometry* geom, const double* ages, int32_t n_ages, double h,
                    const rtt_mixer* mixer, const float* var, double* energy, void* stream);

/*
 * age_window -- for geometry g and the orders in order_mask (0 = all):
 * [*a_min, *a_max], the ages whose probe support |t + a| <= 3h lies inside
 * the source-time window that those orders reach (eq. (13)); a_min > a_max
 * when none does.  boundary (nullable): A_{0,q} of eq. (35), the smallest age
 * of a direct datum (ray p, frame f: age Delta_p - t_f) such that the data of
 * that age or younger carry the fraction q of the direct throughput, every
 * datum weighted by |w_p| as loaded; NaN without direct rays.  Host only
 * (tables kept at load).  Errors: RTT_EINVAL (bad handle, index, h, q).
 */
int age_window(const rtt_geometry* geom, int32_t g, uint32_t order_mask, double h, double q,
               double* a_min, double* a_max, double* boundary);

typedef struct {
    double t_reach;     /* oldest passing age (eq. (30)); NaN if none passes        */
    double l_anchor;    /* extent of the passing run that starts at the anchor;   */
                        /* NaN if there is no anchor or it does not pass          */
    double longest;     /* extent of the longest passing run; NaN if none          */
    double j_old;       /* eq. (35): sum over ages > boundary of log(1 + info)     */
                        /* times the grid step; NaN if boundary is NaN            */
    int32_t anchor;     /* index of the youngest age in [a_min, a_max]; -1: none  */
    int32_t n_pass;     /* passing ages                                          */
} rtt_reach;

/*
 * age_reach -- threshold statistics of Sec. 4.4 on an age grid (ascending,
 * equally spaced ages[n]) from the information info[n] at one sweep point
 * (SNR0^2 / s_ref^2 times age_information's energy): an age passes when
 * info >= rho^2 (eq. (30)); the anchor is the youngest age inside
 * [a_min, a_max] (age_window).  mask (nullable): n bytes, 1 = passes.  Host
 * only.  Errors: RTT_EINVAL.
 */
int age_reach(const double* ages, const double* info, int32_t n, double rho, double a_min, double a_max,
              double boundary, uint8_t* mask, rtt_reach* out);

/*
 * age_window_error -- E(a) of Sec. 4.4 eq. (32) for reconstructions x_hat of
 * x (device [nvec][n_cols]): for every vector, geometry g and age a,
 * ||W_a (x_hat - x)|| / max(||W_a x||, eta), W_a keeping every cell's
 * coefficients at the hats whose centre s_k satisfies |s_k + a| <= half_width
 * (the age window around source time -a; 2M for the paper's 4M grid).  Sums
 * of squares in FP64, fixed order.  err: host double [nvec][G][n_ages].
 * Blocking.  Errors: RTT_EINVAL, RTT_ENOMEM, RTT_EDEVICE.
 */
int age_window_error(const rtt_geometry* geom, const float* x_hat, const float* x, int32_t nvec,
                     const double* ages, int32_t n_ages, double half_width, double eta, double* err,
                     void* stream);

/* ------------------------------------------------- representation synthesis */
/*
 * A synthesis map Q_d (Sec. 3.2 eq. (5)-(8)) evaluated on the coefficient
 * nodes of one geometry g: column (a, b, c), index (a * n_az + b) * n_temporal
 * + c with n_az = 2 m_max + 1, holds R_a(r_i) Phi_b(phi_j) T_c(s_k) at node
 * (cell centre (r_i, phi_j), hat centre s_k).  R_a: clamped cubic B-splines on
 * uniform knots in log r over [r_in, r_out]; Phi_b: 1, cos m phi, sin m phi
 * (m = 1..m_max, in that order); T_c: global DCT-II modes
 * cos(pi c (t - t_lo) / (t_hi - t_lo)), or the compact temporal functions of
 * Sec. 7 (degree-one B-splines on n_temporal uniform knots from t_lo to
 * t_hi).  The default window [s0 - dt_src/2, s0 + (K - 1/2) dt_src] makes the
 * DCT-II modes on the hat nodes the discrete DCT-II vectors.  The paper's
 * S_224 is n_radial = 4, m_max = 3, n_temporal = 8.  A^(d) = A Q_d (eq. (7))
 * is op_apply after synth_expand.
 */
typedef struct rtt_synthesis rtt_synthesis; /* opaque; owns the rows of Q on the device */
enum { RTT_SYNTH_DCT = 0, RTT_SYNTH_HATS = 1 };
typedef struct {
    int32_t n_radial;    /* radial B-splines, 4..64                            */
    int32_t m_max;       /* highest azimuthal mode, 0..32                      */
    int32_t n_temporal;  /* temporal functions, 1..256 (hats: >= 2)            */
    int32_t temporal;    /* RTT_SYNTH_DCT or RTT_SYNTH_HATS                    */
    double t_lo, t_hi;   /* source-time window; t_hi <= t_lo: the default      */
    int32_t reserved[4];
} rtt_synthesis_spec;

/* Build Q for geometry g of geom (d = n_radial (2 m_max + 1) n_temporal <= 4096
 * columns; d x n_cols floats on the device).  Blocking.  Errors: RTT_EINVAL,
 * RTT_ENOMEM, RTT_EDEVICE. */
int synthesis_create(const rtt_geometry* geom, int32_t g, const rtt_synthesis_spec* spec, rtt_synthesis** out);
int synthesis_free(rtt_synthesis* synth);
/* d, the geometry's n_cols, and the device rows of Q ([d][n_cols], column c of Q
 * as row c); any output may be NULL. */
int synthesis_info(const rtt_synthesis* synth, int32_t* d, int64_t* n_cols, const float** rows);
/* x = Q_d c: c device [nvec][d], x device [nvec][n_cols] (MFMA combine).  Keeps a
 * small scratch (d x nvec floats) in the handle; calls must not overlap. */
int synth_expand(const rtt_synthesis* synth, const float* c, float* x, int32_t nvec, void* stream);
/* c = Q_d^T x (the transpose, so Q_d^T A^T is the adjoint of A^(d)): x device
 * [nvec][n_cols], c device [nvec][d]; FP64 accumulation (MFMA Gram). */
int synth_project(const rtt_synthesis* synth, const float* x, float* c, int32_t nvec, void* stream);
/*
 * synthesis_audit -- rank audit of A^(d) = A Q_d restricted to the rows of
 * the orders in order_mask (0 = all): zero (nullable, host uint8[d]) flags the
 * columns that are exactly zero (every datum 0, the Sec. 7 blindness); sigma
 * (nullable, host double[d]) receives the singular values, descending, as the
 * square roots of the eigenvalues of the FP64 Gram (A^(d))^T A^(d) — resolved
 * down to about 1e-7 of sigma_1.  Blocking; allocates d x rows floats.
 */
int synthesis_audit(const rtt_geometry* geom, const rtt_synthesis* synth, uint32_t order_mask, double* sigma,
                    uint8_t* zero, void* stream);

/*
 * age_fisher -- the age-local Fisher matrix M(a) = P(a)^T P(a) of Sec. 3.3
 * eq. (14) for the localised probes q_{a,l} = psi_l(r, phi) g_a(t) / N_{h,l},
 * psi_l = R_a Phi_b the spatial functions of the synthesis `spatial` (l =
 * a (2 m_max + 1) + b; its temporal functions are not used), g_a the Gaussian
 * of eq. (10) with width h, N_{h,l} their continuum L2 norm over the annulus
 * and time (radial integral by Gauss-Legendre quadrature), set on the
 * coefficient nodes of the synthesis' geometry; P(a) = A q_{a,l} on the rows
 * of the orders in order_mask (0 = all), C = I (rows as loaded).  M: host
 * double [n_ages][L][L], L = n_radial (2 m_max + 1); FP64 Gram of the FP32
 * responses.  Blocking.  Errors: RTT_EINVAL, RTT_ENOMEM, RTT_EDEVICE.
 */
int age_fisher(const rtt_geometry* geom, const rtt_synthesis* spatial, const double* ages, int32_t n_ages, double h,
               uint32_t order_mask, double* M, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTT_H */
