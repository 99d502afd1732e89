/*
 * CPU FP64 oracle of the retarded-time imaging operator A and its transpose.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference the GPU library is checked against.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product path
 * never does, and it shares no code, header or table with the GPU library.
 *
 * What it computes (Sec. 3.1 eq. (2), eq. (3); App. A.2 eq. (47)):
 * a row of the order-resolved stack is indexed by (order n, ray p, frame f)
 * and acts on a separable coefficient vector x[s][k] (spatial cell s, hat k)
 * as
 *     y[n][p][f] = w_{n,p} * sum_s psi_s(r_{n,p}, phi_{n,p})
 *                          * sum_k tau_k(t_f - Delta_{n,p}) * x[s][k]
 * with psi_s the nodal bilinear basis on polar cell centres (uniform in r,
 * periodic in phi, constant continuation over the half-cells next to r_in and
 * r_out) and tau_k the degree-one B-spline ("hat") centred at
 * s_k = s0 + k*dt_src with half-width dt_src (Sec. 7).  The adjoint is the
 * transposed accumulation in one fixed serial order.
 *
 * Every row is evaluated directly from the raw ray data in FP64: no table, no
 * sorting, no stepping between frames.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    int n_orders, n_frames;
    double t0, dt_obs;
    int n_r, n_phi;
    double r_in, r_out;
    int n_hat;
    double s0, dt_src;
} ora_grid;

/* Bilinear spatial weights of one source point: 4 cell indices and weights. */
static void spatial_stencil(const ora_grid* g, double r, double phi, int cell[4], double wgt[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    double dr = (g->r_out - g->r_in) / g->n_r;
    double dphi = two_pi / g->n_phi;
    /* radial coordinate in units of cells, measured from the first centre */
    double ur = (r - g->r_in) / dr - 0.5;
    if (ur < 0.0) ur = 0.0;
    if (ur > (double)(g->n_r - 1)) ur = (double)(g->n_r - 1);
    int i = (int)floor(ur);
    if (i > g->n_r - 2) i = g->n_r - 2;
    double fr = ur - i;
    /* azimuth folded into [0, 2 pi), periodic neighbours */
    double p = fmod(phi, two_pi);
    if (p < 0.0) p += two_pi;
    double uphi = p / dphi - 0.5;
    int j = (int)floor(uphi);
    double fphi = uphi - j;
    int j0 = ((j % g->n_phi) + g->n_phi) % g->n_phi;
    int j1 = (j0 + 1) % g->n_phi;
    cell[0] = i * g->n_phi + j0;        wgt[0] = (1.0 - fr) * (1.0 - fphi);
    cell[1] = (i + 1) * g->n_phi + j0;  wgt[1] = fr * (1.0 - fphi);
    cell[2] = i * g->n_phi + j1;        wgt[2] = (1.0 - fr) * fphi;
    cell[3] = (i + 1) * g->n_phi + j1;  wgt[3] = fr * fphi;
}

/* Hats that are nonzero-capable at source time t: up to 2 (index, value). */
static int temporal_hats(const ora_grid* g, double t, int hat[2], double val[2])
{
    double u = (t - g->s0) / g->dt_src;
    double kf = floor(u);
    double theta = u - kf;
    int n = 0;
    if (kf >= 0.0 && kf < (double)g->n_hat) { hat[n] = (int)kf; val[n] = 1.0 - theta; ++n; }
    if (kf + 1.0 >= 0.0 && kf + 1.0 < (double)g->n_hat) { hat[n] = (int)kf + 1; val[n] = theta; ++n; }
    return n;
}

static int check(const ora_grid* g)
{
    if (!g) return -1;
    if (g->n_orders < 1 || g->n_frames < 0 || g->n_r < 2 || g->n_phi < 1 || g->n_hat < 1) return -1;
    if (!(g->r_out > g->r_in) || !(g->dt_src > 0.0)) return -1;
    return 0;
}

/* y (rows n,p,f; frames fastest) = A x.  Rows of orders outside the mask are left untouched. */
int ora_forward(const ora_grid* g, const int64_t* rays_per_order, const double* r,
                const double* phi, const double* delay, const double* weight,
                const double* x, double* y, unsigned order_mask)
{
    if (check(g)) return -1;
    int64_t base = 0;
    for (int n = 0; n < g->n_orders; ++n) {
        int64_t np_ = rays_per_order[n];
        if (order_mask & (1u << n)) {
            for (int64_t p = base; p < base + np_; ++p) {
                int cell[4]; double b[4];
                spatial_stencil(g, r[p], phi[p], cell, b);
                for (int f = 0; f < g->n_frames; ++f) {
                    double t = g->t0 + f * g->dt_obs;
                    int hat[2]; double h[2];
                    int nh = temporal_hats(g, t - delay[p], hat, h);
                    double acc = 0.0;
                    for (int c = 0; c < 4; ++c)
                        for (int q = 0; q < nh; ++q)
                            acc += b[c] * h[q] * x[(int64_t)cell[c] * g->n_hat + hat[q]];
                    y[p * g->n_frames + f] = weight[p] * acc;
                }
            }
        }
        base += np_;
    }
    return 0;
}

/* x = A^T y, accumulated serially in (n, p, f, corner, hat) order; x is overwritten. */
int ora_adjoint(const ora_grid* g, const int64_t* rays_per_order, const double* r,
                const double* phi, const double* delay, const double* weight,
                const double* y, double* x, unsigned order_mask)
{
    if (check(g)) return -1;
    memset(x, 0, sizeof(double) * (size_t)g->n_r * g->n_phi * g->n_hat);
    int64_t base = 0;
    for (int n = 0; n < g->n_orders; ++n) {
        int64_t np_ = rays_per_order[n];
        if (order_mask & (1u << n)) {
            for (int64_t p = base; p < base + np_; ++p) {
                int cell[4]; double b[4];
                spatial_stencil(g, r[p], phi[p], cell, b);
                for (int f = 0; f < g->n_frames; ++f) {
                    double t = g->t0 + f * g->dt_obs;
                    int hat[2]; double h[2];
                    int nh = temporal_hats(g, t - delay[p], hat, h);
                    double v = weight[p] * y[p * g->n_frames + f];
                    for (int c = 0; c < 4; ++c)
                        for (int q = 0; q < nh; ++q)
                            x[(int64_t)cell[c] * g->n_hat + hat[q]] += b[c] * h[q] * v;
                }
            }
        }
        base += np_;
    }
    return 0;
}

/* Expose the per-ray stencil for diagnostics (cells[4], weights[4]). */
int ora_stencil(const ora_grid* g, double r, double phi, int* cells, double* weights)
{
    if (check(g)) return -1;
    spatial_stencil(g, r, phi, cells, weights);
    return 0;
}
