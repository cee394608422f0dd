/*
 * fdw_oracle.c - plain FP64 CPU oracle of the explicit leapfrog discretisation of
 *
 *     u_tt = d_x(h1(x,y) d_x u) + d_y(h2(x,y) d_y u)   on [x0,x1] x [y0,y1],
 *     u = 0 on the boundary,  u(0) = u0,  u_t(0) = u1,
 *
 * the regularised Cauchy problem of arXiv 2005.11931 (Section 2, equation (2.1), with the
 * vector-valued coefficient h = (h1, h2)), on the node grid and with the zero Dirichlet
 * data of the 2D experiment (Section 3.3).
 *
 * TEST INFRASTRUCTURE ONLY: this file is the slow, obviously correct definition that the
 * GPU library is checked against.  It shares no code with that library and nothing in the
 * product path links it.
 *
 * The paper integrates in time with implicit schemes (Crank-Nicolson in 1D, Section 3.1;
 * an implicit scheme with cyclic reduction in 2D, Section 3.3).  What is computed here is
 * the explicit second-order leapfrog scheme; the pieces the paper does not print are the
 * textbook ones, written out plainly:
 *   - face coefficients: arithmetic means of nodal values;
 *   - operator: flux form, (A v)_ij = [hx_{i+1/2}(v_{i+1}-v_i) + hx_{i-1/2}(v_{i-1}-v_i)]/dx^2
 *                                    + [hy_{j+1/2}(v_{j+1}-v_j) + hy_{j-1/2}(v_{j-1}-v_j)]/dy^2;
 *   - start: second-order Taylor step u^1 = u^0 + tau u1 + tau^2/2 A u^0;
 *   - steps: u^{n+1} = 2u^n - u^{n-1} + tau^2 A u^n;
 *   - energy: the discrete counterpart of the conserved quantity of Section 2 (proof of
 *     Theorem 2.1, the identity labelled CL-01): |u_t|^2 + sum_j |h_j^{1/2} d_j u|^2,
 *     E^{n+1/2} = dx dy [ sum ((u^{n+1}-u^n)/tau)^2 + sum_faces h (D u^{n+1})(D u^n)/d^2 ];
 *   - adjoint: the transposed recurrence of the scheme above (reverse leapfrog) for the
 *     gradient of a receiver loss with respect to the nodal coefficients.
 * Each pair of opposite-face terms is summed as a commutative pair, and the file is built
 * without floating-point contraction, so that a mirror-symmetric problem gives a bitwise
 * mirror-symmetric solution.
 */
#include "fdw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(a, j, i) ((a)[(size_t)(j) * (size_t)nx + (size_t)(i)])

int fdwref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Section 2 (eq. 2.1): the coefficient enters as h_j in d_j(h_j d_j u); on the grid it is
 * needed on the faces between nodes, taken as the mean of the two nodal values. */
void fdwref_faces(int nx, int ny, const double* h1, const double* h2, double* hx, double* hy)
{
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            AT(hx, j, i) = (i < nx - 1) ? 0.5 * (AT(h1, j, i) + AT(h1, j, i + 1)) : 0.0;
            AT(hy, j, i) = (j < ny - 1) ? 0.5 * (AT(h2, j, i) + AT(h2, j + 1, i)) : 0.0;
        }
    }
}

/* Section 2 (eq. 2.1): sum_j d_j(h_j d_j v) in flux form; boundary ring fixed (Section 3.3). */
void fdwref_apply(int nx, int ny, double dx, double dy, const double* hx, const double* hy,
                  const double* v, double* out)
{
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
                AT(out, j, i) = 0.0;
                continue;
            }
            double c = AT(v, j, i);
            double east = AT(hx, j, i) * (AT(v, j, i + 1) - c);
            double west = AT(hx, j, i - 1) * (AT(v, j, i - 1) - c);
            double north = AT(hy, j, i) * (AT(v, j + 1, i) - c);
            double south = AT(hy, j - 1, i) * (AT(v, j - 1, i) - c);
            AT(out, j, i) = (east + west) / (dx * dx) + (north + south) / (dy * dy);
        }
    }
}

/* Cauchy data of eq. (2.1): u(0) = u0, u_t(0) = u1; second-order Taylor start.
 * scratch holds A u0 ([ny][nx]). */
static void start_into(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                       const double* u0, const double* u1, const double* f0, double* scratch, double* u_first)
{
    fdwref_apply(nx, ny, dx, dy, hx, hy, u0, scratch);
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
                AT(u_first, j, i) = 0.0;
                continue;
            }
            double acc = AT(scratch, j, i) + (f0 ? AT(f0, j, i) : 0.0);
            AT(u_first, j, i) = AT(u0, j, i) + tau * AT(u1, j, i) + 0.5 * (tau * tau) * acc;
        }
    }
}

/* Leapfrog: central second difference in time of eq. (2.1).  scratch holds A u_cur. */
static void step_into(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                      const double* u_prev, const double* u_cur, const double* f, double* scratch, double* u_next)
{
    fdwref_apply(nx, ny, dx, dy, hx, hy, u_cur, scratch);
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
                AT(u_next, j, i) = 0.0;
                continue;
            }
            double acc = AT(scratch, j, i) + (f ? AT(f, j, i) : 0.0);
            AT(u_next, j, i) = 2.0 * AT(u_cur, j, i) - AT(u_prev, j, i) + (tau * tau) * acc;
        }
    }
}

void fdwref_start(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                  const double* u0, const double* u1, const double* f0, double* u_first)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)nx * (size_t)ny);
    start_into(nx, ny, dx, dy, tau, hx, hy, u0, u1, f0, a, u_first);
    free(a);
}

void fdwref_step(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                 const double* u_prev, const double* u_cur, const double* f, double* u_next)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)nx * (size_t)ny);
    step_into(nx, ny, dx, dy, tau, hx, hy, u_prev, u_cur, f, a, u_next);
    free(a);
}

/* Section 2, proof of Theorem 2.1 (CL-01): d/dt ( |u_t|^2 + sum_j |h_j^{1/2} d_j u|^2 ) = 0.
 * Discrete form for the pair (u^n, u^{n+1}), summed row by row in a fixed order. */
double fdwref_energy(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                     const double* u_n, const double* u_np1)
{
    double* kin = (double*)calloc((size_t)ny, sizeof(double));
    double* px = (double*)calloc((size_t)ny, sizeof(double));
    double* py = (double*)calloc((size_t)ny, sizeof(double));
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        double k = 0.0, sx = 0.0, sy = 0.0;
        for (int i = 0; i < nx; ++i) {
            double v = (AT(u_np1, j, i) - AT(u_n, j, i)) / tau;
            k += v * v;
            if (i < nx - 1)
                sx += AT(hx, j, i) * (AT(u_np1, j, i + 1) - AT(u_np1, j, i)) * (AT(u_n, j, i + 1) - AT(u_n, j, i));
            if (j < ny - 1)
                sy += AT(hy, j, i) * (AT(u_np1, j + 1, i) - AT(u_np1, j, i)) * (AT(u_n, j + 1, i) - AT(u_n, j, i));
        }
        kin[j] = k;
        px[j] = sx;
        py[j] = sy;
    }
    double K = 0.0, X = 0.0, Y = 0.0;
    for (j = 0; j < ny; ++j) {
        K += kin[j];
        X += px[j];
        Y += py[j];
    }
    free(kin);
    free(px);
    free(py);
    return dx * dy * (K + X / (dx * dx) + Y / (dy * dy));
}

static int check_receivers(int nx, int ny, int nrecv, const int* recv)
{
    if (nrecv < 0 || (nrecv > 0 && !recv)) return -1;
    for (int r = 0; r < nrecv; ++r) {
        int i = recv[2 * r], j = recv[2 * r + 1];
        if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2) return -1;
    }
    return 0;
}

static void zero_ring_copy(int nx, int ny, const double* src, double* dst)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            AT(dst, j, i) = (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) ? 0.0 : AT(src, j, i);
}

static void record(int nx, int nrecv, const int* recv, const double* u, double* row)
{
    for (int r = 0; r < nrecv; ++r) row[r] = AT(u, recv[2 * r + 1], recv[2 * r]);
}

int fdwref_forward(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                   const double* u0, const double* u1, long nsteps, double* energy, int nrecv,
                   const int* recv, double* traces, double* u_prev_out, double* u_cur_out)
{
    if (nx < 3 || ny < 3 || !(tau > 0.0) || nsteps < 0 || !h1 || !h2 || !u0 || !u1) return -1;
    if (check_receivers(nx, ny, nrecv, recv)) return -1;
    size_t n = (size_t)nx * (size_t)ny;
    double* hx = (double*)malloc(sizeof(double) * n);
    double* hy = (double*)malloc(sizeof(double) * n);
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    double* c = (double*)malloc(sizeof(double) * n);
    double* v1 = (double*)malloc(sizeof(double) * n);
    double* scr = (double*)malloc(sizeof(double) * n);
    if (!hx || !hy || !a || !b || !c || !v1 || !scr) {
        free(hx); free(hy); free(a); free(b); free(c); free(v1); free(scr);
        return -2;
    }
    fdwref_faces(nx, ny, h1, h2, hx, hy);
    zero_ring_copy(nx, ny, u0, a); /* u^0 */
    zero_ring_copy(nx, ny, u1, v1);
    if (traces) record(nx, nrecv, recv, a, traces);
    double *prev = a, *cur = a, *next = b;
    if (nsteps >= 1) {
        start_into(nx, ny, dx, dy, tau, hx, hy, a, v1, NULL, scr, b);
        if (energy) energy[0] = fdwref_energy(nx, ny, dx, dy, tau, hx, hy, a, b);
        if (traces) record(nx, nrecv, recv, b, traces + (size_t)nrecv);
        prev = a;
        cur = b;
        next = c;
        for (long s = 1; s < nsteps; ++s) {
            step_into(nx, ny, dx, dy, tau, hx, hy, prev, cur, NULL, scr, next);
            if (energy) energy[s] = fdwref_energy(nx, ny, dx, dy, tau, hx, hy, cur, next);
            if (traces) record(nx, nrecv, recv, next, traces + (size_t)(s + 1) * (size_t)nrecv);
            double* t = prev;
            prev = cur;
            cur = next;
            next = t;
        }
    }
    if (u_prev_out) memcpy(u_prev_out, prev, sizeof(double) * n);
    if (u_cur_out) memcpy(u_cur_out, cur, sizeof(double) * n);
    free(hx); free(hy); free(a); free(b); free(c); free(v1); free(scr);
    return 0;
}

double fdwref_misfit(long nrows, int nrecv, const double* traces, const double* d)
{
    double J = 0.0;
    for (long k = 0; k < nrows * (long)nrecv; ++k) {
        double e = traces[k] - d[k];
        J += e * e;
    }
    return J;
}

/* Gradient contribution of one term w * lam . (A(h) u) with respect to the face
 * coefficients: d/d hx_{i+1/2} of lam.(A u) = (lam_i - lam_{i+1})(u_{i+1} - u_i)/dx^2
 * (the face enters the rows of nodes i and i+1 with opposite signs; lam = 0 on the
 * boundary), likewise in y. */
static void accumulate_face_grad(int nx, int ny, double dx, double dy, double w, const double* u,
                                 const double* lam, double* gx, double* gy)
{
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            if (i < nx - 1)
                AT(gx, j, i) += w * (AT(lam, j, i) - AT(lam, j, i + 1)) * (AT(u, j, i + 1) - AT(u, j, i)) / (dx * dx);
            if (j < ny - 1)
                AT(gy, j, i) += w * (AT(lam, j, i) - AT(lam, j + 1, i)) * (AT(u, j + 1, i) - AT(u, j, i)) / (dy * dy);
        }
    }
}

int fdwref_adjoint(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                   const double* u0, const double* u1, long nsteps, int nrecv, const int* recv,
                   const double* trace_grad, long ckpt_every, double* grad_h1, double* grad_h2)
{
    if (nx < 3 || ny < 3 || !(tau > 0.0) || nsteps < 0 || ckpt_every < 0 || !h1 || !h2 || !u0 || !u1 ||
        !grad_h1 || (nrecv > 0 && !trace_grad))
        return -1;
    if (check_receivers(nx, ny, nrecv, recv)) return -1;
    const size_t n = (size_t)nx * (size_t)ny;
    const long N = nsteps;
    const double tt = tau * tau;
    int rc = 0;

    double* hx = (double*)calloc(n, sizeof(double));
    double* hy = (double*)calloc(n, sizeof(double));
    double* gx = (double*)calloc(n, sizeof(double));
    double* gy = (double*)calloc(n, sizeof(double));
    double* w0 = (double*)calloc(n, sizeof(double)); /* u^0 */
    double* v1 = (double*)calloc(n, sizeof(double)); /* u1 */
    double* lam_a = (double*)calloc(n, sizeof(double));
    double* lam_b = (double*)calloc(n, sizeof(double));
    double* lam_c = (double*)calloc(n, sizeof(double));
    double* tmp = (double*)calloc(n, sizeof(double));
    double* scr = (double*)calloc(n, sizeof(double));
    /* Store of forward levels: store-all keeps u^0..u^{N-1}; checkpointed keeps the pairs
     * (u^{s-1}, u^s) for s = c, 2c, ... and a segment buffer of c levels. */
    const long seg = (ckpt_every == 0) ? (N > 0 ? N : 1) : ckpt_every;
    const long nseg = (N + seg - 1) / seg;
    double* levels = (double*)malloc(sizeof(double) * n * (size_t)(seg + 1));
    double* ckpt = NULL;
    if (ckpt_every > 0 && nseg > 1) ckpt = (double*)malloc(sizeof(double) * n * 2 * (size_t)(nseg - 1));
    if (!hx || !hy || !gx || !gy || !w0 || !v1 || !lam_a || !lam_b || !lam_c || !tmp || !scr || !levels ||
        (ckpt_every > 0 && nseg > 1 && !ckpt)) {
        rc = -2;
        goto done;
    }
    fdwref_faces(nx, ny, h1, h2, hx, hy);
    zero_ring_copy(nx, ny, u0, w0);
    zero_ring_copy(nx, ny, u1, v1);

    if (N == 0) goto to_nodes;

    /* Forward sweep storing checkpoints (checkpointed mode only). */
    if (ckpt) {
        double *p = tmp, *q = lam_a, *r = lam_b; /* lam buffers are free during the forward sweep */
        memcpy(p, w0, sizeof(double) * n);
        start_into(nx, ny, dx, dy, tau, hx, hy, w0, v1, NULL, scr, q);
        for (long s = 1; s < N; ++s) {
            if (s % seg == 0) {
                long m = s / seg - 1;
                memcpy(ckpt + (size_t)(2 * m) * n, p, sizeof(double) * n);
                memcpy(ckpt + (size_t)(2 * m + 1) * n, q, sizeof(double) * n);
            }
            step_into(nx, ny, dx, dy, tau, hx, hy, p, q, NULL, scr, r);
            double* t = p;
            p = q;
            q = r;
            r = t;
        }
        memset(lam_a, 0, sizeof(double) * n);
        memset(lam_b, 0, sizeof(double) * n);
    }

    /* Reverse sweep.  lam_next = lam^{n+1}, lam_next2 = lam^{n+2}. */
    {
        double* lam_next = lam_a;
        double* lam_next2 = lam_b;
        double* lam_new = lam_c;
        memset(lam_next2, 0, sizeof(double) * n);
        memset(lam_next, 0, sizeof(double) * n);
        for (int rr = 0; rr < nrecv; ++rr)
            AT(lam_next, recv[2 * rr + 1], recv[2 * rr]) += trace_grad[(size_t)N * (size_t)nrecv + (size_t)rr];

        for (long m = nseg - 1; m >= 0; --m) {
            const long lo = m * seg;
            const long hi = (lo + seg < N) ? lo + seg : N; /* levels lo .. hi-1 are needed */
            /* Recompute u^lo .. u^{hi-1} into levels[0 .. hi-lo-1]. */
            double* L0 = levels;
            if (lo == 0) {
                memcpy(L0, w0, sizeof(double) * n);
                if (hi - lo > 1) start_into(nx, ny, dx, dy, tau, hx, hy, w0, v1, NULL, scr, levels + n);
                for (long s = 2; s < hi - lo; ++s)
                    step_into(nx, ny, dx, dy, tau, hx, hy, levels + (size_t)(s - 2) * n, levels + (size_t)(s - 1) * n,
                              NULL, scr, levels + (size_t)s * n);
            } else {
                /* levels[0] = u^{lo}, computed from the checkpoint pair (u^{lo-1}, u^{lo}). */
                const double* cp = ckpt + (size_t)(2 * (lo / seg - 1)) * n;
                memcpy(tmp, cp, sizeof(double) * n);
                memcpy(L0, cp + n, sizeof(double) * n);
                if (hi - lo > 1) step_into(nx, ny, dx, dy, tau, hx, hy, tmp, L0, NULL, scr, levels + n);
                for (long s = 2; s < hi - lo; ++s)
                    step_into(nx, ny, dx, dy, tau, hx, hy, levels + (size_t)(s - 2) * n, levels + (size_t)(s - 1) * n,
                              NULL, scr, levels + (size_t)s * n);
            }
            for (long k = hi - 1; k >= lo; --k) {
                const double* uk = levels + (size_t)(k - lo) * n;
                /* u^{k+1} = ... + c_k A(h) u^k with c_k = tau^2 (k >= 1) or tau^2/2 (k = 0) */
                accumulate_face_grad(nx, ny, dx, dy, (k == 0) ? 0.5 * tt : tt, uk, lam_next, gx, gy);
                if (k >= 1) {
                    /* lam^k = 2 lam^{k+1} - lam^{k+2} + tau^2 A lam^{k+1} + s_k (lam^{N+1} = 0). */
                    fdwref_apply(nx, ny, dx, dy, hx, hy, lam_next, tmp);
                    int j;
#pragma omp parallel for schedule(static)
                    for (j = 0; j < ny; ++j)
                        for (int i = 0; i < nx; ++i) {
                            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
                                AT(lam_new, j, i) = 0.0;
                                continue;
                            }
                            AT(lam_new, j, i) = 2.0 * AT(lam_next, j, i) - AT(lam_next2, j, i) + tt * AT(tmp, j, i);
                        }
                    for (int rr = 0; rr < nrecv; ++rr)
                        AT(lam_new, recv[2 * rr + 1], recv[2 * rr]) += trace_grad[(size_t)k * (size_t)nrecv + (size_t)rr];
                    double* t = lam_next2;
                    lam_next2 = lam_next;
                    lam_next = lam_new;
                    lam_new = t;
                }
            }
        }
    }

to_nodes:
    /* hx_{i+1/2} = (h1_i + h1_{i+1})/2, so dL/dh1_i = (g_{i-1/2} + g_{i+1/2})/2; likewise in y. */
    {
        int j;
#pragma omp parallel for schedule(static)
        for (j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double g1 = 0.5 * (((i > 0) ? AT(gx, j, i - 1) : 0.0) + ((i < nx - 1) ? AT(gx, j, i) : 0.0));
                double g2 = 0.5 * (((j > 0) ? AT(gy, j - 1, i) : 0.0) + ((j < ny - 1) ? AT(gy, j, i) : 0.0));
                if (grad_h2) {
                    AT(grad_h1, j, i) = g1;
                    AT(grad_h2, j, i) = g2;
                } else {
                    AT(grad_h1, j, i) = g1 + g2;
                }
            }
    }

done:
    free(hx); free(hy); free(gx); free(gy); free(w0); free(v1);
    free(lam_a); free(lam_b); free(lam_c); free(tmp); free(scr); free(levels); free(ckpt);
    return rc;
}

/* ------------------------------------------------------------------------------------------
 * The same forward definition (faces, flux-form operator, Taylor start, three-level leapfrog)
 * evaluated in x87 extended precision (long double, 64-bit significand).  With very small
 * time steps the three-level form loses accuracy to its own rounding: the rounding of every
 * u^{n+1} acts on the following steps like a kick to the velocity (u^{n+1} - u^n)/tau, so
 * those errors add up faster than linearly in n.  This evaluation is the reference that both
 * FP64 computations (this oracle's and the GPU's) are measured against in that regime; its
 * own rounding is 2^11 times finer than FP64's.
 * ------------------------------------------------------------------------------------------ */
typedef long double ld_t;

static void ld_apply(int nx, int ny, ld_t dx2, ld_t dy2, const ld_t* hx, const ld_t* hy, const ld_t* v, ld_t* out)
{
    int j, i;
#pragma omp parallel for collapse(2) schedule(static)
    for (j = 0; j < ny; ++j) {
        for (i = 0; i < nx; ++i) {
            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) {
                AT(out, j, i) = 0.0L;
                continue;
            }
            ld_t c = AT(v, j, i);
            ld_t east = AT(hx, j, i) * (AT(v, j, i + 1) - c);
            ld_t west = AT(hx, j, i - 1) * (AT(v, j, i - 1) - c);
            ld_t north = AT(hy, j, i) * (AT(v, j + 1, i) - c);
            ld_t south = AT(hy, j - 1, i) * (AT(v, j - 1, i) - c);
            AT(out, j, i) = (east + west) / dx2 + (north + south) / dy2;
        }
    }
}

int fdwref_forward_ld(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                      const double* u0, const double* u1, long nsteps, int nrecv, const int* recv, double* traces,
                      int nmarks, const long* marks, double* mark_out, double* u_prev_out, double* u_cur_out)
{
    if (nx < 3 || ny < 3 || !(tau > 0.0) || nsteps < 0 || !h1 || !h2 || !u0 || !u1) return -1;
    if (check_receivers(nx, ny, nrecv, recv)) return -1;
    if (nmarks < 0 || (nmarks > 0 && (!marks || !mark_out))) return -1;
    const size_t n = (size_t)nx * (size_t)ny;
    ld_t* hx = (ld_t*)malloc(sizeof(ld_t) * n);
    ld_t* hy = (ld_t*)malloc(sizeof(ld_t) * n);
    ld_t* a = (ld_t*)malloc(sizeof(ld_t) * n);
    ld_t* b = (ld_t*)malloc(sizeof(ld_t) * n);
    ld_t* c = (ld_t*)malloc(sizeof(ld_t) * n);
    ld_t* scr = (ld_t*)malloc(sizeof(ld_t) * n);
    if (!hx || !hy || !a || !b || !c || !scr) {
        free(hx); free(hy); free(a); free(b); free(c); free(scr);
        return -2;
    }
    const ld_t T = (ld_t)tau, tt = T * T, dx2 = (ld_t)dx * (ld_t)dx, dy2 = (ld_t)dy * (ld_t)dy;
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            const int ring = (i == 0 || j == 0 || i == nx - 1 || j == ny - 1);
            AT(hx, j, i) = (i < nx - 1) ? 0.5L * ((ld_t)AT(h1, j, i) + (ld_t)AT(h1, j, i + 1)) : 0.0L;
            AT(hy, j, i) = (j < ny - 1) ? 0.5L * ((ld_t)AT(h2, j, i) + (ld_t)AT(h2, j + 1, i)) : 0.0L;
            AT(a, j, i) = ring ? 0.0L : (ld_t)AT(u0, j, i);
        }
    }
    if (traces)
        for (int r = 0; r < nrecv; ++r) traces[r] = (double)AT(a, recv[2 * r + 1], recv[2 * r]);
    /* u^s into every snapshot slot that asks for step s */
#define LD_MARK(s_, u_)                                                                              \
    for (int q = 0; q < nmarks; ++q)                                                                 \
        if (marks[q] == (s_))                                                                        \
            for (size_t k = 0; k < n; ++k) mark_out[(size_t)q * n + k] = (double)(u_)[k];
    LD_MARK(0, a)
    ld_t *prev = a, *cur = a, *next = b;
    int i;
    if (nsteps >= 1) {
        ld_apply(nx, ny, dx2, dy2, hx, hy, a, scr);
#pragma omp parallel for collapse(2) schedule(static)
        for (j = 0; j < ny; ++j)
            for (i = 0; i < nx; ++i) {
                const int ring = (i == 0 || j == 0 || i == nx - 1 || j == ny - 1);
                AT(b, j, i) = ring ? 0.0L : AT(a, j, i) + T * (ld_t)AT(u1, j, i) + 0.5L * tt * AT(scr, j, i);
            }
        prev = a;
        cur = b;
        next = c;
        if (traces)
            for (int r = 0; r < nrecv; ++r) traces[nrecv + r] = (double)AT(cur, recv[2 * r + 1], recv[2 * r]);
        LD_MARK(1, cur)
        for (long s = 1; s < nsteps; ++s) {
            ld_apply(nx, ny, dx2, dy2, hx, hy, cur, scr);
#pragma omp parallel for collapse(2) schedule(static)
            for (j = 0; j < ny; ++j)
                for (i = 0; i < nx; ++i) {
                    const int ring = (i == 0 || j == 0 || i == nx - 1 || j == ny - 1);
                    AT(next, j, i) = ring ? 0.0L : 2.0L * AT(cur, j, i) - AT(prev, j, i) + tt * AT(scr, j, i);
                }
            if (traces)
                for (int r = 0; r < nrecv; ++r)
                    traces[(size_t)(s + 1) * (size_t)nrecv + r] = (double)AT(next, recv[2 * r + 1], recv[2 * r]);
            LD_MARK(s + 1, next)
            ld_t* t = prev;
            prev = cur;
            cur = next;
            next = t;
        }
    }
    for (size_t k = 0; k < n; ++k) {
        if (u_prev_out) u_prev_out[k] = (double)prev[k];
        if (u_cur_out) u_cur_out[k] = (double)cur[k];
    }
    free(hx); free(hy); free(a); free(b); free(c); free(scr);
    return 0;
#undef LD_MARK
}

/* ------------------------------------------------------------------------------------------
 * The implicit scheme of the 2D experiment (Section 3.3: an implicit finite-difference scheme
 * whose linear systems are solved by cyclic reduction; Section 4, Table 1 times it on a GPU).
 * The paper names the scheme only by reference; what is computed here is the factorized
 * (alternating-direction) implicit scheme for u_tt = L1 u + L2 u, L1 = d_x(h1 d_x .),
 * L2 = d_y(h2 d_y .):
 *     (I - sigma tau^2 L1)(I - sigma tau^2 L2) (u^{n+1} - 2u^n + u^{n-1}) = tau^2 (L1 + L2) u^n,
 * with the start  u^1 = u^0 + tau u1 + (1/2) w^0,  (I - sigma tau^2 L1)(I - sigma tau^2 L2) w^0 =
 * tau^2 (L1 + L2) u^0 (sigma = 0 is the leapfrog scheme above; sigma >= 1/4 is unconditionally
 * stable for constant coefficients).  Each factor is a set of independent tridiagonal systems,
 * one per grid line, solved here by plain Gaussian elimination (the Thomas algorithm).
 * ------------------------------------------------------------------------------------------ */

/* Solve the tridiagonal system  lo[k] x[k-1] + di[k] x[k] + up[k] x[k+1] = rhs[k], k = 0..n-1
 * (lo[0] and up[n-1] unused) by forward elimination and back substitution; x may alias rhs.
 * scratch: 2n doubles. */
static void thomas(int n, const double* lo, const double* di, const double* up, const double* rhs, double* x,
                   double* scratch)
{
    double* cp = scratch;
    double* dp = scratch + n;
    cp[0] = (n > 1) ? up[0] / di[0] : 0.0;
    dp[0] = rhs[0] / di[0];
    for (int k = 1; k < n; ++k) {
        const double m = di[k] - lo[k] * cp[k - 1];
        cp[k] = (k < n - 1) ? up[k] / m : 0.0;
        dp[k] = (rhs[k] - lo[k] * dp[k - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int k = n - 2; k >= 0; --k) x[k] = dp[k] - cp[k] * x[k + 1];
}

/* w = [(I - sigma tau^2 L1)(I - sigma tau^2 L2)]^{-1} r on interior nodes (0 on the ring):
 * first the x lines (I - sigma tau^2 L1) z = r, then the y lines (I - sigma tau^2 L2) w = z. */
static void adi_solve(int nx, int ny, double dx, double dy, double sigma, double tau, const double* hx,
                      const double* hy, const double* r, double* w)
{
    const double gx = sigma * tau * tau / (dx * dx), gy = sigma * tau * tau / (dy * dy);
    const int mx = nx - 2, my = ny - 2;
    double* z = (double*)calloc((size_t)nx * (size_t)ny, sizeof(double));
    int j;
#pragma omp parallel for schedule(static)
    for (j = 1; j <= ny - 2; ++j) {
        double* lo = (double*)malloc(sizeof(double) * 6 * (size_t)mx);
        double *di = lo + mx, *up = di + mx, *rhs = up + mx, *scr = rhs + mx;
        for (int k = 0; k < mx; ++k) {
            const int i = k + 1;
            lo[k] = -gx * AT(hx, j, i - 1);
            up[k] = -gx * AT(hx, j, i);
            di[k] = 1.0 + gx * (AT(hx, j, i - 1) + AT(hx, j, i));
            rhs[k] = AT(r, j, i);
        }
        thomas(mx, lo, di, up, rhs, rhs, scr);
        for (int k = 0; k < mx; ++k) AT(z, j, k + 1) = rhs[k];
        free(lo);
    }
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nx; ++i) {
        if (i == 0 || i == nx - 1) {
            for (int jj = 0; jj < ny; ++jj) AT(w, jj, i) = 0.0;
            continue;
        }
        double* lo = (double*)malloc(sizeof(double) * 6 * (size_t)my);
        double *di = lo + my, *up = di + my, *rhs = up + my, *scr = rhs + my;
        for (int k = 0; k < my; ++k) {
            const int jj = k + 1;
            lo[k] = -gy * AT(hy, jj - 1, i);
            up[k] = -gy * AT(hy, jj, i);
            di[k] = 1.0 + gy * (AT(hy, jj - 1, i) + AT(hy, jj, i));
            rhs[k] = AT(z, jj, i);
        }
        thomas(my, lo, di, up, rhs, rhs, scr);
        AT(w, 0, i) = 0.0;
        AT(w, ny - 1, i) = 0.0;
        for (int k = 0; k < my; ++k) AT(w, k + 1, i) = rhs[k];
        free(lo);
    }
    free(z);
}

int fdwref_adi_forward(int nx, int ny, double dx, double dy, double tau, double sigma, const double* h1,
                       const double* h2, const double* u0, const double* u1, long nsteps, double* u_prev_out,
                       double* u_cur_out)
{
    if (nx < 3 || ny < 3 || !(tau > 0.0) || !(sigma >= 0.0) || nsteps < 0 || !h1 || !h2 || !u0 || !u1) return -1;
    const size_t n = (size_t)nx * (size_t)ny;
    double* hx = (double*)malloc(sizeof(double) * n);
    double* hy = (double*)malloc(sizeof(double) * n);
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    double* c = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* w = (double*)malloc(sizeof(double) * n);
    if (!hx || !hy || !a || !b || !c || !r || !w) {
        free(hx); free(hy); free(a); free(b); free(c); free(r); free(w);
        return -2;
    }
    fdwref_faces(nx, ny, h1, h2, hx, hy);
    zero_ring_copy(nx, ny, u0, a);
    double *prev = a, *cur = a, *next = b;
    if (nsteps >= 1) {
        /* start: u^1 = u^0 + tau u1 + w^0 / 2 */
        fdwref_apply(nx, ny, dx, dy, hx, hy, a, r);
        for (size_t k = 0; k < n; ++k) r[k] *= tau * tau;
        adi_solve(nx, ny, dx, dy, sigma, tau, hx, hy, r, w);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int ring = (i == 0 || j == 0 || i == nx - 1 || j == ny - 1);
                AT(b, j, i) = ring ? 0.0 : AT(a, j, i) + tau * AT(u1, j, i) + 0.5 * AT(w, j, i);
            }
        prev = a;
        cur = b;
        next = c;
        for (long s = 1; s < nsteps; ++s) {
            fdwref_apply(nx, ny, dx, dy, hx, hy, cur, r);
            for (size_t k = 0; k < n; ++k) r[k] *= tau * tau;
            adi_solve(nx, ny, dx, dy, sigma, tau, hx, hy, r, w);
            for (size_t k = 0; k < n; ++k) next[k] = 2.0 * cur[k] - prev[k] + w[k];
            double* t = prev;
            prev = cur;
            cur = next;
            next = t;
        }
    }
    if (u_prev_out) memcpy(u_prev_out, prev, sizeof(double) * n);
    if (u_cur_out) memcpy(u_cur_out, cur, sizeof(double) * n);
    free(hx); free(hy); free(a); free(b); free(c); free(r); free(w);
    return 0;
}

/* The tridiagonal solver alone (for its own pins): x = T^{-1} rhs. */
void fdwref_tridiag(int n, const double* lo, const double* di, const double* up, const double* rhs, double* x)
{
    double* scr = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    thomas(n, lo, di, up, rhs, x, scr);
    free(scr);
}
