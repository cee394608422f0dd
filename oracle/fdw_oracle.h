/*
 * fdw_oracle.h - plain FP64 CPU oracle for the explicit leapfrog discretisation of the
 * regularised tsunami wave equation (arXiv 2005.11931).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call this
 * code: only the test suite, the smoke check and the CPU-baseline leg of the benchmark use
 * it, to produce the values the GPU library is checked against.
 *
 * Conventions shared by every function:
 *   - grids are nx x ny nodes including the boundary ring; arrays are row-major [ny][nx]
 *     (x fastest), FP64, dense (row pitch nx);
 *   - dx = (x1 - x0)/(nx - 1), dy = (y1 - y0)/(ny - 1) are passed in;
 *   - zero Dirichlet data: the boundary ring of every state is 0 (Section 3.3);
 *   - receivers are int [R][2] pairs (i, j) = (column, row) of interior nodes.
 */
#ifndef FDW_ORACLE_H
#define FDW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Face coefficients: hx[j][i] = (h1[j][i] + h1[j][i+1])/2 for i < nx-1 (0 otherwise),
 * hy[j][i] = (h2[j][i] + h2[j+1][i])/2 for j < ny-1 (0 otherwise). */
void fdwref_faces(int nx, int ny, const double* h1, const double* h2, double* hx, double* hy);

/* out = A v: the flux-form difference operator d_x(h1 d_x v) + d_y(h2 d_y v) on interior
 * nodes, 0 on the boundary ring. */
void fdwref_apply(int nx, int ny, double dx, double dy, const double* hx, const double* hy,
                  const double* v, double* out);

/* Start step: u_first = u0 + tau u1 + (tau^2/2)(A u0 + f0) on interior nodes (f0 may be NULL). */
void fdwref_start(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                  const double* u0, const double* u1, const double* f0, double* u_first);

/* One leapfrog step: u_next = 2 u_cur - u_prev + tau^2 (A u_cur + f) on interior nodes. */
void fdwref_step(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                 const double* u_prev, const double* u_cur, const double* f, double* u_next);

/* Discrete energy E^{n+1/2} of the pair (u_n, u_np1), face-sum form. */
double fdwref_energy(int nx, int ny, double dx, double dy, double tau, const double* hx, const double* hy,
                     const double* u_n, const double* u_np1);

/* Forward solve of nsteps steps from (u0, u1).  energy (NULL or [nsteps]) receives
 * E^{n+1/2}, n = 0..nsteps-1; traces (NULL or [nsteps+1][nrecv]) receives u^n at the
 * receivers, n = 0..nsteps; u_prev_out/u_cur_out (NULL allowed) receive u^{N-1}, u^N
 * (for nsteps = 0: u0, u0).  h2 may equal h1.  Returns 0, or -1 on bad arguments. */
int fdwref_forward(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                   const double* u0, const double* u1, long nsteps, double* energy, int nrecv,
                   const int* recv, double* traces, double* u_prev_out, double* u_cur_out);

/* The forward definition of fdwref_forward (faces, operator, start, three-level steps)
 * evaluated in x87 extended precision (long double, 64-bit significand); inputs are FP64,
 * outputs are rounded to FP64.  The reference at very small time steps, where the FP64
 * three-level recurrence accumulates its own rounding faster than linearly in n.
 * traces (NULL or [nsteps+1][nrecv]), u_prev_out and u_cur_out as in fdwref_forward;
 * mark_out ([nmarks][ny][nx], may be NULL when nmarks = 0) receives u^{marks[q]}. */
int fdwref_forward_ld(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                      const double* u0, const double* u1, long nsteps, int nrecv, const int* recv, double* traces,
                      int nmarks, const long* marks, double* mark_out, double* u_prev_out, double* u_cur_out);

/* Misfit J = sum_{n,r} (traces - d)^2 over [nrows][nrecv]. */
double fdwref_misfit(long nrows, int nrecv, const double* traces, const double* d);

/* Gradient of a trace loss L with respect to the nodal coefficients.  trace_grad is
 * [nsteps+1][nrecv] = dL/du^n at the receivers.  ckpt_every = 0 stores every level;
 * ckpt_every = c > 0 stores the pair (u^{s-1}, u^s) every c steps and recomputes each
 * segment forward.  grad_h1 receives dL/dh1; grad_h2 receives dL/dh2, or, when NULL,
 * dL/dh2 is added into grad_h1 (the case h1 = h2 = h).  Returns 0, -1 on bad arguments,
 * -2 when memory runs out. */
int fdwref_adjoint(int nx, int ny, double dx, double dy, double tau, const double* h1, const double* h2,
                   const double* u0, const double* u1, long nsteps, int nrecv, const int* recv,
                   const double* trace_grad, long ckpt_every, double* grad_h1, double* grad_h2);

/* The implicit factorized (alternating-direction) scheme of the 2D experiment (Section 3.3;
 * Section 4, Table 1): (I - sigma tau^2 L1)(I - sigma tau^2 L2)(u^{n+1} - 2u^n + u^{n-1}) =
 * tau^2 (L1 + L2) u^n with L1, L2 the x and y parts of the operator of fdwref_apply; start
 * u^1 = u^0 + tau u1 + w^0/2 with w^0 the same solve applied to tau^2 A u^0.  Line systems solved
 * by the Thomas algorithm.  u_prev_out/u_cur_out as in fdwref_forward.  Returns 0, -1 on bad
 * arguments, -2 when memory runs out. */
int fdwref_adi_forward(int nx, int ny, double dx, double dy, double tau, double sigma, const double* h1,
                       const double* h2, const double* u0, const double* u1, long nsteps, double* u_prev_out,
                       double* u_cur_out);

/* x = T^{-1} rhs for the tridiagonal T with sub-diagonal lo[1..n-1], diagonal di, super-diagonal
 * up[0..n-2] (the line solver of fdwref_adi_forward). */
void fdwref_tridiag(int n, const double* lo, const double* di, const double* up, const double* rhs, double* x);

/* Number of OpenMP threads the oracle runs on. */
int fdwref_threads(void);

#ifdef __cplusplus
}
#endif
#endif
