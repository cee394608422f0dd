// fdw_adjoint.hip - reverse (adjoint) leapfrog sweep for the gradient of a receiver loss with
// respect to the depth coefficient of u_tt = d_x(h1 d_x u) + d_y(h2 d_y u) (arXiv 2005.11931,
// Section 2 eq. (2.1), zero Dirichlet data of Section 3.3).
//
// Forward recurrence (increment form, L = tau^2 A(h)):
//     du^{n+1} = du^n + L u^n,  u^{n+1} = u^n + du^{n+1}       (n >= 1)
//     u^1 = u^0 + tau u1 + L u^0 / 2                            (start)
// A(h) is symmetric, so the adjoint lam^n = dJ/du^n obeys the same stencil backwards:
//     lam^N = s_N,  lam^n = 2 lam^{n+1} - lam^{n+2} + L lam^{n+1} + s_n,
// carried here in increment form mu^n = lam^n - lam^{n+1}:
//     mu^n = mu^{n+1} + L lam^{n+1} + s_n,   lam^n = lam^{n+1} + mu^n,
// and the gradient collects, for every n, w_n d/dh [lam^{n+1} . L(h) u^n] with w_n = 1
// (w_0 = 1/2 for the start step).  With faces h_{i+1/2} = (h_i + h_{i+1})/2 this is node-local:
//     dJ/dh1_i += -w_n ax sum_{q = i +- 1} (u_q - u_i)(lam_q - lam_i),  ax = tau^2/(2 dx^2)
// (and likewise in y for h2).
//
// The forward state needed in reverse order is rebuilt by time reversal of the same
// recurrence, u^n = u^{n+1} - du^{n+1}, du^n = du^{n+1} - L u^n, re-anchored at exact
// checkpoints stored by the forward replay.  One launch advances K reverse levels with the
// streaming structure of the forward kernel (one wave per strip x segment, K-column halo,
// rows in registers, DPP lane exchange); the gradient of a node collects the K levels in
// registers and is added to the FP64 accumulator plane once per launch.
#include "fdw_internal.h"
#include "fdw_stream.h"

#include <hip/hip_runtime.h>

namespace fdw {

// One reverse work item (strip x segment, K levels, C columns per lane).  Level s (s = 1..K)
// turns the time-(m-s+1) quadruple (u, du, lam, mu) into the time-(m-s) one at row
// r = j - s.  u^{m-s} is produced one row ahead (pointwise from level s-1), so that the
// operator on u^{m-s} and on lam^{m-s+1} can be written in flux form like the forward kernel
// (x fluxes per face, y flux carried from the row above).  The gradient terms are products
// of the face differences, Px = (u_{c+1}-u_c)(lam_{c+1}-lam_c), each shared by the face's two
// nodes; a node collects its K levels in registers and its accumulator plane is updated once
// per launch.  SPLIT keeps the x and y parts (dJ/dh1, dJ/dh2) in separate planes; otherwise
// one plane holds their sum.
template <typename T, int K, int C, int FACE, int SPLIT>
__global__ __launch_bounds__(kWaveSize * kWavesPerBlock) void k_adjoint(AdjArgs a)
{
    constexpr int Hx = ((K + C - 1) / C) * C;
    constexpr int Wv = kWaveSize * C - 2 * Hx;
    // rows are loaded NB - 1 rows ahead: two rows for FP64 with one column per lane and K a
    // multiple of 3 (the default reverse configuration, which stays at two waves per SIMD),
    // one row elsewhere (a deeper prefetch would push the FP32 variants to one wave)
    constexpr int NB = (sizeof(T) == 8 && C == 1 && K % 3 == 0) ? 3 : 2;
    constexpr int U = (K % 2 == 0) ? K : 2 * K;
    static_assert(U % NB == 0 && U % K == 0 && U % 2 == 0, "row unroll");
    const int lane = threadIdx.x & 63;
    // XCD-contiguous block order, as in the forward kernel: neighbouring strips and segments
    // (which read each other's halo rows and columns) then share an L2
    const int wave = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave_in_block();
    if (wave >= a.waves) return;

    const int nx = a.nx, ny = a.ny, ld = a.ld;
    const int strip = wave % a.strips;
    const int seg = wave / a.strips;
    const int cb = strip * Wv - Hx + lane * C;
    const bool lane_live = (cb >= 0) && (cb < ld);
    const bool lane_owned = lane_live && (lane * C >= Hx) && (lane * C < Hx + Wv);
    T colm[C];
#pragma unroll
    for (int c = 0; c < C; ++c) colm[c] = ((cb + c >= 1) && (cb + c <= nx - 2)) ? T(1) : T(0);
    const int r0 = seg * a.seg_rows;
    const int r1 = min(r0 + a.seg_rows, ny);
    const T ax = (T)a.ax, ay = (T)a.ay;
    const double axd = a.ax, ayd = a.ay;
    constexpr bool split = SPLIT != 0;

    // even segments stream downwards, odd ones upwards, as in the forward kernel (the shared
    // halo rows of two neighbouring segments are then read at about the same time); position p
    // of the stream is row rfirst + dir * p, and the result is the same bit for bit
    const int dir = (seg & 1) ? -1 : 1;
    const int rfirst = (dir > 0) ? r0 - K : r1 + K - 1;
    const int jbase = max(r0 - K, 0);
    const size_t base_el = (size_t)jbase * ld;
    const size_t span = (size_t)(ny - jbase) * ld * sizeof(T);
    const unsigned int nbytes = (unsigned int)min(span, (size_t)kBufferOutOfRange - 16);
    const __amdgpu_buffer_rsrc_t ru = plane_rsrc((const T*)a.uin + base_el, nbytes);
    const __amdgpu_buffer_rsrc_t rd = plane_rsrc((const T*)a.din + base_el, nbytes);
    const __amdgpu_buffer_rsrc_t rl = plane_rsrc((const T*)a.lin + base_el, nbytes);
    const __amdgpu_buffer_rsrc_t rm = plane_rsrc((const T*)a.min + base_el, nbytes);
    const __amdgpu_buffer_rsrc_t rh = plane_rsrc((const T*)a.h + base_el, nbytes);
    const __amdgpu_buffer_rsrc_t rhy = plane_rsrc((const T*)(FACE ? a.hy : a.h) + base_el, nbytes);
    const unsigned int row_bytes = (unsigned int)(ld * (int)sizeof(T));
    const unsigned int lane_col = lane_live ? (unsigned int)(cb * (int)sizeof(T)) : kBufferOutOfRange;
    // gradient accumulator planes (double), read through buffers as well
    const size_t gspan = (size_t)(ny - jbase) * ld * sizeof(double);
    const unsigned int gbytes = (unsigned int)min(gspan, (size_t)kBufferOutOfRange - 16);
    const __amdgpu_buffer_rsrc_t rg1 = plane_rsrc(a.g1 + base_el, gbytes);
    const __amdgpu_buffer_rsrc_t rg2 = plane_rsrc(a.g2 + base_el, gbytes);
    const unsigned int grow_bytes = (unsigned int)(ld * (int)sizeof(double));
    const unsigned int glane_col = lane_owned ? (unsigned int)(cb * (int)sizeof(double)) : kBufferOutOfRange;
    // receiver CSR (row pointers, columns, ids) and the trace gradient are not written during
    // the launch: read them as constant memory, so that their (wave-uniform) lookups are scalar
    // loads and do not wait behind the vector loads of the row prefetch
    const ConstPtr<int> rowptr = (ConstPtr<int>)a.rec_rowptr;
    const ConstPtr<int> rcol = (ConstPtr<int>)a.rec_col;
    const ConstPtr<int> rid = (ConstPtr<int>)a.rec_id;
    const ConstPtr<double> tgrad = (ConstPtr<double>)a.trace_grad;
    // items whose rows (halo included) hold no receiver skip the source code entirely
    const bool any_rec = a.R > 0 && rowptr[max(r0 - K, 0)] < rowptr[min(r1 + K, ny)];
    const int col_lo = strip * Wv - Hx;  // first column the strip computes
    T* __restrict__ uout = (T*)a.uout;
    T* __restrict__ dout = (T*)a.dout;
    T* __restrict__ lout = (T*)a.lout;
    T* __restrict__ mout = (T*)a.mout;

    T Ur[K + 1][2][C];  // u^{m-s}, rows by parity (level s >= 1 runs one row ahead)
    T Dr[K][2][C];      // du^{m-s}
    T Lr[K][2][C];      // lam^{m-s}
    T Mr[K][2][C];      // mu^{m-s}
    T Gu[K][C];         // y flux of u^{m-s} below row r (level s stores at s-1)
    T Gl[K][C];         // y flux of lam^{m-s+1} below row r
    double Py[K][C];    // y face products below row r
    double GX[K][C], GY[K][C];  // gradient of rows p-1 .. p-K (by position modulo K); GY only if SPLIT
    double gbuf[NB][C], g2buf[NB][C];  // accumulator rows, loaded NB - 1 iterations ahead
    T FXr[K][C], FYr[K][C];
    T hprev[C], hyprev[C];
    T bu[NB][C], bd[NB][C], bl[NB][C], bm[NB][C], bh[NB][C], bhy[NB][C];  // rows by row modulo NB
    // receiver range [RPb, RPe) of the rows p-1 .. p-K (by position modulo K), looked up once per
    // row when it enters level 1
    int RPb[K], RPe[K];
#pragma unroll
    for (int t = 0; t < K; ++t) RPb[t] = RPe[t] = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int t = 0; t <= K; ++t) Ur[t][0][c] = Ur[t][1][c] = T(0);
#pragma unroll
        for (int t = 0; t < K; ++t) {
            Dr[t][0][c] = Dr[t][1][c] = Lr[t][0][c] = Lr[t][1][c] = Mr[t][0][c] = Mr[t][1][c] = T(0);
            Gu[t][c] = Gl[t][c] = T(0);
            Py[t][c] = GX[t][c] = GY[t][c] = 0.0;
            FXr[t][c] = FYr[t][c] = T(0);
        }
        hprev[c] = hyprev[c] = T(0);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            bu[q][c] = bd[q][c] = bl[q][c] = bm[q][c] = bh[q][c] = bhy[q][c] = T(0);
            gbuf[q][c] = g2buf[q][c] = 0.0;
        }
    }
    auto load_row = [&](int p, T (&u)[C], T (&d)[C], T (&l)[C], T (&m)[C], T (&h)[C], T (&hy)[C]) {
        const int j = rfirst + dir * p;
        const unsigned int off = (j < jbase) ? kBufferOutOfRange : (unsigned int)(j - jbase) * row_bytes + lane_col;
        buffer_row<T, C>(ru, off, u);
        buffer_row<T, C>(rd, off, d);
        buffer_row<T, C>(rl, off, l);
        buffer_row<T, C>(rm, off, m);
        buffer_row<T, C>(rh, off, h);
        if (FACE) buffer_row<T, C>(rhy, off, hy);
    };
    // accumulator row of stream position p (the row completed NB - 1 iterations later)
    // only the segment's own rows are accumulated, so only those are read (an out-of-range
    // buffer offset costs no memory traffic)
    auto load_g = [&](int p, double (&g1)[C], double (&g2)[C]) {
        const int j = rfirst + dir * p;
        const unsigned int goff =
            (j < r0 || j >= r1) ? kBufferOutOfRange : (unsigned int)(j - jbase) * grow_bytes + glane_col;
        buffer_row<double, C>(rg1, goff, g1);
        if (split) buffer_row<double, C>(rg2, goff, g2);
    };
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) {
        load_row(q, bu[q], bd[q], bl[q], bm[q], bh[q], bhy[q]);
        load_g(q - K, gbuf[q], g2buf[q]);
    }
    const int nblk = (r1 - r0 + 2 * K + U - 1) / U;

    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int p = blk * U + s;  // stream position of the row loaded last
            const int pb = s % NB;
            {
                const int pn = (s + NB - 1) % NB;
                load_row(p + NB - 1, bu[pn], bd[pn], bl[pn], bm[pn], bh[pn], bhy[pn]);
                load_g(p + NB - 1 - K, gbuf[pn], g2buf[pn]);
            }
            // coefficient faces of row p-1, scaled by tau^2/(2 dx^2) and tau^2/(2 dy^2) as in
            // the forward kernel (the y face between rows p-1 and p is stored with the upper of
            // the two grid rows)
            {
                const int q = pmod(s - 1, K);
                if (FACE) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        FXr[q][c] = ax * hprev[c];
                        FYr[q][c] = ay * ((dir > 0) ? hyprev[c] : bhy[pb][c]);
                        hprev[c] = bh[pb][c];
                        hyprev[c] = bhy[pb][c];
                    }
                } else {
                    const T hr = lane_from_right(hprev[0]);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        FXr[q][c] = ax * (hprev[c] + ((c < C - 1) ? hprev[c + 1] : hr));
                        FYr[q][c] = ay * (hprev[c] + bh[pb][c]);
                    }
#pragma unroll
                    for (int c = 0; c < C; ++c) hprev[c] = bh[pb][c];
                }
            }
            // level 0 (time m): row p
            {
                const int p0 = pmod(s, 2);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Ur[0][p0][c] = bu[pb][c];
                    Dr[0][p0][c] = bd[pb][c];
                    Lr[0][p0][c] = bl[pb][c];
                    Mr[0][p0][c] = bm[pb][c];
                }
            }
#pragma unroll
            for (int t = 1; t <= K; ++t) {
                const int r = rfirst + dir * (p - t);  // grid row of stream position p - t
                const int pr = pmod(s - t, 2);
                const int pr1 = pmod(s - t + 1, 2);
                const int q = pmod(s - t, K);
                const bool rin = (r >= 1) && (r <= ny - 2);
                const bool rown = (r >= r0) && (r < r1);
                const int64_t n = a.n_top - t;  // time of this level's forward state
                const double w = (n == 0) ? 0.5 : 1.0;
                // u^{m-t}(r+1) = u^{m-t+1}(r+1) - du^{m-t+1}(r+1); u and du are zero on the
                // Dirichlet rows at every level (and rows outside the grid load as zero), so
                // this needs no row test
#pragma unroll
                for (int c = 0; c < C; ++c) Ur[t][pr1][c] = fma_t(-Dr[t - 1][pr1][c], colm[c], Ur[t - 1][pr1][c]);
                // x fluxes and face differences of u^{m-t} and lam^{m-t+1} at row r
                const T uR = lane_from_right(Ur[t][pr][0]);
                const T lR = lane_from_right(Lr[t - 1][pr][0]);
                T Fu[C], Fl[C];
                double Px[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const T du = ((c < C - 1) ? Ur[t][pr][c + 1] : uR) - Ur[t][pr][c];
                    const T dl = ((c < C - 1) ? Lr[t - 1][pr][c + 1] : lR) - Lr[t - 1][pr][c];
                    Fu[c] = FXr[q][c] * du;
                    Fl[c] = FXr[q][c] * dl;
                    Px[c] = (double)du * (double)dl;
                }
                const T FuL = lane_from_left(Fu[C - 1]);
                const T FlL = lane_from_left(Fl[C - 1]);
                const double PxL = lane_from_left(Px[C - 1]);
                T nd[C], nm[C], nl[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const T duy = Ur[t][pr1][c] - Ur[t][pr][c];
                    const T dly = Lr[t - 1][pr1][c] - Lr[t - 1][pr][c];
                    const T Gun = FYr[q][c] * duy;
                    const T Gln = FYr[q][c] * dly;
                    const double Pyn = (double)duy * (double)dly;
                    const T Lu = (Fu[c] - ((c > 0) ? Fu[c - 1] : FuL)) + (Gun - Gu[t - 1][c]);
                    const T Ll = (Fl[c] - ((c > 0) ? Fl[c - 1] : FlL)) + (Gln - Gl[t - 1][c]);
                    Gu[t - 1][c] = Gun;
                    Gl[t - 1][c] = Gln;
                    const double gx = Px[c] + ((c > 0) ? Px[c - 1] : PxL);
                    const double gy = Pyn + Py[t - 1][c];
                    Py[t - 1][c] = Pyn;
                    GX[q][c] = __builtin_fma(-w * axd, gx, GX[q][c]);
                    if (split)
                        GY[q][c] = __builtin_fma(-w * ayd, gy, GY[q][c]);
                    else
                        GX[q][c] = __builtin_fma(-w * ayd, gy, GX[q][c]);
                    // pin the accumulation here: it is consumed only when the row completes,
                    // and left alone the compiler may defer it there, keeping face products
                    // of several rows alive
                    asm volatile("" : "+v"(GX[q][c]));
                    if (split) asm volatile("" : "+v"(GY[q][c]));
                    nd[c] = fma_t(-Lu, colm[c], Dr[t - 1][pr][c]);
                    nm[c] = fma_t(Ll, colm[c], Mr[t - 1][pr][c]);
                }
                // Dirichlet rows keep du = mu = 0 (and with them u = lam = 0); the row test is
                // wave-uniform, and the empty asm keeps it a scalar branch instead of selects
                if (__builtin_expect(!rin, 0)) {
#pragma unroll
                    for (int c = 0; c < C; ++c) nd[c] = nm[c] = T(0);
                    asm volatile("");
                }
                if (t == 1 && __builtin_expect(any_rec, 0)) {
                    // receivers of row r in the columns this strip computes (halo included:
                    // every copy of a node takes its source), once per row
                    int kb = 0, ke = 0;
                    if (rin) {
                        kb = rowptr[r];
                        ke = rowptr[r + 1];
                        if (kb < ke) {
                            kb = lower_bound_col(rcol, kb, ke, col_lo);
                            ke = lower_bound_col(rcol, kb, ke, col_lo + kWaveSize * C);
                        }
                    }
                    RPb[q] = kb;
                    RPe[q] = ke;
                }
                if (__builtin_expect(any_rec && rin && RPb[q] < RPe[q], 0)) {
                    const int kb = RPb[q], ke = RPe[q];
                    for (int k = kb; k < ke; ++k) {
                        const int off = rcol[k] - cb;
                        if (off >= 0 && off < C) {
                            const T sv = (T)tgrad[n * a.R + rid[k]];
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                if (off == c) nm[c] += sv;
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) nl[c] = fma_t(nm[c], colm[c], Lr[t - 1][pr][c]);
                if (t < K) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        Dr[t][pr][c] = nd[c];
                        Lr[t][pr][c] = nl[c];
                        Mr[t][pr][c] = nm[c];
                    }
                } else if (rown && lane_owned) {
                    const size_t off = (size_t)(ptrdiff_t)r * ld + (size_t)(ptrdiff_t)cb;
                    T uo[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) uo[c] = Ur[t][pr][c];
                    if (a.stream_nt) {
                        store_row_nt<T, C>(uout + off, uo);
                        store_row_nt<T, C>(dout + off, nd);
                        store_row_nt<T, C>(lout + off, nl);
                        store_row_nt<T, C>(mout + off, nm);
                    } else {
                        store_pack<T, C>(uout + off, uo);
                        store_pack<T, C>(dout + off, nd);
                        store_pack<T, C>(lout + off, nl);
                        store_pack<T, C>(mout + off, nm);
                    }
                }
            }
            // the row at position p-K has all K contributions (ring index (p-K) mod K = s mod K)
            {
                const int qd = pmod(s, K);
                const int r = rfirst + dir * (p - K);
                if (r >= r0 && r < r1 && lane_owned) {
                    const size_t off = (size_t)(ptrdiff_t)r * ld + (size_t)(ptrdiff_t)cb;
                    double o1[C], o2[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        o1[c] = gbuf[pb][c] + GX[qd][c];
                        o2[c] = g2buf[pb][c] + GY[qd][c];
                    }
                    if (a.stream_nt) {
                        store_row_nt<double, C>(a.g1 + off, o1);
                        if (split) store_row_nt<double, C>(a.g2 + off, o2);
                    } else {
                        store_pack<double, C>(a.g1 + off, o1);
                        if (split) store_pack<double, C>(a.g2 + off, o2);
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) GX[qd][c] = GY[qd][c] = 0.0;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <typename T, int K, int C>
static hipError_t adj_launch_kc(const AdjArgs& a, int grid, hipStream_t s)
{
    const dim3 g(grid), b(kWaveSize * kWavesPerBlock);
    const bool split = a.g2 != a.g1;
    if (a.face && split)
        hipLaunchKernelGGL((k_adjoint<T, K, C, 1, 1>), g, b, 0, s, a);
    else if (a.face)
        hipLaunchKernelGGL((k_adjoint<T, K, C, 1, 0>), g, b, 0, s, a);
    else if (split)
        hipLaunchKernelGGL((k_adjoint<T, K, C, 0, 1>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, K, C, 0, 0>), g, b, 0, s, a);
    return hipGetLastError();
}

// reverse time blocks 1..KMAX of one (T, C) configuration
template <typename T, int C, int KMAX>
static hipError_t adj_launch_c(const AdjArgs& a, int K, int grid, hipStream_t s)
{
    switch (K) {
    case 1: return adj_launch_kc<T, 1, C>(a, grid, s);
    case 2: return adj_launch_kc<T, 2, C>(a, grid, s);
    case 3: return adj_launch_kc<T, 3, C>(a, grid, s);
    case 4: return adj_launch_kc<T, 4, C>(a, grid, s);
    case 5: return KMAX >= 5 ? adj_launch_kc<T, (KMAX >= 5 ? 5 : 1), C>(a, grid, s) : hipErrorInvalidValue;
    case 6: return KMAX >= 6 ? adj_launch_kc<T, (KMAX >= 6 ? 6 : 1), C>(a, grid, s) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

// One 8-byte value per lane and row (FP32 pairs, FP64 singles) goes up to 6 reverse steps per
// launch at two waves per SIMD; the wider configurations to 4.
template <>
hipError_t launch_adjoint_block<float>(const AdjArgs& a, int K, int C, int grid, hipStream_t s)
{
    if (C == 2) return adj_launch_c<float, 2, 6>(a, K, grid, s);
    if (C == 4) return adj_launch_c<float, 4, 4>(a, K, grid, s);
    return hipErrorInvalidValue;
}
template <>
hipError_t launch_adjoint_block<double>(const AdjArgs& a, int K, int C, int grid, hipStream_t s)
{
    if (C == 1) return adj_launch_c<double, 1, 6>(a, K, grid, s);
    if (C == 2) return adj_launch_c<double, 2, 4>(a, K, grid, s);
    return hipErrorInvalidValue;
}

// Work items (waves) of one reverse launch that the device holds at once, for the item-size
// choice: a launch whose items exceed this by a little runs a second, mostly idle round.
template <typename T, int K, int C>
static int adj_resident_kc(bool face, bool split)
{
    int per_cu = 0;
    const int bs = kWaveSize * kWavesPerBlock;
    hipError_t e;
    if (face && split)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<T, K, C, 1, 1>, bs, 0);
    else if (face)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<T, K, C, 1, 0>, bs, 0);
    else if (split)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<T, K, C, 0, 1>, bs, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<T, K, C, 0, 0>, bs, 0);
    if (e != hipSuccess) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus * kWavesPerBlock;
}

template <typename T, int C, int KMAX>
static int adj_resident_c(int K, bool face, bool split)
{
    switch (K) {
    case 1: return adj_resident_kc<T, 1, C>(face, split);
    case 2: return adj_resident_kc<T, 2, C>(face, split);
    case 3: return adj_resident_kc<T, 3, C>(face, split);
    case 4: return adj_resident_kc<T, 4, C>(face, split);
    case 5: return KMAX >= 5 ? adj_resident_kc<T, (KMAX >= 5 ? 5 : 1), C>(face, split) : 0;
    case 6: return KMAX >= 6 ? adj_resident_kc<T, (KMAX >= 6 ? 6 : 1), C>(face, split) : 0;
    default: return 0;
    }
}

template <>
int adjoint_resident_waves<float>(int K, int C, bool face, bool split)
{
    if (C == 2) return adj_resident_c<float, 2, 6>(K, face, split);
    if (C == 4) return adj_resident_c<float, 4, 4>(K, face, split);
    return 0;
}
template <>
int adjoint_resident_waves<double>(int K, int C, bool face, bool split)
{
    if (C == 1) return adj_resident_c<double, 1, 6>(K, face, split);
    if (C == 2) return adj_resident_c<double, 2, 4>(K, face, split);
    return 0;
}

// lam^N = mu^N = s_N at the receivers (planes already zero).
template <typename T>
__global__ void k_adjoint_seed(T* lam, T* mu, int ld, const int* rec_ij, int R, const double* tg)
{
    // one thread scatters all receivers in order so that coincident receivers add up
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int r = 0; r < R; ++r) {
            const size_t k = (size_t)rec_ij[2 * r + 1] * ld + rec_ij[2 * r];
            lam[k] += (T)tg[r];
            mu[k] += (T)tg[r];
        }
}
template <typename T>
hipError_t launch_adjoint_seed(const AdjArgs& a, int64_t N, hipStream_t s)
{
    // rec_rowptr is unused here; rec_col holds the raw (i, j) pairs in this call
    hipLaunchKernelGGL((k_adjoint_seed<T>), dim3(1), dim3(64), 0, s, (T*)a.lout, (T*)a.mout, a.ld, a.rec_col, a.R,
                       a.trace_grad + N * a.R);
    return hipGetLastError();
}
template hipError_t launch_adjoint_seed<float>(const AdjArgs&, int64_t, hipStream_t);
template hipError_t launch_adjoint_seed<double>(const AdjArgs&, int64_t, hipStream_t);

__global__ void k_grad_out(const double* __restrict__ g, int ld, int nx, int ny, double* __restrict__ out)
{
    const int64_t total = (int64_t)nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / nx), i = (int)(k % nx);
        out[k] = g[(size_t)j * ld + i];
    }
}
hipError_t launch_grad_out(const double* g, int ld, int nx, int ny, double* out, hipStream_t s)
{
    const int64_t total = (int64_t)nx * ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_grad_out, dim3(blocks), dim3(256), 0, s, g, ld, nx, ny, out);
    return hipGetLastError();
}

}  // namespace fdw
