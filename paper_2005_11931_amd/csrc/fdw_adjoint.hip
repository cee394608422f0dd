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

#include <hip/hip_runtime.h>

namespace fdw {

__device__ __forceinline__ int adj_from_left_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int adj_from_right_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float adj_from_left(float v)
{
    return __builtin_bit_cast(float, adj_from_left_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float adj_from_right(float v)
{
    return __builtin_bit_cast(float, adj_from_right_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double adj_from_left(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = adj_from_left_i((int)(b & 0xffffffffLL));
    int hi = adj_from_left_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double adj_from_right(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = adj_from_right_i((int)(b & 0xffffffffLL));
    int hi = adj_from_right_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Same operation order as the forward point update (fdw_kernels.hip), so that the reverse
// reconstruction uses bit-identical operator values.
template <typename T>
__device__ __forceinline__ T adj_flux(T uc, T ue, T uw, T un, T us, T fxe, T fxw, T fyn, T fys, T ax, T ay)
{
    T pe = fxe * (ue - uc);
    T pw = fxw * (uw - uc);
    T pn = fyn * (un - uc);
    T ps = fys * (us - uc);
    T sx = pe + pw;
    T sy = pn + ps;
    return __builtin_fma(ax, sx, ay * sy);
}
template <>
__device__ __forceinline__ float adj_flux<float>(float uc, float ue, float uw, float un, float us, float fxe, float fxw,
                                                 float fyn, float fys, float ax, float ay)
{
    float pe = fxe * (ue - uc);
    float pw = fxw * (uw - uc);
    float pn = fyn * (un - uc);
    float ps = fys * (us - uc);
    float sx = pe + pw;
    float sy = pn + ps;
    return __builtin_fmaf(ax, sx, ay * sy);
}

template <typename T, int C>
struct alignas(sizeof(T) * C) APack {
    T v[C];
};
template <typename T, int C>
__device__ __forceinline__ void aload(const T* __restrict__ p, T (&o)[C])
{
    APack<T, C> q = *reinterpret_cast<const APack<T, C>*>(p);
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = q.v[c];
}
template <typename T, int C>
__device__ __forceinline__ void astore(T* __restrict__ p, const T (&in)[C])
{
    APack<T, C> q;
#pragma unroll
    for (int c = 0; c < C; ++c) q.v[c] = in[c];
    *reinterpret_cast<APack<T, C>*>(p) = q;
}

template <typename T>
struct ALanes;
template <>
struct ALanes<float> {
    static constexpr int C = 4;
};
template <>
struct ALanes<double> {
    static constexpr int C = 2;
};

template <typename T, int K, int FACE>
__global__ __launch_bounds__(kWaveSize * kWavesPerBlock) void k_adjoint(AdjArgs a)
{
    constexpr int C = ALanes<T>::C;
    constexpr int Hx = ((K + C - 1) / C) * C;
    constexpr int Wv = kWaveSize * C - 2 * Hx;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wave >= a.waves) return;

    const int nx = a.nx, ny = a.ny, ld = a.ld;
    const int strip = wave % a.strips;
    const int seg = wave / a.strips;
    const int cb = strip * Wv - Hx + lane * C;
    const bool lane_live = (cb >= 0) && (cb < ld);
    const bool lane_owned = lane_live && (lane * C >= Hx) && (lane * C < Hx + Wv);
    bool colin[C];
#pragma unroll
    for (int c = 0; c < C; ++c) colin[c] = (cb + c >= 1) && (cb + c <= nx - 2);
    const int r0 = seg * a.seg_rows;
    const int r1 = min(r0 + a.seg_rows, ny);

    const T* __restrict__ uin = (const T*)a.uin;
    const T* __restrict__ din = (const T*)a.din;
    const T* __restrict__ lin = (const T*)a.lin;
    const T* __restrict__ mi = (const T*)a.min;
    T* __restrict__ uout = (T*)a.uout;
    T* __restrict__ dout = (T*)a.dout;
    T* __restrict__ lout = (T*)a.lout;
    T* __restrict__ mout = (T*)a.mout;
    const T* __restrict__ hp = (const T*)a.h;
    const T* __restrict__ hyp = (const T*)a.hy;
    const T ax = (T)a.ax, ay = (T)a.ay;
    const double axd = a.ax, ayd = a.ay;
    const bool split = (a.g2 != a.g1);

    // W[s-1]: u^{m-s} rows (r-1, r, r+1) for level s (s = 1..K)
    // D[s], LM[s], MU[s]: level s increments / adjoint / adjoint increments (s = 0..K-1)
    T W[K][3][C];
    T D[K][2][C];
    T LA[K][3][C];
    T MU[K][2][C];
    constexpr int HR = FACE ? 1 : (K + 2);
    constexpr int XR = FACE ? (K + 1) : 1;
    constexpr int YR = FACE ? (K + 2) : 1;
    T Hn[HR][C + 2];
    T FX[XR][C + 1];
    T FY[YR][C];
    double GX[K][C], GY[K][C];  // gradient accumulators: GX[s-1] is row j - s
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            W[s][0][c] = W[s][1][c] = W[s][2][c] = T(0);
            D[s][0][c] = D[s][1][c] = T(0);
            LA[s][0][c] = LA[s][1][c] = LA[s][2][c] = T(0);
            MU[s][0][c] = MU[s][1][c] = T(0);
            GX[s][c] = GY[s][c] = 0.0;
        }
#pragma unroll
    for (int q = 0; q < HR; ++q)
#pragma unroll
        for (int c = 0; c < C + 2; ++c) Hn[q][c] = T(0);
#pragma unroll
    for (int q = 0; q < XR; ++q)
#pragma unroll
        for (int c = 0; c < C + 1; ++c) FX[q][c] = T(0);
#pragma unroll
    for (int q = 0; q < YR; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) FY[q][c] = T(0);

    for (int j = r0 - K; j < r1 + K; ++j) {
        T lu[C], ldd[C], ll[C], lm[C], lh[C], lhy[C];
        const bool rl = lane_live && (j >= 0) && (j < ny);
        if (rl) {
            const size_t off = (size_t)j * ld + cb;
            aload<T, C>(uin + off, lu);
            aload<T, C>(din + off, ldd);
            aload<T, C>(lin + off, ll);
            aload<T, C>(mi + off, lm);
            aload<T, C>(hp + off, lh);
            if (FACE) aload<T, C>(hyp + off, lhy);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) lu[c] = ldd[c] = ll[c] = lm[c] = lh[c] = lhy[c] = T(0);
        }
        const bool jin = (j >= 1) && (j <= ny - 2);
        // level 0 rings
#pragma unroll
        for (int c = 0; c < C; ++c) {
            D[0][0][c] = D[0][1][c];
            D[0][1][c] = ldd[c];
            LA[0][0][c] = LA[0][1][c];
            LA[0][1][c] = LA[0][2][c];
            LA[0][2][c] = ll[c];
            MU[0][0][c] = MU[0][1][c];
            MU[0][1][c] = lm[c];
            // newest row of level 1's u: u^{m-1}(j) = u^m(j) - du^m(j)
            W[0][0][c] = W[0][1][c];
            W[0][1][c] = W[0][2][c];
            W[0][2][c] = (jin && colin[c]) ? (lu[c] - ldd[c]) : T(0);
        }
        if (FACE) {
#pragma unroll
            for (int q = 0; q < XR - 1; ++q)
#pragma unroll
                for (int c = 0; c < C + 1; ++c) FX[q][c] = FX[q + 1][c];
            FX[XR - 1][0] = adj_from_left(lh[C - 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) FX[XR - 1][c + 1] = lh[c];
#pragma unroll
            for (int q = 0; q < YR - 1; ++q)
#pragma unroll
                for (int c = 0; c < C; ++c) FY[q][c] = FY[q + 1][c];
#pragma unroll
            for (int c = 0; c < C; ++c) FY[YR - 1][c] = lhy[c];
        } else {
#pragma unroll
            for (int q = 0; q < HR - 1; ++q)
#pragma unroll
                for (int c = 0; c < C + 2; ++c) Hn[q][c] = Hn[q + 1][c];
            Hn[HR - 1][0] = adj_from_left(lh[C - 1]);
            Hn[HR - 1][C + 1] = adj_from_right(lh[0]);
#pragma unroll
            for (int c = 0; c < C; ++c) Hn[HR - 1][c + 1] = lh[c];
        }

#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int r = j - s;
            const bool rin = (r >= 1) && (r <= ny - 2);
            const bool rown = (r >= r0) && (r < r1);
            const int64_t n = a.n_top - s;  // time index of this level's forward state
            const double w = (n == 0) ? 0.5 : 1.0;
            // u^{n} rows r-1..r+1 (W[s-1]); lam^{n+1} rows r-1..r+1 (LA[s-1])
            const T uL = adj_from_left(W[s - 1][1][C - 1]);
            const T uR = adj_from_right(W[s - 1][1][0]);
            const T lL = adj_from_left(LA[s - 1][1][C - 1]);
            const T lR = adj_from_right(LA[s - 1][1][0]);
            T nd[C], nl[C], nm[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T fxe, fxw, fyn, fys;
                if (FACE) {
                    fxe = FX[K - s][c + 1];
                    fxw = FX[K - s][c];
                    fyn = FY[K + 1 - s][c];
                    fys = FY[K - s][c];
                } else {
                    const int q = K + 1 - s;
                    const T hc = Hn[q][c + 1];
                    fxe = hc + Hn[q][c + 2];
                    fxw = Hn[q][c] + hc;
                    fyn = hc + Hn[q + 1][c + 1];
                    fys = Hn[q - 1][c + 1] + hc;
                }
                const T uc = W[s - 1][1][c];
                const T ue = (c < C - 1) ? W[s - 1][1][c + 1] : uR;
                const T uw = (c > 0) ? W[s - 1][1][c - 1] : uL;
                const T un = W[s - 1][2][c];
                const T us = W[s - 1][0][c];
                const T lc = LA[s - 1][1][c];
                const T le = (c < C - 1) ? LA[s - 1][1][c + 1] : lR;
                const T lw = (c > 0) ? LA[s - 1][1][c - 1] : lL;
                const T ln = LA[s - 1][2][c];
                const T ls = LA[s - 1][0][c];
                const bool in = rin && colin[c];
                const T Lu = adj_flux<T>(uc, ue, uw, un, us, fxe, fxw, fyn, fys, ax, ay);
                nd[c] = in ? (D[s - 1][0][c] - Lu) : T(0);
                const T Ll = adj_flux<T>(lc, le, lw, ln, ls, fxe, fxw, fyn, fys, ax, ay);
                nm[c] = in ? (MU[s - 1][0][c] + Ll) : T(0);
                // gradient (FP64): -w ax [(u_e-u_c)(l_e-l_c) + (u_w-u_c)(l_w-l_c)], likewise in y
                const double gx = (double)(ue - uc) * (double)(le - lc) + (double)(uw - uc) * (double)(lw - lc);
                const double gy = (double)(un - uc) * (double)(ln - lc) + (double)(us - uc) * (double)(ls - lc);
                GX[s - 1][c] += -w * axd * gx;
                GY[s - 1][c] += -w * ayd * gy;
            }
            // adjoint source s_n at the receivers of row r (interior)
            if (a.R > 0 && rin) {
                const int kb = a.rec_rowptr[r], ke = a.rec_rowptr[r + 1];
                for (int k = kb; k < ke; ++k) {
                    const int off = a.rec_col[k] - cb;
                    if (off >= 0 && off < C) {
                        const T sv = (T)a.trace_grad[n * a.R + a.rec_id[k]];
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            if (off == c) nm[c] += sv;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) nl[c] = (rin && colin[c]) ? (LA[s - 1][1][c] + nm[c]) : T(0);
            if (s < K) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    D[s][0][c] = D[s][1][c];
                    D[s][1][c] = nd[c];
                    LA[s][0][c] = LA[s][1][c];
                    LA[s][1][c] = LA[s][2][c];
                    LA[s][2][c] = nl[c];
                    MU[s][0][c] = MU[s][1][c];
                    MU[s][1][c] = nm[c];
                    // newest row of level s+1's u: u^{n-1}(r) = u^n(r) - du^n(r)
                    W[s][0][c] = W[s][1][c];
                    W[s][1][c] = W[s][2][c];
                    W[s][2][c] = (rin && colin[c]) ? (W[s - 1][1][c] - nd[c]) : T(0);
                }
            } else if (rown && lane_owned) {
                const size_t off = (size_t)r * ld + cb;
                T uo[C];
#pragma unroll
                for (int c = 0; c < C; ++c) uo[c] = W[s - 1][1][c];
                astore<T, C>(uout + off, uo);
                astore<T, C>(dout + off, nd);
                astore<T, C>(lout + off, nl);
                astore<T, C>(mout + off, nm);
            }
        }
        // row j - K has all K contributions: add them to the accumulator plane(s)
        {
            const int r = j - K;
            if (r >= r0 && r < r1 && lane_owned) {
                const size_t off = (size_t)r * ld + cb;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (split) {
                        a.g1[off + c] += GX[K - 1][c];
                        a.g2[off + c] += GY[K - 1][c];
                    } else {
                        a.g1[off + c] += GX[K - 1][c] + GY[K - 1][c];
                    }
                }
            }
#pragma unroll
            for (int s = K - 1; s > 0; --s)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    GX[s][c] = GX[s - 1][c];
                    GY[s][c] = GY[s - 1][c];
                }
#pragma unroll
            for (int c = 0; c < C; ++c) GX[0][c] = GY[0][c] = 0.0;
        }
    }
}

template <typename T, int K>
static hipError_t adj_launch_k(const AdjArgs& a, int grid, hipStream_t s)
{
    if (a.face)
        hipLaunchKernelGGL((k_adjoint<T, K, 1>), dim3(grid), dim3(kWaveSize * kWavesPerBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, K, 0>), dim3(grid), dim3(kWaveSize * kWavesPerBlock), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_block(const AdjArgs& a, int K, int grid, hipStream_t s)
{
    switch (K) {
    case 1: return adj_launch_k<T, 1>(a, grid, s);
    case 2: return adj_launch_k<T, 2>(a, grid, s);
    case 3: return adj_launch_k<T, 3>(a, grid, s);
    case 4: return adj_launch_k<T, 4>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_adjoint_block<float>(const AdjArgs&, int, int, hipStream_t);
template hipError_t launch_adjoint_block<double>(const AdjArgs&, int, int, hipStream_t);

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
