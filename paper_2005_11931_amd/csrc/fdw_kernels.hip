// fdw_kernels.hip - gfx950 kernels of the explicit leapfrog solver of
//     u_tt = d_x(h1 d_x u) + d_y(h2 d_y u),  zero Dirichlet data,
// the regularised Cauchy problem of arXiv 2005.11931 (Section 2, eq. (2.1); grid and
// boundary data of Section 3.3).
//
// The hot kernel (k_step) is a y-streaming, temporally blocked sweep.  Each wavefront owns a
// column strip of the grid and a segment of rows; its 64 lanes hold C consecutive columns
// each (one 16-byte vector per lane and row, so a wave reads 1 KiB contiguous per row and
// array).  The wave walks down its segment one row at a time and advances K time levels at
// once: level t computes row j - t from level t-1's rows j-t-1 .. j-t+1, which it holds in
// registers, so every input element is read from HBM once per K steps and every output is
// written once per K steps.  Horizontal neighbours cross lanes with DPP wave shifts; the
// strip carries a K-column halo on each side (recomputed, never written) so that waves are
// independent and need no barrier.  All variants (any K, any segment length, batched or
// not) evaluate each grid point with the same function in the same operation order, so
// their results agree bit for bit.
//
// State: increment form (u^n, du^n = u^n - u^{n-1}); the step is
//     du^{n+1} = du^n + L(u^n),   u^{n+1} = u^n + du^{n+1},   L = tau^2 A(h),
// identical to u^{n+1} = 2u^n - u^{n-1} + tau^2 A u^n in exact arithmetic.
// Energy (discrete CL-01 of Section 2): E^{n+1/2} = (dx dy / tau^2) sum (du^{n+1})^2 - u^{n+1} L(u^n),
// accumulated in FP64 per wave, reduced in a fixed order.
#include "fdw_internal.h"
#include "fdw_stream.h"

#include <hip/hip_runtime.h>

namespace fdw {

// stencil launchers, one per instantiation unit (fdw_step_*.hip)
hipError_t launch_step_f32c4(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s);
hipError_t launch_step_f32c2(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s);
hipError_t launch_step_f64c2(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s);
hipError_t launch_step_f64c1(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s);
hipError_t launch_persistent_f32c4(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s);
hipError_t launch_persistent_f32c2(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s);
hipError_t launch_persistent_f64c2(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s);
hipError_t launch_persistent_f64c1(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s);
int persistent_max_f32c4(int K, int face_mode, bool energy);
int persistent_max_f32c2(int K, int face_mode, bool energy);
int persistent_max_f64c2(int K, int face_mode, bool energy);
int persistent_max_f64c1(int K, int face_mode, bool energy);

template <>
hipError_t launch_step<float>(const StepArgs& a, int K, int C, int face_mode, int grid, hipStream_t s)
{
    if (C == 4) return launch_step_f32c4(a, K, face_mode, grid, s);
    if (C == 2) return launch_step_f32c2(a, K, face_mode, grid, s);
    return hipErrorInvalidValue;
}
template <>
hipError_t launch_step<double>(const StepArgs& a, int K, int C, int face_mode, int grid, hipStream_t s)
{
    if (C == 2) return launch_step_f64c2(a, K, face_mode, grid, s);
    if (C == 1) return launch_step_f64c1(a, K, face_mode, grid, s);
    return hipErrorInvalidValue;
}
template <>
hipError_t launch_step_persistent<float>(const StepArgs& a, int K, int C, int face_mode, int phases, int grid, int* bar,
                                         const PersistentExtra& x, hipStream_t s)
{
    if (C == 4) return launch_persistent_f32c4(a, K, face_mode, phases, grid, bar, x, s);
    if (C == 2) return launch_persistent_f32c2(a, K, face_mode, phases, grid, bar, x, s);
    return hipErrorInvalidValue;
}
template <>
hipError_t launch_step_persistent<double>(const StepArgs& a, int K, int C, int face_mode, int phases, int grid,
                                          int* bar, const PersistentExtra& x, hipStream_t s)
{
    if (C == 2) return launch_persistent_f64c2(a, K, face_mode, phases, grid, bar, x, s);
    if (C == 1) return launch_persistent_f64c1(a, K, face_mode, phases, grid, bar, x, s);
    return hipErrorInvalidValue;
}
template <>
int persistent_max_blocks<float>(int K, int C, int face_mode, bool energy)
{
    if (C == 4) return persistent_max_f32c4(K, face_mode, energy);
    if (C == 2) return persistent_max_f32c2(K, face_mode, energy);
    return 0;
}
template <>
int persistent_max_blocks<double>(int K, int C, int face_mode, bool energy)
{
    if (C == 2) return persistent_max_f64c2(K, face_mode, energy);
    if (C == 1) return persistent_max_f64c1(K, face_mode, energy);
    return 0;
}

// ------------------------------------------------------------------------------------------
// Energy finalisation: E = escale * sum over waves of the per-wave partials, fixed order.
// grid = (levels, nmembers, time blocks)
// ------------------------------------------------------------------------------------------
// Sum of one level's per-wave partials by a block of 256 (fixed order: four strided chains per
// thread, then a tree).
__device__ double level_partial_sum(const MemberDev& M, int slot, int t, double* red)
{
    const double* p = M.epart + ((size_t)slot * kMaxTimeBlock + t) * M.epart_stride;
    // four independent chains so that the loads of a thread are in flight together
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    const int nw = M.waves;
    int w = threadIdx.x;
    for (; w + 3 * 256 < nw; w += 4 * 256) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s4[q] += p[w + q * 256];
    }
    for (; w < nw; w += 256) s4[0] += p[w];
    red[threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_energy_finalize(const MemberDev* table, int first, double* energy_base,
                                                         int64_t energy_stride, int64_t energy_offset, int* health,
                                                         int slot)
{
    const int t = blockIdx.x;
    const int m = first + blockIdx.y;
    const int j = blockIdx.z;  // time block within the group
    const MemberDev& M = table[m];
    __shared__ double red[256];
    const double E = level_partial_sum(M, slot + j, t, red) * M.escale;
    const int64_t off = energy_offset + (int64_t)j * gridDim.x + t;
    const int64_t row = (int64_t)M.energy_row * energy_stride;
    // the first energy of the call, for the growth test: written by an earlier launch, or (when
    // this group starts the call) summed here again from its partials, the same way
    double E0 = 0.0;
    if (health && off > 0) E0 = (energy_offset == 0) ? level_partial_sum(M, slot, 0, red) * M.escale : energy_base[row];
    if (threadIdx.x == 0) {
        energy_base[row + off] = E;
        if (health) {
            // failure detection: a non-finite energy (bit 0), or growth beyond 10x the first
            // energy of the call (bit 1)
            if (!isfinite(E)) atomicOr(health, 1);
            if (off > 0 && fabs(E) > 10.0 * fabs(E0)) atomicOr(health, 2);
        }
    }
}

template <typename T>
hipError_t launch_energy_finalize(const MemberDev* table, int first, int nmembers, int levels, double* energy_base,
                                  int64_t energy_stride, int64_t energy_offset, int* health, hipStream_t s, int slot,
                                  int nslots)
{
    hipLaunchKernelGGL(k_energy_finalize, dim3(levels, nmembers, nslots), dim3(256), 0, s, table, first, energy_base,
                       energy_stride, energy_offset, health, slot);
    return hipGetLastError();
}
template hipError_t launch_energy_finalize<float>(const MemberDev*, int, int, int, double*, int64_t, int64_t, int*,
                                                  hipStream_t, int, int);
template hipError_t launch_energy_finalize<double>(const MemberDev*, int, int, int, double*, int64_t, int64_t, int*,
                                                   hipStream_t, int, int);

// ------------------------------------------------------------------------------------------
// Block reduction helpers (fixed order) for the generic two-stage reductions.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of partials[0..n) into *out, fixed order (one block of 256).
__global__ __launch_bounds__(256) void k_sum_partials(const double* partials, int n, double scale, double* out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partials[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s * scale;
}

// ------------------------------------------------------------------------------------------
// Coefficient preparation.  Nodal layout: copy h (dense) into the pitched plane.  Face
// layout: FX = h1_i + h1_{i+1}, FY = h2_j + h2_{j+1} (twice the face means).  Statistics for
// validation and the stability check go to red[]: per block {min h, max hx face, max hy face,
// non-finite count}.
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_prepare_coeff(const T* __restrict__ h1, const T* __restrict__ h2, int nx,
                                                       int ny, int ld, int face, T* __restrict__ H, T* __restrict__ HY,
                                                       double* red)
{
    __shared__ double sh[256];
    double mn = 1e300, mx = 0.0, my = 0.0, bad = 0.0;
    const int64_t total = (int64_t)ld * ny;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int j = (int)(k / ld), i = (int)(k % ld);
        if (i >= nx) {
            H[k] = T(0);
            if (face) HY[k] = T(0);
            continue;
        }
        const T a = h1[(size_t)j * nx + i];
        const T b = h2[(size_t)j * nx + i];
        const double ad = (double)a, bd = (double)b;
        if (!(ad == ad) || ad - ad != 0.0 || !(bd == bd) || bd - bd != 0.0) bad += 1.0;
        mn = fmin(mn, fmin(ad, bd));
        if (i < nx - 1) mx = fmax(mx, 0.5 * (ad + (double)h1[(size_t)j * nx + i + 1]));
        if (j < ny - 1) my = fmax(my, 0.5 * (bd + (double)h2[(size_t)(j + 1) * nx + i]));
        if (face) {
            H[k] = (i < nx - 1) ? (a + h1[(size_t)j * nx + i + 1]) : T(0);
            HY[k] = (j < ny - 1) ? (b + h2[(size_t)(j + 1) * nx + i]) : T(0);
        } else {
            H[k] = a;
        }
    }
    // block min/max via shared memory (order-independent)
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x * 4 + 0] = sh[0];
    __syncthreads();
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x * 4 + 1] = sh[0];
    __syncthreads();
    sh[threadIdx.x] = my;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x * 4 + 2] = sh[0];
    __syncthreads();
    const double nb = block_sum(bad, sh);
    if (threadIdx.x == 0) red[blockIdx.x * 4 + 3] = nb;
}

__global__ __launch_bounds__(256) void k_coeff_stats_final(double* red, int nblocks)
{
    __shared__ double sh[256];
    double mn = 1e300, mx = 0.0, my = 0.0, bad = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        mn = fmin(mn, red[b * 4 + 0]);
        mx = fmax(mx, red[b * 4 + 1]);
        my = fmax(my, red[b * 4 + 2]);
        bad += red[b * 4 + 3];
    }
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double rmn = sh[0];
    __syncthreads();
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double rmx = sh[0];
    __syncthreads();
    sh[threadIdx.x] = my;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double rmy = sh[0];
    __syncthreads();
    const double rb = block_sum(bad, sh);
    if (threadIdx.x == 0) {
        // results land after the per-block area: red[4*kRedBlocks + 0..3]
        red[4 * kRedBlocks + 0] = rmn;
        red[4 * kRedBlocks + 1] = rmx;
        red[4 * kRedBlocks + 2] = rmy;
        red[4 * kRedBlocks + 3] = rb;
    }
}

template <typename T>
hipError_t launch_prepare_coeff(const MemberDev* m, const void* h1, const void* h2, int face, double* red,
                                hipStream_t s)
{
    const int64_t total = (int64_t)m->ld * m->ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL((k_prepare_coeff<T>), dim3(blocks), dim3(256), 0, s, (const T*)h1, (const T*)(h2 ? h2 : h1),
                       m->nx, m->ny, m->ld, face, (T*)m->h, (T*)m->hy, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_coeff_stats_final, dim3(1), dim3(256), 0, s, red, blocks);
    return hipGetLastError();
}
template hipError_t launch_prepare_coeff<float>(const MemberDev*, const void*, const void*, int, double*, hipStream_t);
template hipError_t launch_prepare_coeff<double>(const MemberDev*, const void*, const void*, int, double*, hipStream_t);

// ------------------------------------------------------------------------------------------
// Start step.  du^1 = tau u1 + L(u^0)/2, u^1 = u^0 + du^1 (interior), written to pair 0;
// energy partials per block into red[], optional trace row 1.
// ------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void face_sums(const MemberDev& M, const T* hp, const T* hyp, int j, int i, T& fxe, T& fxw,
                                          T& fyn, T& fys)
{
    const size_t k = (size_t)j * M.ld + i;
    if (M.face) {
        fxe = hp[k];
        fxw = hp[k - 1];
        fyn = hyp[k];
        fys = hyp[k - M.ld];
    } else {
        const T hc = hp[k];
        fxe = hc + hp[k + 1];
        fxw = hp[k - 1] + hc;
        fyn = hc + hp[k + M.ld];
        fys = hp[k - M.ld] + hc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_start(MemberDev M, const T* __restrict__ u0, const T* __restrict__ u1, T tau,
                                               int want_energy, double* red)
{
    __shared__ double sh[256];
    const T* hp = (const T*)M.h;
    const T* hyp = (const T*)M.hy;
    T* uo = (T*)M.u[0];
    T* dout = (T*)M.d[0];
    const T ax = (T)M.ax, ay = (T)M.ay;
    double acc = 0.0;
    const int64_t total = (int64_t)M.ld * M.ny;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int j = (int)(k / M.ld), i = (int)(k % M.ld);
        const bool in = (i >= 1) && (i <= M.nx - 2) && (j >= 1) && (j <= M.ny - 2);
        T nu = T(0), nd = T(0);
        if (in) {
            T fxe, fxw, fyn, fys;
            face_sums<T>(M, hp, hyp, j, i, fxe, fxw, fyn, fys);
            const T uc = u0[k];
            const T L = flux_L<T>(uc, u0[k + 1], u0[k - 1], u0[k + M.ld], u0[k - M.ld], fxe, fxw, fyn, fys, ax, ay);
            const T a = tau * u1[k];
            const T b = T(0.5) * L;
            nd = a + b;
            nu = uc + nd;
            if (want_energy) acc += __builtin_fma(-(double)nu, (double)L, (double)nd * (double)nd);
        }
        uo[k] = nu;
        dout[k] = nd;
    }
    if (want_energy) {
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) red[blockIdx.x] = s;
    }
}

template <typename T>
hipError_t launch_start(const MemberDev* m, const MemberDev* m_dev, const void* u0, const void* u1, T tau,
                        int want_energy, int want_trace, double* energy_out, double* red, hipStream_t s)
{
    const int64_t total = (int64_t)m->ld * m->ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL((k_start<T>), dim3(blocks), dim3(256), 0, s, *m, (const T*)u0, (const T*)u1, tau, want_energy,
                       red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (want_energy) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, red, blocks, m->escale, energy_out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    (void)m_dev;
    (void)want_trace;
    return hipSuccess;
}
template hipError_t launch_start<float>(const MemberDev*, const MemberDev*, const void*, const void*, float, int, int,
                                        double*, double*, hipStream_t);
template hipError_t launch_start<double>(const MemberDev*, const MemberDev*, const void*, const void*, double, int,
                                         int, double*, double*, hipStream_t);

// ------------------------------------------------------------------------------------------
// E^{n-1/2} of a stored state (u^n, du^n): escale * sum du^2 - (u - du) L(u).
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_state_energy(MemberDev M, int cur, double* red)
{
    __shared__ double sh[256];
    const T* hp = (const T*)M.h;
    const T* hyp = (const T*)M.hy;
    const T* u = (const T*)M.u[cur];
    const T* du = (const T*)M.d[cur];
    const T ax = (T)M.ax, ay = (T)M.ay;
    double acc = 0.0;
    const int64_t total = (int64_t)M.ld * M.ny;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int j = (int)(k / M.ld), i = (int)(k % M.ld);
        if (i < 1 || i > M.nx - 2 || j < 1 || j > M.ny - 2) continue;
        T fxe, fxw, fyn, fys;
        face_sums<T>(M, hp, hyp, j, i, fxe, fxw, fyn, fys);
        const T L = flux_L<T>(u[k], u[k + 1], u[k - 1], u[k + M.ld], u[k - M.ld], fxe, fxw, fyn, fys, ax, ay);
        const double d = (double)du[k];
        const double prev = (double)u[k] - d;
        acc += __builtin_fma(-prev, (double)L, d * d);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

template <typename T>
hipError_t launch_state_energy(const MemberDev* m, int cur, double* red, double* out, hipStream_t s)
{
    const int64_t total = (int64_t)m->ld * m->ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL((k_state_energy<T>), dim3(blocks), dim3(256), 0, s, *m, cur, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, red, blocks, m->escale, out);
    return hipGetLastError();
}
template hipError_t launch_state_energy<float>(const MemberDev*, int, double*, double*, hipStream_t);
template hipError_t launch_state_energy<double>(const MemberDev*, int, double*, double*, hipStream_t);

// ------------------------------------------------------------------------------------------
// Trace gather of one state row, and the FP64 misfit with its adjoint source.
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_gather(const T* __restrict__ u, int ld, const int* __restrict__ rec_ij, int R, T* __restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) out[r] = u[(size_t)rec_ij[2 * r + 1] * ld + rec_ij[2 * r]];
}
template <typename T>
hipError_t launch_gather(const void* u, int ld, const int* rec_ij, int R, void* out_row, hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather<T>), dim3((R + 255) / 256), dim3(256), 0, s, (const T*)u, ld, rec_ij, R, (T*)out_row);
    return hipGetLastError();
}
template hipError_t launch_gather<float>(const void*, int, const int*, int, void*, hipStream_t);
template hipError_t launch_gather<double>(const void*, int, const int*, int, void*, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_misfit(const T* __restrict__ tr, const double* __restrict__ d, int64_t n,
                                                double* __restrict__ grad, double* red)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        const double e = (double)tr[k] - d[k];
        acc += e * e;
        if (grad) grad[k] = 2.0 * e;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}
template <typename T>
hipError_t launch_misfit(const void* traces, const double* d, int64_t n, double* J, double* grad, double* red,
                         hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_misfit<T>), dim3(blocks), dim3(256), 0, s, (const T*)traces, d, n, grad, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, red, blocks, 1.0, J);
    return hipGetLastError();
}
template hipError_t launch_misfit<float>(const void*, const double*, int64_t, double*, double*, double*, hipStream_t);
template hipError_t launch_misfit<double>(const void*, const double*, int64_t, double*, double*, double*, hipStream_t);

// ------------------------------------------------------------------------------------------
// Squared L2 distance of two fields (FP64 accumulation, fixed order).
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_diff_norm(const T* __restrict__ a, const T* __restrict__ b, int ld, int nx,
                                                   int64_t total, double* red)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        if ((int)(k % ld) >= nx) continue;
        const double d = (double)a[k] - (double)b[k];
        acc += d * d;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = sum;
}
template <typename T>
hipError_t launch_diff_norm(const void* a, const void* b, int ld, int nx, int ny, double scale, double* red,
                            double* out, hipStream_t s)
{
    const int64_t total = (int64_t)ld * ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL((k_diff_norm<T>), dim3(blocks), dim3(256), 0, s, (const T*)a, (const T*)b, ld, nx, total, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, red, blocks, scale, out);
    return hipGetLastError();
}
template hipError_t launch_diff_norm<float>(const void*, const void*, int, int, int, double, double*, double*,
                                            hipStream_t);
template hipError_t launch_diff_norm<double>(const void*, const void*, int, int, int, double, double*, double*,
                                             hipStream_t);

// ------------------------------------------------------------------------------------------
// Layout conversion: dense caller arrays <-> pitched planes (boundary ring zeroed on input).
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_copy_in(const T* __restrict__ src, int nx, int ny, T* __restrict__ dst, int ld, int zero_ring)
{
    const int64_t total = (int64_t)ld * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / ld), i = (int)(k % ld);
        T v = T(0);
        if (i < nx) {
            const bool ring = (i == 0) || (j == 0) || (i == nx - 1) || (j == ny - 1);
            v = (zero_ring && ring) ? T(0) : src[(size_t)j * nx + i];
        }
        dst[k] = v;
    }
}
template <typename T>
hipError_t launch_copy_in(const void* src, int nx, int ny, void* dst, int ld, int zero_ring, hipStream_t s)
{
    const int64_t total = (int64_t)ld * ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_copy_in<T>), dim3(blocks), dim3(256), 0, s, (const T*)src, nx, ny, (T*)dst, ld, zero_ring);
    return hipGetLastError();
}
template hipError_t launch_copy_in<float>(const void*, int, int, void*, int, int, hipStream_t);
template hipError_t launch_copy_in<double>(const void*, int, int, void*, int, int, hipStream_t);

template <typename T>
__global__ void k_copy_out(const T* __restrict__ src, int ld, int nx, int ny, T* __restrict__ dst)
{
    const int64_t total = (int64_t)nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / nx), i = (int)(k % nx);
        dst[k] = src[(size_t)j * ld + i];
    }
}
template <typename T>
hipError_t launch_copy_out(const void* src, int ld, int nx, int ny, void* dst, hipStream_t s)
{
    const int64_t total = (int64_t)nx * ny;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_copy_out<T>), dim3(blocks), dim3(256), 0, s, (const T*)src, ld, nx, ny, (T*)dst);
    return hipGetLastError();
}
template hipError_t launch_copy_out<float>(const void*, int, int, int, void*, hipStream_t);
template hipError_t launch_copy_out<double>(const void*, int, int, int, void*, hipStream_t);

__global__ void k_fill_bytes(uint4* p, size_t n16, unsigned char* tail, size_t ntail)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
        p[k] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}
__global__ void k_set_int(int* p, int v) { *p = v; }
hipError_t launch_set_int(int* p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_fill_bytes(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    // p is 256-byte aligned (workspace carving); bytes may have a tail below 16
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_bytes, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16,
                       (unsigned char*)p + n16 * 16, ntail);
    return hipGetLastError();
}

// Receivers (i, j) -> CSR by row, sorted by (row, column), with validation.  One block; R is
// at most kMaxReceivers.  status[0] = 0 on success, 1 if a receiver is not an interior node;
// status[1] = number of receivers that share their node with an earlier one in that order.
__global__ __launch_bounds__(256) void k_receivers_csr(const int* __restrict__ rec, int R, int nx, int ny,
                                                       int* __restrict__ rowptr, int* __restrict__ col,
                                                       int* __restrict__ id, int* status)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += 256) {
        const int i = rec[2 * r], j = rec[2 * r + 1];
        if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) status[0] = 1;
        return;
    }
    // rank of each receiver in (row, column, index) order: O(R^2 / 256), fine for R <= 16384
    for (int r = threadIdx.x; r < R; r += 256) {
        const int i = rec[2 * r], j = rec[2 * r + 1];
        int rank = 0;
        for (int q = 0; q < R; ++q) {
            const int iq = rec[2 * q], jq = rec[2 * q + 1];
            const bool before = (jq < j) || (jq == j && (iq < i || (iq == i && q < r)));
            rank += before ? 1 : 0;
        }
        col[rank] = i;
        id[rank] = r;
    }
    // row pointers: rowptr[y] = number of receivers with row < y
    for (int y = threadIdx.x; y <= ny; y += 256) {
        int c = 0;
        for (int q = 0; q < R; ++q) c += (rec[2 * q + 1] < y) ? 1 : 0;
        rowptr[y] = c;
    }
    __shared__ int dups;
    if (threadIdx.x == 0) dups = 0;
    __syncthreads();  // col / id complete
    for (int k = 1 + (int)threadIdx.x; k < R; k += 256) {
        const int a = id[k], b = id[k - 1];
        if (rec[2 * a] == rec[2 * b] && rec[2 * a + 1] == rec[2 * b + 1]) atomicAdd(&dups, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        status[0] = 0;
        status[1] = dups;
    }
}

// The stepping kernels record one trace per receiver node (the first receiver of each run of
// coincident ones in CSR order); copy that column to the other receivers of the run for trace
// rows lo..hi.
__global__ void k_trace_dups(char* __restrict__ traces, int es, int R, const int* __restrict__ rec,
                             const int* __restrict__ id, int64_t lo, int64_t hi)
{
    const int64_t total = (hi - lo + 1) * (int64_t)R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = lo + e / R;
        const int k = (int)(e % R);
        if (k == 0) continue;
        const int a = id[k];
        int k0 = k;
        while (k0 > 0 && rec[2 * id[k0 - 1]] == rec[2 * a] && rec[2 * id[k0 - 1] + 1] == rec[2 * a + 1]) --k0;
        if (k0 == k) continue;
        const int src = id[k0];
        char* row = traces + n * (int64_t)R * es;
        if (es == 8)
            ((double*)row)[a] = ((const double*)row)[src];
        else
            ((float*)row)[a] = ((const float*)row)[src];
    }
}
hipError_t launch_trace_dups(void* traces, int es, int R, const int* rec_ij, const int* id, int64_t lo, int64_t hi,
                             hipStream_t s)
{
    if (hi < lo || R <= 1) return hipSuccess;
    const int64_t total = (hi - lo + 1) * (int64_t)R;
    const int64_t want = (total + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_trace_dups, dim3(blocks), dim3(256), 0, s, (char*)traces, es, R, rec_ij, id, lo, hi);
    return hipGetLastError();
}
hipError_t launch_receivers_csr(const int* rec_ij, int R, int nx, int ny, int* rowptr, int* col, int* id, int* status,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_receivers_csr, dim3(1), dim3(256), 0, s, rec_ij, R, nx, ny, rowptr, col, id, status);
    return hipGetLastError();
}

}  // namespace fdw
