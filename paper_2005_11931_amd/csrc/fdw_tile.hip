// fdw_tile.hip - the leapfrog time block for small grids (Section 2, the explicit scheme of
// eq. (2.1) on the Section 3.3 grid; the same point update as the streaming kernel).
//
// On a grid of a few hundred nodes a side the streaming kernel has too few work items to fill
// the device, and each of them is a long serial chain: one wave walks S + 2K rows through K
// levels.  Here one workgroup owns a tile of 64 columns (48 owned, 8 halo columns on each
// side) and NW * 4 rows (8 halo rows above and below), held in registers: each wave keeps 4
// rows of (u, du) and their face coefficients, and the waves advance the tile level by level
// together, exchanging their edge rows through LDS with one barrier per level.  The halo is
// deep enough for any time block up to 8: after K levels the owned nodes are exact, and they
// are computed with the same operations in the same order as in the streaming kernel, so both
// kernels produce the same bits.  Energy partials: one per tile and level, summed over the
// tile's waves in a fixed order.
#include "fdw_stream.h"
#include "fdw_tile.h"

namespace fdw {

namespace {

// v from another lane of the same row of 16 lanes (DPP control CTRL; every source lane exists)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const unsigned int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const unsigned int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// MODE bit 0: per-step energy partials.  FACE: coefficient layout as in the streaming kernel.
template <typename T, int FACE, int MODE>
__global__ __launch_bounds__(kWaveSize * kMaxTileWaves) void k_step_tile(StepArgs a, int K)
{
    constexpr bool want_energy = (MODE & 1) != 0;
    constexpr int RW = kTileRowsPerWave;
    __shared__ T s_edge[2][kMaxTileWaves][2][kWaveSize];  // first / last row of every wave, two levels
    __shared__ double s_e[kMaxTimeBlock][kMaxTileWaves];  // energy partial of every wave and level

    const int NW = (int)(blockDim.x >> 6);
    const int w = wave_in_block();
    const int lane = threadIdx.x & 63;
    const int gb = (int)blockIdx.x + a.block_offset;
    const int m = (a.nmembers == 1) ? a.first : find_member(a.table, a.first, a.nmembers, gb);
    const MemberDev& M = a.table[m];
    // Every field of the member the prologue needs is read here, before any of them is used, so
    // that all table reads are one round of scalar loads ahead of the plane loads (left to the
    // scheduler they were split into several dependent rounds around the index arithmetic).
    // Both pointers of each pair are read and then selected by the parity.  The grid holds
    // exactly the members' tiles: no tile test.
    const int nx = M.nx, ny = M.ny, ld = M.ld;
    const int strips = M.strips, seg_rows = M.seg_rows, block_base = M.block_base, cur0 = M.cur0;
    void* const u0p = M.u[0];
    void* const u1p = M.u[1];
    void* const d0p = M.d[0];
    void* const d1p = M.d[1];
    void* const hv = M.h;
    void* const hyv = M.hy;
    const double axd = M.ax, ayd = M.ay;
    __builtin_amdgcn_sched_barrier(0);
    const int tile = gb - block_base;

    const int strip = tile % strips;
    const int seg = tile / strips;
    const int cb = strip * kTileCols - kTileHalo + lane;  // grid column of this lane
    const bool lane_live = (cb >= 0) && (cb < ld);
    const bool lane_owned = lane_live && (lane >= kTileHalo) && (lane < kTileHalo + kTileCols);
    const T colm = ((cb >= 1) && (cb <= nx - 2)) ? T(1) : T(0);
    const int r0 = seg * seg_rows;
    const int r1 = min(r0 + seg_rows, ny);
    const int g0 = r0 - kTileHalo + w * RW;  // grid row of the wave's first row

    const bool cur = ((cur0 ^ a.parity) & 1) != 0;
    const T* __restrict__ uin = (const T*)(cur ? u1p : u0p);
    const T* __restrict__ din = (const T*)(cur ? d1p : d0p);
    T* __restrict__ uout = (T*)(cur ? u0p : u1p);
    T* __restrict__ dout = (T*)(cur ? d0p : d1p);
    const T* __restrict__ hp = (const T*)hv;
    const T* __restrict__ hyp = (const T*)hyv;
    const T ax = (T)axd, ay = (T)ayd;

    // Rows and columns outside the plane read as 0, as in the streaming kernel: the loads go
    // through buffer resources, whose out-of-range offsets return 0 in hardware.  (A load under
    // a lane test compiles to a branch around it and a wait right after it: fourteen
    // serialised memory latencies before the first level.)  The resources start at the first
    // row the tile reads, so that every offset stays far below 2^31.
    const int jbase = max(r0 - kTileHalo - 1, 0);
    const size_t span = (size_t)(ny - jbase) * ld * sizeof(T);
    const unsigned int nbytes =
        __builtin_amdgcn_readfirstlane((unsigned int)min(span, (size_t)kBufferOutOfRange - 16));
    const size_t base_el = (size_t)jbase * ld;
    const __amdgpu_buffer_rsrc_t ru = plane_rsrc(uniform_ptr(uin + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rd = plane_rsrc(uniform_ptr(din + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rh = plane_rsrc(uniform_ptr(hp + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rhy = plane_rsrc(uniform_ptr((FACE ? hyp : hp) + base_el), nbytes);
    auto at = [&](__amdgpu_buffer_rsrc_t r, int g) -> T {
        const unsigned int off = (lane_live && g >= 0 && g < ny)
                                     ? (unsigned int)((g - jbase) * ld + cb) * (unsigned int)sizeof(T)
                                     : kBufferOutOfRange;
        if constexpr (sizeof(T) == 8) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
        }
    };

    T u[RW], d[RW], FX[RW], FY[RW];  // FY[i]: face between rows i and i + 1 of the wave
    T FYup;                          // face between the row above the wave and its first row
    if (FACE) {
        // face sums: FX = h1_c + h1_{c+1} in h, FY = h2_r + h2_{r+1} in hy (stored at row r)
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            u[i] = at(ru, g0 + i);
            d[i] = at(rd, g0 + i);
            FX[i] = ax * at(rh, g0 + i);
            FY[i] = ay * at(rhy, g0 + i);
        }
        FYup = ay * at(rhy, g0 - 1);
    } else {
        T hr[RW + 2];  // nodal h of rows g0 - 1 .. g0 + RW
#pragma unroll
        for (int j = 0; j < RW + 2; ++j) hr[j] = at(rh, g0 - 1 + j);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            u[i] = at(ru, g0 + i);
            d[i] = at(rd, g0 + i);
            FX[i] = ax * (hr[i + 1] + lane_from_right(hr[i + 1]));
            FY[i] = ay * (hr[i + 1] + hr[i + 2]);
        }
        FYup = ay * (hr[0] + hr[1]);
    }

    // per-lane energy terms of every level, reduced over the wave once after the last level
    // (the K reductions are then independent and their lane exchanges overlap; reduced level
    // by level they would put six dependent exchanges into every level's critical path)
    double acc[kMaxTimeBlock];
#pragma unroll
    for (int t = 0; t < kMaxTimeBlock; ++t) acc[t] = 0.0;

#pragma unroll
    for (int t = 0; t < kMaxTimeBlock; ++t) {
        if (t >= K) break;
        const int b = t & 1;
        s_edge[b][w][0][lane] = u[0];
        s_edge[b][w][1][lane] = u[RW - 1];
        __syncthreads();
        // the tile's first and last rows see 0 beyond them: only halo rows are affected
        const T above = (w > 0) ? s_edge[b][w - 1][1][lane] : T(0);
        const T below = (w < NW - 1) ? s_edge[b][w + 1][0][lane] : T(0);
        // y flux across the face above each row, carried from row to row:
        // sy = fy_{r+1/2}(u_{r+1} - u_r) - fy_{r-1/2}(u_r - u_{r-1})
        T Gp = FYup * (u[0] - above);
        T eb = T(0);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const T un = (i < RW - 1) ? u[i + 1] : below;
            const T Gn = FY[i] * (un - u[i]);
            const T F = FX[i] * (lane_from_right(u[i]) - u[i]);
            const T Fl = lane_from_left(F);
            const T sx = F - Fl;
            const T sy = Gn - Gp;
            Gp = Gn;
            const T L = sx + sy;
            const int g = g0 + i;
            T nd = fma_t(L, colm, d[i]);
            if (!((g >= 1) && (g <= ny - 2))) nd = T(0);  // Dirichlet rows (and rows outside the grid)
            const T nu = u[i] + nd;
            if (want_energy && g >= r0 && g < r1) {
                eb = fma_t(nd, nd, eb);
                eb = fma_t(-nu, L, eb);
            }
            u[i] = nu;
            d[i] = nd;
        }
        if (want_energy) acc[t] = lane_owned ? (double)eb : 0.0;
    }

#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int g = g0 + i;
        if (g >= r0 && g < r1 && lane_owned) {
            const size_t off = (size_t)g * ld + cb;
            uout[off] = u[i];
            dout[off] = d[i];
        }
    }

    if (want_energy) {
        // wave sums by DPP within rows of 16 lanes (pairs, quads, half rows, rows), then the four
        // row sums read from lanes 0, 16, 32, 48: a few cycles per exchange where a general lane
        // permutation waits on the LDS crossbar
#pragma unroll
        for (int t = 0; t < kMaxTimeBlock; ++t) {
            double v = acc[t];
            v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
            v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
            v += dpp_f64<0x141>(v);  // row_half_mirror
            v += dpp_f64<0x140>(v);  // row_mirror
            acc[t] = (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
        }
        if (lane == 0) {
#pragma unroll
            for (int t = 0; t < kMaxTimeBlock; ++t) s_e[t][w] = acc[t];
        }
        __syncthreads();
        if (w == 0 && lane < K) {
            double s = 0.0;
            for (int v = 0; v < NW; ++v) s += s_e[lane][v];
            M.epart[((size_t)a.eslot * kMaxTimeBlock + lane) * M.epart_stride + tile] = s;
        }
    }
}

template <typename T, int FACE>
hipError_t launch_tile_f(const StepArgs& a, int K, int waves, int grid, hipStream_t s)
{
    const dim3 g(grid), b(kWaveSize * waves);
    if (a.want_energy)
        hipLaunchKernelGGL((k_step_tile<T, FACE, 1>), g, b, 0, s, a, K);
    else
        hipLaunchKernelGGL((k_step_tile<T, FACE, 0>), g, b, 0, s, a, K);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_step_tile(const StepArgs& a, int K, int face_mode, int waves, int grid, hipStream_t s)
{
    if (K < 1 || K > kMaxTimeBlock || waves < 1 || waves > kMaxTileWaves || a.want_trace) return hipErrorInvalidValue;
    return face_mode == 1 ? launch_tile_f<T, 1>(a, K, waves, grid, s) : launch_tile_f<T, 0>(a, K, waves, grid, s);
}
template hipError_t launch_step_tile<float>(const StepArgs&, int, int, int, int, hipStream_t);
template hipError_t launch_step_tile<double>(const StepArgs&, int, int, int, int, hipStream_t);

}  // namespace fdw
