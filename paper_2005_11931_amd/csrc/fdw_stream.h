// fdw_stream.h - the streaming, temporally blocked leapfrog kernel (device code), included
// by one instantiation unit per (storage type, columns per lane) so that the variants build
// in parallel.  See fdw_kernels.hip for the overview of the method and its citations.
#pragma once

#include "fdw_internal.h"

#include <hip/hip_runtime.h>

namespace fdw {

// ------------------------------------------------------------------------------------------
// Lane exchange across the whole wave (DPP wave shift by one lane; lanes with no source get 0
// through the bound control bit, so no register has to be cleared first)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_from_left_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);  // lane l <- lane l-1
}
__device__ __forceinline__ int lane_from_right_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);  // lane l <- lane l+1
}
__device__ __forceinline__ float lane_from_left(float v)
{
    return __builtin_bit_cast(float, lane_from_left_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_from_right(float v)
{
    return __builtin_bit_cast(float, lane_from_right_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_from_left(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = lane_from_left_i((int)(b & 0xffffffffLL));
    int hi = lane_from_left_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = lane_from_right_i((int)(b & 0xffffffffLL));
    int hi = lane_from_right_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------------------------------
// The point update, shared by every kernel that advances the state.
//   f* are face sums (2x the face coefficient: h_c + h_neighbour), ax = tau^2/(2 dx^2).
// Opposite faces are added as commutative pairs so that mirror-symmetric data stay
// mirror-symmetric bit for bit.  The file is compiled without contraction; the one fused
// multiply-add is explicit.
// ------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T flux_L(T uc, T ue, T uw, T un, T us, T fxe, T fxw, T fyn, T fys, T ax, T ay)
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
__device__ __forceinline__ float flux_L<float>(float uc, float ue, float uw, float un, float us, float fxe, float fxw,
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

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int C>
struct alignas(sizeof(T) * C) Pack {
    T v[C];
};

template <typename T, int C>
__device__ __forceinline__ void load_pack(const T* __restrict__ p, T (&out)[C])
{
    Pack<T, C> q = *reinterpret_cast<const Pack<T, C>*>(p);
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = q.v[c];
}
template <typename T, int C>
__device__ __forceinline__ void store_pack(T* __restrict__ p, const T (&in)[C])
{
    Pack<T, C> q;
#pragma unroll
    for (int c = 0; c < C; ++c) q.v[c] = in[c];
    *reinterpret_cast<Pack<T, C>*>(p) = q;
}

template <typename T>
struct Lanes;  // columns per lane: one 16-byte vector
template <>
struct Lanes<float> {
    static constexpr int C = 4;
};
template <>
struct Lanes<double> {
    static constexpr int C = 2;
};

// Pointer into the constant address space, for tables a kernel only reads (receiver lists):
// wave-uniform loads through it become scalar loads, which complete on their own counter
// instead of waiting behind the outstanding vector loads of the row prefetch.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;
// Pointer into the global address space: stores through it are global (not flat) stores.
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T*;

// Index of the calling wave in its workgroup, as a wave-uniform (scalar) value.  Written as
// threadIdx.x / 64 it is a per-lane value to the compiler, and everything derived from it
// (work item, row range, buffer descriptors) would live in vector registers, with every
// buffer load wrapped in a loop over the distinct descriptors of the lanes.
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Wave-uniform copies of a pointer and of a 64-bit integer (scalar registers).
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
    return (P*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int64_t uniform_i64(int64_t x)
{
    const unsigned long long v = (unsigned long long)x;
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
    return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Receiver lists are sorted by (row, column): the first entry of col[lo, hi) whose column is
// at least x, by bisection over wave-uniform (scalar) loads.  Used to cut a row's receivers down
// to the columns of one strip.
__device__ __forceinline__ int lower_bound_col(ConstPtr<int> col, int lo, int hi, int x)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); give each
    // XCD a contiguous range of logical blocks so that neighbouring strips share an L2.
    int xcd = b & 7, per = nb >> 3, rem = nb & 7;
    return xcd * per + min(xcd, rem) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------------------------------
// One streaming work item: member M, strip, segment; K time levels; C columns per lane.
//
// The work item streams its rows in one direction (down for even segments, up for odd ones);
// at stream position p, level t (t = 1..K) computes the row at position p - t from level
// t-1's rows at positions p - t and p - t + 1 (u) and p - t (du).  Below, the rows are
// written as for the downward direction.  The x part of the operator is written with one flux per face,
// F_c = fx_{c+1/2} (u_{c+1} - u_c), and the y part with the flux G_r = fy_{r+1/2}
// (u_{r+1} - u_r) carried over from the previous row: sx = F_c - F_{c-1}, sy = G_r - G_{r-1}.
// Since fx_{c-1/2}(u_{c-1} - u_c) = -F_{c-1} exactly, this is bit-identical to summing the
// two opposite-face terms of every node.  Rings are indexed by the position modulo 2 and K, and the
// loaded input rows by the position modulo NB; the row loop is unrolled by lcm(2, K, NB) so that
// every ring index is a compile-time constant.  Input rows are loaded NB - 1 rows ahead of
// their use: one row of loads per wave in flight is far too little to cover the HBM latency
// at the occupancy these register footprints allow.
// ------------------------------------------------------------------------------------------
template <int K>
struct RowUnroll {
    static constexpr int NB = (K % 2 == 0) ? 4 : 2;  // row buffers (odd K: keep the unroll at 2K)
    static constexpr int U = (K % 2 == 0) ? ((K % 4 == 0) ? K : 2 * K) : 2 * K;
};
__host__ __device__ constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

// compile-time flag passed to generic lambdas (selects a specialised copy of a loop body)
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

// Row loads go through buffer resources: an offset at or beyond the resource's size returns
// zeros in hardware, so rows above/below the grid and lanes outside the plane need no branch
// (a load under a divergent branch would force the prefetch to be waited on at once).
typedef unsigned int fdw_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int fdw_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int fdw_u32x8 __attribute__((ext_vector_type(8)));
constexpr unsigned int kBufferOutOfRange = 0x80000000u;  // offsets >= 2^31 are never valid
constexpr int kBufferWord3 = 0x00020000;                // raw (untyped) buffer access, GFX9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
}

// Loads the whole C-element vector; every element is consumed by the caller.  AUX: cache
// policy bits of the load (2 = non-temporal).
template <typename T, int C, int AUX = 0>
__device__ __forceinline__ void buffer_row(__amdgpu_buffer_rsrc_t r, unsigned int off, T (&out)[C])
{
    static_assert(sizeof(T) * C == 32 || sizeof(T) * C == 16 || sizeof(T) * C == 8, "8/16/32-byte lane vectors");
    Pack<T, C> q;
    if constexpr (sizeof(T) * C == 32) {
        const fdw_u32x4 v0 = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AUX);
        const fdw_u32x4 v1 = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(off + 16u), 0, AUX);
        const fdw_u32x8 v = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
        q = __builtin_bit_cast(Pack<T, C>, v);
    } else if constexpr (sizeof(T) * C == 16) {
        const fdw_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AUX);
        q = __builtin_bit_cast(Pack<T, C>, v);
    } else {
        const fdw_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX);
        q = __builtin_bit_cast(Pack<T, C>, v);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = q.v[c];
}

// Non-temporal row stores, for working sets larger than the caches: the next launch reads the
// rows back from HBM anyway, and keeping them out of L2 leaves room for the halo rows that
// neighbouring work items share.
template <typename T, int C>
__device__ __forceinline__ void store_row_nt(T* __restrict__ p, const T (&in)[C])
{
    constexpr int B = (int)sizeof(T) * C;
    static_assert(B == 8 || B == 16 || B == 32, "8-, 16- or 32-byte rows per lane");
    Pack<T, C> q;
#pragma unroll
    for (int c = 0; c < C; ++c) q.v[c] = in[c];
    if constexpr (B == 8) {
        __builtin_nontemporal_store(__builtin_bit_cast(fdw_u32x2, q), reinterpret_cast<fdw_u32x2*>(p));
    } else if constexpr (B == 16) {
        __builtin_nontemporal_store(__builtin_bit_cast(fdw_u32x4, q), reinterpret_cast<fdw_u32x4*>(p));
    } else {
        const fdw_u32x8 v = __builtin_bit_cast(fdw_u32x8, q);
        const fdw_u32x4 lo = {v[0], v[1], v[2], v[3]}, hi = {v[4], v[5], v[6], v[7]};
        __builtin_nontemporal_store(lo, reinterpret_cast<fdw_u32x4*>(p));
        __builtin_nontemporal_store(hi, reinterpret_cast<fdw_u32x4*>(p) + 1);
    }
}

// MODE bit 0: per-step energy partials; bit 1: receiver traces; bit 2: non-temporal loads of
// the state rows (FP32 launches whose working set exceeds the last-level cache).
template <typename T, int K, int C, int FACE, int MODE>
__device__ __forceinline__ void sweep_item(const MemberDev& M, int wave, int parity, int64_t ctx_step, int eslot = 0)
{
    constexpr bool want_energy = (MODE & 1) != 0;
    constexpr bool want_trace = (MODE & 2) != 0;
    constexpr bool nt_loads = (MODE & 4) != 0;
    constexpr int Hx = ((K + C - 1) / C) * C;   // halo columns on each side (multiple of C)
    constexpr int Wv = kWaveSize * C - 2 * Hx;  // owned columns per strip
    constexpr int U = RowUnroll<K>::U;
    constexpr int NB = RowUnroll<K>::NB;
    static_assert(U % NB == 0 && U % K == 0 && U % 2 == 0, "row unroll");
    const int lane = threadIdx.x & 63;

    const int nx = M.nx, ny = M.ny, ld = M.ld;
    const int strip = wave % M.strips;
    const int seg = wave / M.strips;
    const int cb = strip * Wv - Hx + lane * C;
    const bool lane_live = (cb >= 0) && (cb < ld);
    const bool lane_owned = lane_live && (lane * C >= Hx) && (lane * C < Hx + Wv);
    T colm[C];  // 1 on interior columns, 0 on the boundary ring / padding
#pragma unroll
    for (int c = 0; c < C; ++c) colm[c] = ((cb + c >= 1) && (cb + c <= nx - 2)) ? T(1) : T(0);

    const int r0 = seg * M.seg_rows;
    const int r1 = min(r0 + M.seg_rows, ny);
    const int cur = M.cur0 ^ parity;
    const T* __restrict__ uin = (const T*)M.u[cur];
    const T* __restrict__ din = (const T*)M.d[cur];
    T* __restrict__ uout = (T*)M.u[cur ^ 1];
    T* __restrict__ dout = (T*)M.d[cur ^ 1];
    const T* __restrict__ hp = (const T*)M.h;
    const T* __restrict__ hyp = (const T*)M.hy;
    const T ax = (T)M.ax, ay = (T)M.ay;
    const int64_t n0 = ctx_step + M.n_offset;

    // Even segments stream downwards (rows r0-K .. r1+K-1), odd ones upwards (r1+K-1 ..
    // r0-K): two neighbouring segments then pass over the 2K rows both of them read at about
    // the same time - both at their start or both at their end - so that the second read of
    // those rows usually hits L2.  Position p of the stream is row rfirst + dir * p.  The
    // result does not depend on the direction, bit for bit (see the y-flux below).
    const int dir = (seg & 1) ? -1 : 1;
    const int rfirst = (dir > 0) ? r0 - K : r1 + K - 1;
    // buffer resources starting at the lowest streamed row inside the grid
    const int jbase = max(r0 - K, 0);
    const size_t base_el = (size_t)jbase * ld;
    const size_t span = (size_t)(ny - jbase) * ld * sizeof(T);
    const unsigned int nbytes = __builtin_amdgcn_readfirstlane((unsigned int)min(span, (size_t)kBufferOutOfRange - 16));
    // the descriptors are wave-uniform: build them from values the compiler knows to be uniform
    // (otherwise, where it cannot prove it - inside the persistent kernel's item loop - every
    // buffer load is wrapped in a loop over the distinct descriptors of the wave)
    const __amdgpu_buffer_rsrc_t ru = plane_rsrc(uniform_ptr(uin + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rd = plane_rsrc(uniform_ptr(din + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rh = plane_rsrc(uniform_ptr(hp + base_el), nbytes);
    const __amdgpu_buffer_rsrc_t rhy = plane_rsrc(uniform_ptr((FACE ? hyp : hp) + base_el), nbytes);
    const unsigned int row_bytes = (unsigned int)(ld * (int)sizeof(T));
    const unsigned int lane_col = lane_live ? (unsigned int)(cb * (int)sizeof(T)) : kBufferOutOfRange;

    // (rings are indexed by stream position p, "row p" meaning the row at position p)
    T Ur[K][2][C];  // level t at rows of stream parity 0/1
    T Dr[K][2][C];
    T Gy[K][C];     // Gy[t-1]: y-flux of level t-1 across the face before the row level t computes next
    T FXr[K][C];    // x-face sums of the rows p-K .. p-1 (by position modulo K)
    T FYr[K][C];    // y-face sums between those rows and the next one in the stream
    T hprev[C];     // coefficient row p-1 (nodal h, or the x-face row in the face layout)
    T hyprev[C];    // face layout: y-face row p-1
    T bu[NB][C], bd[NB][C], bh[NB][C], bhy[NB][C];  // loaded rows p .. p+NB-1 (by position modulo NB)
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            Ur[t][0][c] = Ur[t][1][c] = T(0);
            Dr[t][0][c] = Dr[t][1][c] = T(0);
            Gy[t][c] = T(0);
            FXr[t][c] = FYr[t][c] = T(0);
        }
        hprev[c] = hyprev[c] = T(0);
#pragma unroll
        for (int q = 0; q < NB; ++q) bu[q][c] = bd[q][c] = bh[q][c] = bhy[q][c] = T(0);
    }
    double acc[K];
#pragma unroll
    for (int t = 0; t < K; ++t) acc[t] = 0.0;

    // receiver tables (trace mode): read as constant memory, so that their wave-uniform lookups
    // are scalar loads; items whose own rows hold no receiver skip the trace code entirely
    const ConstPtr<int> rowptr = (ConstPtr<int>)M.rec_rowptr;
    const ConstPtr<int> rcol = (ConstPtr<int>)M.rec_col;
    const ConstPtr<int> rid = (ConstPtr<int>)M.rec_id;
    const bool item_rec = want_trace && (rowptr[r0] < rowptr[r1]);
    const int own_lo = strip * Wv;  // first owned column of the strip
    // trace output, read once into scalar registers: loaded where it is used, these would be
    // vector loads waited for on the spot, and that wait drains every outstanding row load.
    // The pointer is declared global: a generic (flat) store also counts as an LDS access, so
    // the next LDS or scalar-load wait would wait for the store to reach memory.
    GlobalPtr<T> const trace_out = want_trace ? (GlobalPtr<T>)uniform_ptr((T*)M.traces) : nullptr;
    const int trace_R = want_trace ? __builtin_amdgcn_readfirstlane(M.R) : 0;
    const int64_t trace_rows = want_trace ? uniform_i64(M.trace_rows) : 0;
    int RPb[K], RPe[K];  // receiver ranges of the rows in flight (by position modulo K)
#pragma unroll
    for (int t = 0; t < K; ++t) RPb[t] = RPe[t] = 0;
    // Receiver of each lane column in the rows in flight (by position modulo K; -1: none), in a
    // wave-private slice of LDS.  The level loop then records a trace with one store per lane
    // and no loop: a loop around vector stores would make the compiler wait for every
    // outstanding row load before each level.  Coincident receivers keep the first of their
    // run here; the library copies the others' columns after the call.
    constexpr int kSlotRows = want_trace ? K : 1;
    constexpr int kSlotCols = want_trace ? kWaveSize * C : 1;
    __shared__ int s_slot[kWavesPerBlock][kSlotRows][kSlotCols];
    const int wib = wave_in_block();
    if (want_trace && item_rec) {
#pragma unroll
        for (int t = 0; t < K; ++t)
#pragma unroll
            for (int c = 0; c < C; ++c) s_slot[wib][t][lane * C + c] = -1;
    }
    // Items of up to 128 rows look their receivers up once, here, with vector loads issued
    // before the row stream starts (their waits then do not wait for row loads): a bit mask of
    // the item's rows that hold receivers (wave-uniform, two words), and the slots of the first
    // kPreRows such rows in LDS.  The level loop then tests a bit for every row entering level 1
    // and copies a row's slots from LDS, instead of searching the receiver tables (a chain of
    // dependent scalar loads per row); rows past the kPreRows-th receiver row, and longer
    // items, still search.
    constexpr int kPreRows = 4;
    __shared__ int s_pre[kWavesPerBlock][want_trace ? kPreRows : 1][kSlotCols];
    uint64_t rmask0 = 0, rmask1 = 0;
    int rrank1 = 0;
    const bool pre_item = want_trace && item_rec && (r1 - r0 <= 2 * kWaveSize);
    if (pre_item) {
        int found = 0;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int r = r0 + w * kWaveSize + lane;
            const int rq = min(r, r1 - 1);  // in range for every lane (no branch around the loads)
            const bool has = (r < r1) && (rowptr[rq] < rowptr[rq + 1]);
            uint64_t m = __ballot(has);
            if (w == 0) {
                rmask0 = m;
                rrank1 = __popcll(m);
            } else {
                rmask1 = m;
            }
            while (m != 0 && found < kPreRows) {
                const int rr = r0 + w * kWaveSize + (int)__builtin_ctzll(m);
                m &= m - 1;
                int* const pre = s_pre[wib][found];
#pragma unroll
                for (int c = 0; c < C; ++c) pre[lane * C + c] = -1;
                // this row's receivers in the strip's owned columns, first of each run of
                // coincident ones (every lane takes one receiver of the row's range)
                const int kb = rowptr[rr], ke = rowptr[rr + 1];
                for (int k0 = kb; k0 < ke; k0 += kWaveSize) {
                    const int k = min(k0 + lane, ke - 1);
                    const int col = rcol[k];
                    const int prev = (k > kb) ? rcol[k - 1] : -1;
                    const int id = rid[k];
                    if (k0 + lane < ke && col >= own_lo && col < own_lo + Wv && (k == kb || prev != col))
                        pre[col - own_lo + Hx] = id;
                }
                ++found;
            }
        }
    }

    // r1 - r0 + 2K rows are streamed (rounded up to whole unrolled blocks; rows outside the
    // grid load as zeros and are never stored).
    const int nblk = (r1 - r0 + 2 * K + U - 1) / U;
    const size_t lane_off = (size_t)(ptrdiff_t)cb;
    // Working sets above the last-level cache are streamed: outputs with non-temporal stores,
    // and in FP32 the state rows with non-temporal loads (MODE bit 2: measured faster there,
    // slower in FP64).  Sets that fit keep normal accesses, so that the next launch finds them
    // cached.
    const bool nt = M.stream_nt != 0;
    constexpr int kStatePolicy = nt_loads ? 2 : 0;
    auto load_row = [&](int p, T (&u)[C], T (&d)[C], T (&h)[C], T (&hy)[C]) {
        const int j = rfirst + dir * p;
        const unsigned int off = (j < jbase) ? kBufferOutOfRange : (unsigned int)(j - jbase) * row_bytes + lane_col;
        buffer_row<T, C, kStatePolicy>(ru, off, u);
        buffer_row<T, C, kStatePolicy>(rd, off, d);
        buffer_row<T, C>(rh, off, h);
        if (FACE) buffer_row<T, C>(rhy, off, hy);
    };
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) load_row(q, bu[q], bd[q], bh[q], bhy[q]);

    {
        for (int blk = 0; blk < nblk; ++blk) {
            T eb[K];
#pragma unroll
            for (int t = 0; t < K; ++t) eb[t] = T(0);
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int p = blk * U + s;  // stream position of the row loaded last
                const int pb = s % NB;      // buffer holding row p
                // prefetch row p+NB-1 into the buffer row p-1 used
                {
                    const int pn = (s + NB - 1) % NB;
                    load_row(p + NB - 1, bu[pn], bd[pn], bh[pn], bhy[pn]);
                }

                // ---- coefficient faces of row p-1 into the ring (index (p-1) mod K), scaled
                // by tau^2/(2 dx^2) and tau^2/(2 dy^2) once per row, so that every level's
                // operator is the plain sum of its x and y flux differences; the y face between
                // rows p-1 and p is stored with the upper of the two grid rows
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
                // ---- level 0: row p of the input state
                {
                    const int p0 = pmod(s, 2);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        Ur[0][p0][c] = bu[pb][c];
                        Dr[0][p0][c] = bd[pb][c];
                    }
                }
                // ---- levels 1..K
#pragma unroll
                for (int t = 1; t <= K; ++t) {
                    const int r = rfirst + dir * (p - t);  // grid row of stream position p - t
                    const int pr = pmod(s - t, 2);         // parity index of row r
                    const int pr1 = pmod(s - t + 1, 2);    // ... of the next row in the stream, r + dir
                    const int q = pmod(s - t, K);          // coefficient ring index of row r
                    const bool rin = (r >= 1) && (r <= ny - 2);
                    const bool rown = (r >= r0) && (r < r1);
                    const T right = lane_from_right(Ur[t - 1][pr][0]);
                    T F[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const T ue = (c < C - 1) ? Ur[t - 1][pr][c + 1] : right;
                        F[c] = FXr[q][c] * (ue - Ur[t - 1][pr][c]);
                    }
                    const T Fl = lane_from_left(F[C - 1]);
                    T nu[C], nd[C], L[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        // Gn = fy (u_{r+dir} - u_r): downwards this is F_{r+1/2}, upwards it is
                        // -F_{r-1/2} exactly (negation is exact), and Gy holds the previous
                        // row's Gn; so Gn - Gy is F_{r+1/2} - F_{r-1/2} bit for bit in both
                        // directions
                        const T Gn = FYr[q][c] * (Ur[t - 1][pr1][c] - Ur[t - 1][pr][c]);
                        const T sx = F[c] - ((c > 0) ? F[c - 1] : Fl);
                        const T sy = Gn - Gy[t - 1][c];
                        Gy[t - 1][c] = Gn;
                        L[c] = sx + sy;
                    }
                    // Dirichlet rows keep du = 0 (and with it u = 0, which they hold at every
                    // level); the row test is wave-uniform, and the empty asm keeps it a scalar
                    // branch instead of a select per value
#pragma unroll
                    for (int c = 0; c < C; ++c) nd[c] = fma_t(L[c], colm[c], Dr[t - 1][pr][c]);
                    if (__builtin_expect(!rin, 0)) {
#pragma unroll
                        for (int c = 0; c < C; ++c) nd[c] = T(0);
                        asm volatile("");
                    }
#pragma unroll
                    for (int c = 0; c < C; ++c) nu[c] = Ur[t - 1][pr][c] + nd[c];
                    if (want_energy && rown) {
                        // per-node terms du^2 - u L in the storage type, summed over the lane's
                        // columns and the rows of this unrolled block; FP64 across blocks
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            eb[t - 1] = fma_t(nd[c], nd[c], eb[t - 1]);
                            eb[t - 1] = fma_t(-nu[c], L[c], eb[t - 1]);
                        }
                        // an empty asm that reads and writes the partial sum pins the
                        // accumulation here: otherwise the compiler defers the energy
                        // arithmetic of the whole unrolled block to its end, keeping every
                        // level's nu, nd and L of every row alive (several hundred registers
                        // at K >= 3)
                        asm volatile("" : "+v"(eb[t - 1]));
                    }
                    if (want_trace && __builtin_expect(item_rec, 0)) {
                        // receivers of row r in this strip's owned columns, looked up once when
                        // the row enters level 1 (none for rows the item does not own or that lie
                        // on the boundary), and entered in the row's slots
                        if (t == 1) {
                            int kb = 0, ke = 0;
                            bool search = rown && rin;
                            if (pre_item && search) {
                                // the item's row mask: no receivers, or slots looked up already
                                const int ri = r - r0;
                                const uint64_t m = (ri < kWaveSize) ? rmask0 : rmask1;
                                const int b = ri & (kWaveSize - 1);
                                search = false;
                                if ((m >> b) & 1) {
                                    const int j = ((ri < kWaveSize) ? 0 : rrank1) + __popcll(m & ((uint64_t(1) << b) - 1));
                                    if (j < kPreRows) {
#pragma unroll
                                        for (int c = 0; c < C; ++c) s_slot[wib][q][lane * C + c] = s_pre[wib][j][lane * C + c];
                                        kb = 0;
                                        ke = 1;
                                    } else {
                                        search = true;
                                    }
                                }
                            }
                            if (search) {
                                kb = rowptr[r];
                                ke = rowptr[r + 1];
                                if (kb < ke) {
                                    kb = lower_bound_col(rcol, kb, ke, own_lo);
                                    ke = lower_bound_col(rcol, kb, ke, own_lo + Wv);
                                }
                                for (int k = kb; k < ke; ++k) {
                                    const int col = rcol[k];
                                    if ((k == kb || rcol[k - 1] != col) && lane == 0) s_slot[wib][q][col - own_lo + Hx] = rid[k];
                                }
                            }
                            RPb[q] = kb;
                            RPe[q] = ke;
                        }
                        if (RPb[q] < RPe[q]) {
                            const int64_t row = n0 + t;
#pragma unroll
                            for (int c = 0; c < C; ++c) {
                                const int id = s_slot[wib][q][lane * C + c];
                                if (id >= 0 && row < trace_rows) trace_out[row * trace_R + id] = nu[c];
                                if (t == K) s_slot[wib][q][lane * C + c] = -1;
                            }
                        }
                    }
                    if (t < K) {
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            Ur[t][pr][c] = nu[c];
                            Dr[t][pr][c] = nd[c];
                        }
                    } else if (rown && lane_owned) {
                        const size_t off = (size_t)(ptrdiff_t)r * ld + lane_off;
                        if (nt) {
                            store_row_nt<T, C>(uout + off, nu);
                            store_row_nt<T, C>(dout + off, nd);
                        } else {
                            store_pack<T, C>(uout + off, nu);
                            store_pack<T, C>(dout + off, nd);
                        }
                    }
                }
                // keep the scheduler from interleaving consecutive rows (bounds register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            if (want_energy && lane_owned) {
#pragma unroll
                for (int t = 0; t < K; ++t) acc[t] += (double)eb[t];
            }
        }
    }

    if (want_energy) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double sum = wave_sum(acc[t]);
            // every lane stores the same sum (the butterfly leaves it in all lanes): no lane-0
            // branch, which inside the persistent kernel's item loop could be moved out of the
            // loop for lane 0 alone
            M.epart[((size_t)eslot * kMaxTimeBlock + t) * M.epart_stride + wave] = sum;
        }
    }
}

__device__ __forceinline__ int find_member(const MemberDev* table, int first, int nmembers, int gb)
{
    int m = first;
    for (int k = first + 1; k < first + nmembers; ++k)
        if (table[k].block_base <= gb) m = k;
    return m;
}

// The double trace-recording variant (one column per lane, nodal coefficients) is held to four
// waves per SIMD (128 registers, a few values spilled): its 135 registers otherwise leave three,
// and the traced forward run of a gradient evaluation measured 5% faster with four.
template <typename T, int K, int C, int FACE, int MODE>
__global__ __launch_bounds__(kWaveSize * kWavesPerBlock, (sizeof(T) == 8 && C == 1 && FACE == 0 && MODE == 2) ? 4 : 1) void k_step(StepArgs a)
{
    int lb = xcd_remap(blockIdx.x, a.total_blocks);
    if (a.reverse) lb = a.total_blocks - 1 - lb;
    const int gb = lb + a.block_offset;
    const int m = find_member(a.table, a.first, a.nmembers, gb);
    const MemberDev& M = a.table[m];
    const int wave = (gb - M.block_base) * kWavesPerBlock + wave_in_block();
    if (wave >= M.waves) return;
    sweep_item<T, K, C, FACE, MODE>(M, wave, a.parity, a.ctx_step, a.eslot);
}

template <typename T, int K, int C, int FACE>
static hipError_t launch_step_kcf(const StepArgs& a, int grid, hipStream_t s)
{
    const dim3 g(grid), b(kWaveSize * kWavesPerBlock);
    const int mode = (a.want_energy ? 1 : 0) | (a.want_trace ? 2 : 0);
    if constexpr (sizeof(T) == 4) {
        if (a.stream_nt) {
            switch (mode) {
            case 3: hipLaunchKernelGGL((k_step<T, K, C, FACE, 7>), g, b, 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_step<T, K, C, FACE, 5>), g, b, 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_step<T, K, C, FACE, 6>), g, b, 0, s, a); break;
            default: hipLaunchKernelGGL((k_step<T, K, C, FACE, 4>), g, b, 0, s, a); break;
            }
            return hipGetLastError();
        }
    }
    switch (mode) {
    case 3: hipLaunchKernelGGL((k_step<T, K, C, FACE, 3>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_step<T, K, C, FACE, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_step<T, K, C, FACE, 2>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_step<T, K, C, FACE, 0>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}

template <typename T, int K, int C>
static hipError_t launch_step_kc(const StepArgs& a, int face_mode, int grid, hipStream_t s)
{
    return face_mode == 1 ? launch_step_kcf<T, K, C, 1>(a, grid, s) : launch_step_kcf<T, K, C, 0>(a, grid, s);
}

// K = 1..KMAX of one (T, C) configuration
template <typename T, int C, int KMAX>
static hipError_t launch_step_c(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s)
{
    switch (K) {
    case 1: return launch_step_kc<T, 1, C>(a, face_mode, grid, s);
    case 2: return launch_step_kc<T, 2, C>(a, face_mode, grid, s);
    case 3: return launch_step_kc<T, 3, C>(a, face_mode, grid, s);
    case 4: return launch_step_kc<T, 4, C>(a, face_mode, grid, s);
    case 5: return KMAX >= 5 ? launch_step_kc<T, (KMAX >= 5 ? 5 : 1), C>(a, face_mode, grid, s) : hipErrorInvalidValue;
    case 6: return KMAX >= 6 ? launch_step_kc<T, (KMAX >= 6 ? 6 : 1), C>(a, face_mode, grid, s) : hipErrorInvalidValue;
    case 7: return KMAX >= 7 ? launch_step_kc<T, (KMAX >= 7 ? 7 : 1), C>(a, face_mode, grid, s) : hipErrorInvalidValue;
    case 8: return KMAX >= 8 ? launch_step_kc<T, (KMAX >= 8 ? 8 : 1), C>(a, face_mode, grid, s) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------------------------------
// Persistent batched variant: one cooperative launch runs `phases` time blocks of K steps over
// all members, with a grid-wide barrier between time blocks.  The barrier spin is bounded: on
// expiry it records an error flag and lets the wave continue, so a launch always drains.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void grid_barrier(int* bar, int nblocks, int& gen, int* err)
{
    // The block's stores reach its L2 by the workgroup barrier; one agent-scope release by
    // the arriving thread then writes that L2 back for the other XCDs (the L2 write-back and
    // invalidate act on the whole cache, so one per block is enough) ...
    // The counter operations themselves are relaxed: an acquire on every poll would invalidate
    // the XCD's L2 under the blocks still computing the time block; the fences around them give
    // the ordering (a release fence before the arrival, one acquire fence after the wait).
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int arrived = __hip_atomic_fetch_add(&bar[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1L << 26)) {
                    // the wait is bounded: record the timeout in the caller's error word (the host
                    // reads it after the call) and carry on, so that the launch always drains
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
    }
    // ... and its acquire invalidates this CU's L1 and the XCD's L2 before any wave of the
    // block reads the other blocks' results
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    gen += 1;
    __syncthreads();
}

// Energy of one (member, level) of a finished time block, summed by one wave in a fixed order
// (lane l takes the partials l, l + 64, ... in turn, then a butterfly whose two operands are the
// same in both lanes of a pair, so every lane ends with the same sum): the in-kernel counterpart
// of k_energy_finalize, with the same failure-detection bits.  Every lane stores that same
// value: a store under `lane == 0` inside the caller's loop let the compiler move lane 0 out of
// the loop on its own, leaving the other lanes of the wave looping.
__device__ __forceinline__ void finalize_energy_wave(const MemberDev& M, int t, int slot, int64_t row_off,
                                                     const PersistentExtra& x, bool growth_ok)
{
    const int lane = threadIdx.x & 63;
    const double* p = M.epart + ((size_t)slot * kMaxTimeBlock + t) * M.epart_stride;
    double acc = 0.0;
    for (int w = lane; w < M.waves; w += kWaveSize) acc += p[w];
    const double E = wave_sum(acc) * M.escale;
    x.energy_base[(int64_t)M.energy_row * x.energy_stride + row_off + t] = E;
    int bits = isfinite(E) ? 0 : 1;
    if (growth_ok && fabs(E) > 10.0 * fabs(x.energy_base[(int64_t)M.energy_row * x.energy_stride])) bits |= 2;
    if (bits) atomicOr(x.health, bits);
}

// MODE 0: plain steps; MODE 1: with the per-step energy.  In energy mode the time blocks write
// their per-wave partials into two alternating slots, and the partials of time block p - 1 are
// summed at the start of time block p (one wave per (member, level), handed out before the
// stencil items); the last block's partials are summed by the host's k_energy_finalize.
template <typename T, int K, int C, int FACE, int MODE>
__global__ __launch_bounds__(kWaveSize * kWavesPerBlock) void k_step_persistent(StepArgs a, int phases, int* bar,
                                                                                PersistentExtra x)
{
    const int total_waves = a.total_blocks * kWavesPerBlock;  // work items of one time block
    // Workgroups land on the 8 XCDs round-robin (block b on XCD b mod 8).  Each XCD takes a
    // contiguous eighth of the work items, so that neighbouring strips and segments (which
    // share halo rows and columns) go through the same L2; within it, waves take items one at
    // a time from a per-(time block, XCD) counter, which balances uneven items.  With fewer
    // than 8 blocks there is one range and one counter.
    const bool by_xcd = gridDim.x >= 8;
    const int xcd = by_xcd ? (int)(blockIdx.x & 7) : 0;
    const int lo = by_xcd ? (int)((int64_t)total_waves * xcd / 8) : 0;
    const int hi = by_xcd ? (int)((int64_t)total_waves * (xcd + 1) / 8) : total_waves;
    const int lane = threadIdx.x & 63;
    int* const counters = bar + 16;  // [phases][8] stencil items
    const int nfin = (MODE & 1) ? a.nmembers * K : 0;
    const int gwave = (int)blockIdx.x * kWavesPerBlock + wave_in_block();
    const int nwaves = (int)gridDim.x * kWavesPerBlock;
    int gen = 0;
    int parity = a.parity;
    int64_t step = a.ctx_step;
    for (int p = 0; p < phases; ++p) {
        if ((MODE & 1) && p > 0) {
            // energies of time block p - 1 (its partials are complete: a grid barrier separates
            // them), one (member, level) per wave of the grid in turn: a loop with a wave-uniform
            // (scalar) trip count
            const int64_t q = p - 1;
            for (int k = gwave; k < nfin; k += nwaves) {
                const int m = a.first + k / K;
                finalize_energy_wave(a.table[m], k % K, (int)(q & 1), x.energy_offset + q * K, x,
                                     x.energy_offset > 0 || q >= 2);
            }
        }
        for (;;) {
            int k = 0;
            if (lane == 0) k = __hip_atomic_fetch_add(&counters[8 * p + xcd], 1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            // lane 0's ticket, read from lane 0 whatever the active lanes
            const int item = lo + __builtin_amdgcn_readlane(k, 0);
            if (item >= hi) break;
            const int gb = item / kWavesPerBlock + a.block_offset;
            const int m = find_member(a.table, a.first, a.nmembers, gb);
            const MemberDev& M = a.table[m];
            const int wave = (gb - M.block_base) * kWavesPerBlock + (item % kWavesPerBlock);
            if (wave < M.waves) sweep_item<T, K, C, FACE, MODE>(M, wave, parity, step, p & 1);
        }
        parity ^= 1;
        step += K;
        if (p + 1 < phases) grid_barrier(bar, gridDim.x, gen, x.err);
    }
}

template <typename T, int K, int C>
static hipError_t launch_persistent_kc(const StepArgs& a, int face_mode, int phases, int grid, int* bar,
                                       const PersistentExtra& x, hipStream_t s)
{
    void* args[] = {(void*)&a, (void*)&phases, (void*)&bar, (void*)&x};
    const dim3 g(grid), b(kWaveSize * kWavesPerBlock);
    const bool e = a.want_energy != 0;
    const void* f = face_mode == 1 ? (e ? (const void*)k_step_persistent<T, K, C, 1, 1> : (const void*)k_step_persistent<T, K, C, 1, 0>)
                                   : (e ? (const void*)k_step_persistent<T, K, C, 0, 1> : (const void*)k_step_persistent<T, K, C, 0, 0>);
    return hipLaunchCooperativeKernel(f, g, b, args, 0, s);
}

template <typename T, int K, int C>
static int persistent_blocks_kc(int face_mode, bool energy)
{
    int per_cu = 0;
    const int bs = kWaveSize * kWavesPerBlock;
    // the grid is sized for the variant that runs: every one of its blocks must be resident
    // (a grid sized for the energy variant, which holds more registers, left the plain one at
    // its occupancy)
    const void* f = face_mode ? (energy ? (const void*)k_step_persistent<T, K, C, 1, 1> : (const void*)k_step_persistent<T, K, C, 1, 0>)
                              : (energy ? (const void*)k_step_persistent<T, K, C, 0, 1> : (const void*)k_step_persistent<T, K, C, 0, 0>);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, bs, 0);
    if (e != hipSuccess) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

// time blocks 1, 2, 4 and (when the configuration allows it) 8
template <typename T, int C, int KMAX>
static hipError_t launch_persistent_c(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                      const PersistentExtra& x, hipStream_t s)
{
    switch (K) {
    case 1: return launch_persistent_kc<T, 1, C>(a, face_mode, phases, grid, bar, x, s);
    case 2: return launch_persistent_kc<T, 2, C>(a, face_mode, phases, grid, bar, x, s);
    case 4: return launch_persistent_kc<T, 4, C>(a, face_mode, phases, grid, bar, x, s);
    case 8:
        return KMAX >= 8 ? launch_persistent_kc<T, (KMAX >= 8 ? 8 : 1), C>(a, face_mode, phases, grid, bar, x, s)
                         : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}
template <typename T, int C, int KMAX>
static int persistent_max_c(int K, int face_mode, bool energy)
{
    switch (K) {
    case 1: return persistent_blocks_kc<T, 1, C>(face_mode, energy);
    case 2: return persistent_blocks_kc<T, 2, C>(face_mode, energy);
    case 4: return persistent_blocks_kc<T, 4, C>(face_mode, energy);
    case 8: return KMAX >= 8 ? persistent_blocks_kc<T, (KMAX >= 8 ? 8 : 1), C>(face_mode, energy) : 0;
    default: return 0;
    }
}


}  // namespace fdw
