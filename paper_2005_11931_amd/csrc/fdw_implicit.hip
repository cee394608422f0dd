// fdw_implicit.hip - the implicit scheme of the paper's 2D experiment (Section 3.3: an implicit
// finite-difference scheme whose linear systems are solved by cyclic reduction; Section 4,
// Table 1 times it on a GPU), for gfx950.
//
// Scheme (factorized, alternating-direction form; L1 = d_x(h1 d_x .), L2 = d_y(h2 d_y .) with the
// face coefficients of the explicit solver):
//     (I - s tau^2 L1)(I - s tau^2 L2) w^n = tau^2 (L1 + L2) u^n,
//     du^{n+1} = du^n + w^n,  u^{n+1} = u^n + du^{n+1}    (i.e. u^{n+1} - 2u^n + u^{n-1} = w^n),
// start du^1 = tau u1 + w^0 / 2.  One step is four kernels:
//   1. x lines: the right-hand side tau^2 A u is formed from three rows of u and the row's
//      tridiagonal system (I - s tau^2 L1) z = r is solved, one workgroup per grid row: each
//      thread eliminates within a contiguous chunk of the line (in registers), which leaves two
//      interface unknowns per chunk coupled in a tridiagonal system of their own; that one is
//      solved by cyclic reduction in LDS, and each thread then recovers its chunk's interior;
//   2. z is transposed (64 x 64 LDS tiles) so that the y lines are contiguous;
//   3. y lines: the same cyclic-reduction solve on the rows of z^T with the transposed y faces;
//   4. w^T is transposed back through LDS tiles and added into (du, u).
// The line systems are symmetric and strictly diagonally dominant (1 + s tau^2 (f_l + f_r)/d^2 on
// the diagonal against s tau^2 f/d^2 off it), so cyclic reduction needs no pivoting.
#include "../../include/fdw.h"
#include "fdw_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int kLineThreads = 256;            // threads of a line-solve workgroup (one chunk each)
constexpr int kReducedPad = 1023;            // 2^10 - 1 >= the 2 x 256 interface unknowns
template <typename T>
constexpr int line_chunk() { return sizeof(T) == 8 ? 17 : 33; }  // most unknowns per thread
// longest line (interior unknowns) one workgroup solves
template <typename T>
constexpr int max_line_unknowns() { return kLineThreads * line_chunk<T>(); }
constexpr int kTile = 64;          // transpose tile
constexpr size_t kAdiAlign = 256;
inline size_t adi_align(size_t v) { return (v + kAdiAlign - 1) / kAdiAlign * kAdiAlign; }
inline int pad64(int n) { return (n + 63) / 64 * 64; }

// Cyclic reduction of the system a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k, k = 0..M-1, M = 2^p - 1
// (a_0 = c_{M-1} = 0), in LDS; the solution replaces d.  Forward: at stride s the rows
// k = 2s-1, 4s-1, ... eliminate their neighbours k -/+ s (which this level does not touch), until
// only the middle row is left; backward: the rows k = s-1, 3s-1, ... solved from k -/+ s.
template <typename T>
__device__ void cyclic_reduction(T* a, T* b, T* c, T* d, int M)
{
    const int half = (M + 1) / 2;
    for (int s = 1; s < half; s *= 2) {
        __syncthreads();
        for (int k = threadIdx.x;; k += blockDim.x) {
            const int i = 2 * s * k + 2 * s - 1;
            if (i >= M) break;
            const T al = -a[i] / b[i - s];
            const T ga = -c[i] / b[i + s];
            const T na = al * a[i - s];
            const T nc = ga * c[i + s];
            const T nb = b[i] + al * c[i - s] + ga * a[i + s];
            const T nd = d[i] + al * d[i - s] + ga * d[i + s];
            a[i] = na;
            c[i] = nc;
            b[i] = nb;
            d[i] = nd;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) d[half - 1] = d[half - 1] / b[half - 1];
    for (int s = half / 2; s >= 1; s /= 2) {
        __syncthreads();
        for (int k = threadIdx.x;; k += blockDim.x) {
            const int i = 2 * s * k + s - 1;
            if (i >= M) break;
            const T xl = (i - s >= 0) ? d[i - s] : T(0);
            const T xr = (i + s < M) ? d[i + s] : T(0);
            d[i] = (d[i] - a[i] * xl - c[i] * xr) / b[i];
        }
    }
    __syncthreads();
}

struct LineArgs {
    int lines;      // number of lines (rows of the source layout)
    int len;        // nodes per line (including the two boundary nodes)
    int ld;         // pitch of the line layout (elements)
    double g;       // s tau^2 / d^2 along the line
    const void* F;  // face coefficients along the line: F[line][i] between nodes i and i+1
    void* out;      // solution, [lines][ld]
    // FROM_U: right-hand side tau^2 A u from u (normal layout) and both face planes
    const void* u;
    const void* hx;
    const void* hy;
    double idx2, idy2;  // 1 / dx^2, 1 / dy^2
    double tt;      // tau^2
    const void* rhs;  // !FROM_U: right-hand side rows [lines][ld]
};

// LDS index of element k of a staged line: one pad slot per chunk of MT elements, so that
// threads reading the elements of their own chunks spread over the banks
template <int MT>
__device__ __host__ constexpr int lds_pad(int k)
{
    return k + k / MT;
}

// Chunk length (unknowns per thread) for lines of n unknowns: the shortest of 5, 9, 17, 33 that
// covers the line with 256 threads.  The odd lengths keep the number of interface unknowns of
// lines of 2^k - 2 unknowns (grids of 2^k nodes) below a power of two, so that the padded
// interface system is not twice as large as needed.
template <typename T>
int line_chunk_for(int n)
{
    int mt = 5;
    while (mt < line_chunk<T>() && kLineThreads * mt < n) mt = 2 * mt - 1;
    return mt;
}

// LDS (elements) of a line workgroup: in turn the staged right-hand sides and faces of P chunks
// of MT unknowns, the interface system (four arrays of 2^q - 1 >= 2P), and the staged solution
inline int line_lds_elems(int n, int MT, bool from_u)
{
    const int P = std::max(1, (n + MT - 1) / MT);
    int M = 1;
    while (M < 2 * P) M = 2 * M + 1;
    const int span = P * MT;  // right-hand sides d_0 .. d_{P MT - 1}
    return std::max(span + span / MT + 2, 4 * M);
}

// One line system per workgroup: a_k z_{k-1} + b_k z_k + c_k z_{k+1} = d_k, k = 0..n-1 (unknowns at
// the interior nodes i = k + 1), a_k = -g F_{i-1}, c_k = -g F_i, b_k = 1 + g (F_{i-1} + F_i).
// Partition method: the unknowns are split into P = ceil(n / MT) chunks of MT, one per thread,
// the last one padded with identity rows (decoupled: c_{n-1} = 0).  Each thread loads its chunk's
// faces and right-hand sides (the x lines form the right-hand side from u first, with coalesced
// loads staged through LDS).  In chunk [lo, lo + MT) a downward sweep over rows lo+1 .., with
// z_lo kept as a parameter, gives z_k = d'_k - a'_k z_lo - c'_k z_{k+1}; an upward sweep then
// gives z_k = d~_k - a~_k z_lo - c~_k z_hi (hi = lo + MT - 1) for lo < k < hi.  Row lo (with
// z_{lo+1} substituted) and the last row of the downward sweep couple (z_lo, z_hi) of
// neighbouring chunks in a tridiagonal system of 2P unknowns, solved by cyclic reduction in LDS;
// the interior follows.  Eliminations without pivoting are safe: the systems are strictly
// diagonally dominant.
template <typename T, int MT, bool FROM_U>
__global__ __launch_bounds__(kLineThreads) void k_adi_lines(LineArgs A)
{
    static_assert(MT >= 4, "chunks of at least four unknowns");
    extern __shared__ unsigned char smem[];
    T* const sD = reinterpret_cast<T*>(smem);
    const int line = blockIdx.x;
    const int n = A.len - 2;
    const int ld = A.ld;
    const int P = max(1, (n + MT - 1) / MT);
    T* out = (T*)A.out + (size_t)line * ld;
    if (line == 0 || line == A.lines - 1) {  // boundary lines: zero (the whole block returns)
        for (int i = threadIdx.x; i < A.len; i += blockDim.x) out[i] = T(0);
        return;
    }
    const T g = (T)A.g;
    const int span = P * MT;  // unknowns of the padded line
    // ---- the line's faces F_0 .. F_span and right-hand sides d_0 .. d_{span-1} (zero past the
    // line) are read with coalesced loads and passed through LDS to the threads whose chunks
    // hold them; every thread has at most MT + 1 elements of each.  Loads past the line read the
    // last element instead and their values are replaced by zero afterwards: no branch around a
    // load, so that the loads of one thread are in flight together
    constexpr int NQ = MT + 1;
    T fq[NQ];
    {
        const T* F = (const T*)A.F + (size_t)line * ld;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = (int)threadIdx.x + q * kLineThreads;
            const T f = F[min(i, n)];
            fq[q] = (i <= n) ? f : T(0);
        }
    }
    if constexpr (FROM_U) {
        // tau^2 (A u)_{line, i} in flux form, opposite faces added as pairs (as the explicit
        // solver and the oracle form it; the scalings by 1/dx^2 and 1/dy^2 are products with the
        // reciprocals, which differ from the quotients by rounding only); the loads of a few
        // nodes per thread are issued together (3 in double, 6 in float: measured best)
        const T* u = (const T*)A.u + (size_t)line * ld;
        const T* hx = (const T*)A.hx + (size_t)line * ld;
        const T* hy = (const T*)A.hy + (size_t)line * ld;
        const T idx2 = (T)A.idx2, idy2 = (T)A.idy2, tt = (T)A.tt;
        constexpr int kBatch = sizeof(T) == 8 ? 3 : 6;
#pragma unroll
        for (int q0 = 0; q0 < MT; q0 += kBatch) {
            T dv[kBatch];
#pragma unroll
            for (int q = q0; q < q0 + kBatch; ++q) {
                const int iq = 1 + (int)threadIdx.x + q * kLineThreads;
                const int i = min(iq, n);
                const T uc = u[i];
                const T east = hx[i] * (u[i + 1] - uc);
                const T west = hx[i - 1] * (u[i - 1] - uc);
                const T north = hy[i] * (u[i + ld] - uc);
                const T south = hy[i - ld] * (u[i - ld] - uc);
                const T d = ((east + west) * idx2 + (north + south) * idy2) * tt;
                dv[q - q0] = (iq <= n) ? d : T(0);
            }
#pragma unroll
            for (int q = q0; q < q0 + kBatch; ++q) {
                const int k = (int)threadIdx.x + q * kLineThreads;
                if (k < span) sD[lds_pad<MT>(k)] = dv[q - q0];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const T* r = (const T*)A.rhs + (size_t)line * ld;
        T dq[MT];
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int i = 1 + (int)threadIdx.x + q * kLineThreads;
            const T d = r[min(i, n)];
            dq[q] = (i <= n) ? d : T(0);
        }
#pragma unroll
        for (int q = 0; q < MT; ++q) {
            const int k = (int)threadIdx.x + q * kLineThreads;
            if (k < span) sD[lds_pad<MT>(k)] = dq[q];
        }
    }
    __syncthreads();
    const int p = threadIdx.x;
    const bool act = p < P;
    const int lo = p * MT;
    T fv[MT + 1], dv[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) dv[q] = act ? sD[lds_pad<MT>(lo + q)] : T(0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = (int)threadIdx.x + q * kLineThreads;
        if (i <= span) sD[lds_pad<MT>(i)] = fq[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q <= MT; ++q) fv[q] = act ? sD[lds_pad<MT>(lo + q)] : T(0);
    // row j of the chunk (identity rows past the line)
    auto row = [&](int j, T& a, T& b, T& c, T& d) {
        const int k = lo + j;
        const T fl = fv[j], fr = fv[j + 1];
        const bool real = k < n;
        a = (k > 0 && real) ? -g * fl : T(0);
        c = (k < n - 1) ? -g * fr : T(0);
        b = real ? T(1) + g * (fl + fr) : T(1);
        d = dv[j];
    };
    T ap[MT], cp[MT], dp[MT];
    T a0, b0, c0, d0;
    row(0, a0, b0, c0, d0);
    // downward sweep over rows lo+1 .. hi
    {
        T a, b, c, d;
        row(1, a, b, c, d);
        const T rr = T(1) / b;
        ap[1] = a * rr;
        cp[1] = c * rr;
        dp[1] = d * rr;
    }
#pragma unroll
    for (int j = 2; j < MT; ++j) {
        T a, b, c, d;
        row(j, a, b, c, d);
        const T rr = T(1) / (b - a * cp[j - 1]);
        cp[j] = c * rr;
        dp[j] = (d - a * dp[j - 1]) * rr;
        ap[j] = -(a * ap[j - 1]) * rr;
    }
    const T ha = ap[MT - 1], hc = cp[MT - 1], hr = dp[MT - 1];
    // upward sweep: rows hi-2 .. lo+1 in terms of z_lo and z_hi
#pragma unroll
    for (int j = MT - 3; j >= 1; --j) {
        const T q = cp[j];
        dp[j] = dp[j] - q * dp[j + 1];
        ap[j] = ap[j] - q * ap[j + 1];
        cp[j] = -(q * cp[j + 1]);
    }
    const T la = a0, lb = b0 - c0 * ap[1], lc = -(c0 * cp[1]), lr = d0 - c0 * dp[1];
    // interface system in the same LDS (once every thread has read its rows): unknowns
    // (z_lo, z_hi) of chunk p at 2p, 2p+1, padded with identity rows to 2^q - 1
    int M = 1;
    while (M < 2 * P) M = 2 * M + 1;
    T* const ra = sD;
    T* const rb = ra + M;
    T* const rc = rb + M;
    T* const rd = rc + M;
    __syncthreads();
    if (act) {
        ra[2 * p] = la, rb[2 * p] = lb, rc[2 * p] = lc, rd[2 * p] = lr;
        ra[2 * p + 1] = ha, rb[2 * p + 1] = T(1), rc[2 * p + 1] = hc, rd[2 * p + 1] = hr;
    }
    for (int k = 2 * P + threadIdx.x; k < M; k += blockDim.x) ra[k] = T(0), rb[k] = T(1), rc[k] = T(0), rd[k] = T(0);
    cyclic_reduction<T>(ra, rb, rc, rd, M);
    // the chunk's solution, staged in LDS (over the interface system, once every thread has read
    // its two values) and stored with coalesced writes
    T xl = T(0), xh = T(0);
    if (act) xl = rd[2 * p], xh = rd[2 * p + 1];
    __syncthreads();
    T* const sX = sD;
    if (act) {
        sX[lds_pad<MT>(lo)] = xl;
#pragma unroll
        for (int j = 1; j < MT - 1; ++j) sX[lds_pad<MT>(lo + j)] = dp[j] - ap[j] * xl - cp[j] * xh;
        sX[lds_pad<MT>(lo + MT - 1)] = xh;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < A.len; i += blockDim.x) out[i] = (i >= 1 && i <= n) ? sX[lds_pad<MT>(i - 1)] : T(0);
}

// out[c][r] = in[r][c] for r < rows, c < cols (pitches ld_in, ld_out), through 64 x 64 LDS tiles.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, int rows, int cols, int ld_in,
                                                   T* __restrict__ out, int ld_out)
{
    __shared__ T tile[kTile][kTile + 1];
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int y = ty; y < kTile; y += 4) {
        const int r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) tile[y][tx] = in[(size_t)r * ld_in + c];
    }
    __syncthreads();
    for (int y = ty; y < kTile; y += 4) {
        const int c = c0 + y, r = r0 + tx;
        if (c < cols && r < rows) out[(size_t)c * ld_out + r] = tile[tx][y];
    }
}

// w = (w^T)^T through LDS tiles, then du = du + w, u = u + du (START: du = tau u1 + w/2,
// u = u0 + du); interior nodes only (w is 0 on the ring; du and u stay 0 there).
template <typename T, bool START>
__global__ __launch_bounds__(256) void k_adi_update(const T* __restrict__ wT, int ldT, int nx, int ny, int ld,
                                                    T* __restrict__ du, T* __restrict__ u, const T* __restrict__ u0,
                                                    const T* __restrict__ u1, T tau)
{
    __shared__ T tile[kTile][kTile + 1];
    const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // wT[i][j]: rows i0.., columns j0..
    for (int y = ty; y < kTile; y += 4) {
        const int i = i0 + y, j = j0 + tx;
        if (i < nx && j < ny) tile[y][tx] = wT[(size_t)i * ldT + j];
    }
    __syncthreads();
    for (int y = ty; y < kTile; y += 4) {
        const int j = j0 + y, i = i0 + tx;
        if (j < 1 || j > ny - 2 || i < 1 || i > nx - 2) continue;
        const size_t k = (size_t)j * ld + i;
        const T w = tile[tx][y];
        if constexpr (START) {
            const T nd = tau * u1[k] + T(0.5) * w;
            du[k] = nd;
            u[k] = u0[k] + nd;
        } else {
            const T nd = du[k] + w;
            du[k] = nd;
            u[k] = u[k] + nd;
        }
    }
}

// Faces (means of nodal values, 0 past the last node) and validation statistics of h1, h2:
// red[block] = {min h, max x face, max y face, non-finite count}.
template <typename T>
__global__ __launch_bounds__(256) void k_adi_faces(const T* __restrict__ h1, const T* __restrict__ h2, int nx, int ny,
                                                   int ld, T* __restrict__ hx, T* __restrict__ hy, double* red)
{
    __shared__ double s[4][256];
    double mn = INFINITY, mxx = 0.0, mxy = 0.0, bad = 0.0;
    const int64_t total = (int64_t)nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int j = (int)(k / nx), i = (int)(k % nx);
        const T a = h1[k], b2 = h2[k];
        if (!isfinite((double)a) || !isfinite((double)b2)) bad += 1.0;
        mn = fmin(mn, fmin((double)a, (double)b2));
        const T fx = (i < nx - 1) ? T(0.5) * (a + h1[k + 1]) : T(0);
        const T fy = (j < ny - 1) ? T(0.5) * (b2 + h2[k + nx]) : T(0);
        hx[(size_t)j * ld + i] = fx;
        hy[(size_t)j * ld + i] = fy;
        mxx = fmax(mxx, (double)fx);
        mxy = fmax(mxy, (double)fy);
    }
    s[0][threadIdx.x] = mn;
    s[1][threadIdx.x] = mxx;
    s[2][threadIdx.x] = mxy;
    s[3][threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] += s[3][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) red[4 * blockIdx.x + q] = s[q][0];
}

// dense [ny][nx] -> pitched [ny][ld], boundary ring zeroed
template <typename T>
__global__ void k_adi_copy_in(const T* __restrict__ src, int nx, int ny, int ld, T* __restrict__ dst)
{
    const int64_t total = (int64_t)ld * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / ld), i = (int)(k % ld);
        const bool in = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
        dst[k] = in ? src[(size_t)j * nx + i] : T(0);
    }
}
template <typename T>
__global__ void k_adi_copy_out(const T* __restrict__ src, int nx, int ny, int ld, T* __restrict__ dst)
{
    const int64_t total = (int64_t)nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[(size_t)(k / nx) * ld + (k % nx)];
}

}  // namespace

struct fdw_adi {
    fdw_problem p;
    int nx = 0, ny = 0, ld = 0, ldT = 0;
    int64_t N = 0, n = 0;
    double dx = 0, dy = 0, sigma = 0.25;
    hipStream_t stream = nullptr;
    std::string err;
    void *u = nullptr, *du = nullptr, *u0 = nullptr, *u1 = nullptr, *hx = nullptr, *hy = nullptr, *hyT = nullptr;
    void *z = nullptr, *zT = nullptr, *wT = nullptr;
    double* red = nullptr;
    // kAdiGraphSteps steps (after the start step) captured once in a hipGraph on a private
    // stream and replayed on `stream`
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
};

namespace {

constexpr int kAdiRedBlocks = 256;

size_t adi_plane(int ld, int rows, int dtype) { return adi_align((size_t)ld * rows * (dtype == FDW_F32 ? 4 : 8)); }

int adi_fail(fdw_adi* s, int code, const std::string& msg)
{
    if (s) s->err = msg;
    return code;
}

#define ADICHK(s, expr)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return adi_fail((s), FDW_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T, int MT>
bool allow_lds_mt(int bytes)
{
    return hipFuncSetAttribute((const void*)k_adi_lines<T, MT, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               bytes) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_adi_lines<T, MT, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               bytes) == hipSuccess;
}

// let the line kernel that lines of up to n unknowns use take the LDS it needs
template <typename T>
int allow_line_lds(int n)
{
    const int mt = line_chunk_for<T>(n);
    const int bytes = line_lds_elems(n, mt, true) * (int)sizeof(T);
    bool ok = true;
    switch (mt) {
    case 5: ok = allow_lds_mt<T, 5>(bytes); break;
    case 9: ok = allow_lds_mt<T, 9>(bytes); break;
    case 17: ok = allow_lds_mt<T, 17>(bytes); break;
    default: ok = allow_lds_mt<T, line_chunk<T>()>(bytes); break;
    }
    return ok ? FDW_OK : FDW_EHIP;
}

template <typename T, int MT>
void launch_lines_mt(bool from_u, dim3 gr, dim3 bl, size_t shmem, hipStream_t st, const LineArgs& A)
{
    if (from_u)
        hipLaunchKernelGGL((k_adi_lines<T, MT, true>), gr, bl, shmem, st, A);
    else
        hipLaunchKernelGGL((k_adi_lines<T, MT, false>), gr, bl, shmem, st, A);
}

template <typename T>
hipError_t launch_lines(const fdw_adi* s, bool from_u, const void* F, int lines, int len, int ld, double g,
                        const void* rhs, void* out, hipStream_t st)
{
    LineArgs A;
    std::memset(&A, 0, sizeof(A));
    A.lines = lines;
    A.len = len;
    A.ld = ld;
    A.g = g;
    A.F = F;
    A.out = out;
    A.u = (s->n == 0) ? s->u0 : s->u;  // the start step solves with the initial displacement
    A.hx = s->hx;
    A.hy = s->hy;
    A.idx2 = 1.0 / (s->dx * s->dx);
    A.idy2 = 1.0 / (s->dy * s->dy);
    A.tt = s->p.tau * s->p.tau;
    A.rhs = rhs;
    const int mt = line_chunk_for<T>(len - 2);
    const size_t shmem = (size_t)line_lds_elems(len - 2, mt, from_u) * sizeof(T);
    const dim3 gr(lines), bl(kLineThreads);
    switch (mt) {
    case 5: launch_lines_mt<T, 5>(from_u, gr, bl, shmem, st, A); break;
    case 9: launch_lines_mt<T, 9>(from_u, gr, bl, shmem, st, A); break;
    case 17: launch_lines_mt<T, 17>(from_u, gr, bl, shmem, st, A); break;
    default: launch_lines_mt<T, line_chunk<T>()>(from_u, gr, bl, shmem, st, A); break;
    }
    return hipGetLastError();
}

// one solve w = B^{-1} tau^2 A u (into wT, transposed) and the update of (du, u), on stream st
template <typename T>
int adi_step(fdw_adi* s, bool start, hipStream_t st)
{
    const double tt = s->p.tau * s->p.tau;
    // x lines: rows of the normal layout
    ADICHK(s, launch_lines<T>(s, true, s->hx, s->ny, s->nx, s->ld, s->sigma * tt / (s->dx * s->dx), nullptr, s->z, st));
    // z -> z^T
    const dim3 tg((s->nx + kTile - 1) / kTile, (s->ny + kTile - 1) / kTile);
    hipLaunchKernelGGL((k_transpose<T>), tg, dim3(256), 0, st, (const T*)s->z, s->ny, s->nx, s->ld, (T*)s->zT, s->ldT);
    ADICHK(s, hipGetLastError());
    // y lines: rows of the transposed layout
    ADICHK(s, launch_lines<T>(s, false, s->hyT, s->nx, s->ny, s->ldT, s->sigma * tt / (s->dy * s->dy), s->zT,
                              s->wT, st));
    // w^T -> (du, u)
    const dim3 ug((s->nx + kTile - 1) / kTile, (s->ny + kTile - 1) / kTile);
    if (start)
        hipLaunchKernelGGL((k_adi_update<T, true>), ug, dim3(256), 0, st, (const T*)s->wT, s->ldT, s->nx, s->ny,
                           s->ld, (T*)s->du, (T*)s->u, (const T*)s->u0, (const T*)s->u1, (T)s->p.tau);
    else
        hipLaunchKernelGGL((k_adi_update<T, false>), ug, dim3(256), 0, st, (const T*)s->wT, s->ldT, s->nx, s->ny,
                           s->ld, (T*)s->du, (T*)s->u, (const T*)s->u0, (const T*)s->u1, (T)s->p.tau);
    ADICHK(s, hipGetLastError());
    return FDW_OK;
}

constexpr int kAdiGraphSteps = 16;

// capture kAdiGraphSteps ordinary steps once (their launches depend on nothing but the solver's
// fixed buffers); on any failure the solver keeps launching step by step
template <typename T>
void adi_capture(fdw_adi* s)
{
    if (!s->cap && hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess) {
        s->cap = nullptr;
        s->graph_failed = true;
        return;
    }
    if (hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        s->graph_failed = true;
        return;
    }
    int rc = FDW_OK;
    for (int k = 0; k < kAdiGraphSteps && rc == FDW_OK; ++k) rc = adi_step<T>(s, false, s->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->cap, &g);
    if (rc != FDW_OK || e != hipSuccess || !g || hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        s->exec = nullptr;
        s->graph_failed = true;
    }
    if (g) hipGraphDestroy(g);
}

template <typename T>
int adi_setup(fdw_adi* s, const void* u0, const void* u1, const void* h1, const void* h2)
{
    const int nx = s->nx, ny = s->ny;
    hipLaunchKernelGGL((k_adi_copy_in<T>), dim3(512), dim3(256), 0, s->stream, (const T*)u0, nx, ny, s->ld, (T*)s->u0);
    hipLaunchKernelGGL((k_adi_copy_in<T>), dim3(512), dim3(256), 0, s->stream, (const T*)u1, nx, ny, s->ld, (T*)s->u1);
    hipLaunchKernelGGL((k_adi_faces<T>), dim3(kAdiRedBlocks), dim3(256), 0, s->stream, (const T*)h1,
                       (const T*)(h2 ? h2 : h1), nx, ny, s->ld, (T*)s->hx, (T*)s->hy, s->red);
    ADICHK(s, hipGetLastError());
    // y faces, transposed: hyT[i][j] = hy[j][i]
    const dim3 tg((nx + kTile - 1) / kTile, (ny + kTile - 1) / kTile);
    hipLaunchKernelGGL((k_transpose<T>), tg, dim3(256), 0, s->stream, (const T*)s->hy, ny, nx, s->ld, (T*)s->hyT,
                       s->ldT);
    ADICHK(s, hipGetLastError());
    std::vector<double> red(4 * kAdiRedBlocks);
    ADICHK(s, hipMemcpyAsync(red.data(), s->red, red.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    ADICHK(s, hipStreamSynchronize(s->stream));
    double mn = INFINITY, mxx = 0, mxy = 0, bad = 0;
    for (int b = 0; b < kAdiRedBlocks; ++b) {
        mn = std::min(mn, red[4 * b]);
        mxx = std::max(mxx, red[4 * b + 1]);
        mxy = std::max(mxy, red[4 * b + 2]);
        bad += red[4 * b + 3];
    }
    if (bad != 0.0) return adi_fail(s, FDW_EINVAL, "h contains non-finite values");
    const bool allow0 = (s->p.flags & FDW_ALLOW_ZERO_H) != 0;
    if (allow0 ? !(mn >= 0.0) : !(mn > 0.0)) return adi_fail(s, FDW_EINVAL, allow0 ? "h must be >= 0" : "h must be > 0");
    if (s->sigma < 0.25 && !(s->p.flags & FDW_ALLOW_UNSTABLE)) {
        // below sigma = 1/4 the scheme is stable for tau^2 lambda_max (1 - 4 sigma) <= 4 only
        const double tt = s->p.tau * s->p.tau;
        const double bound = tt * (4.0 * mxx / (s->dx * s->dx) + 4.0 * mxy / (s->dy * s->dy)) * (1.0 - 4.0 * s->sigma);
        if (bound > 4.0 * (1.0 + 1e-12)) return adi_fail(s, FDW_ECFL, "time step above the stability bound for sigma < 1/4");
    }
    return FDW_OK;
}

}  // namespace

extern "C" {

size_t fdw_adi_workspace_bytes(const fdw_problem* p)
{
    if (!p || p->nx < 3 || p->ny < 3 || (p->dtype != FDW_F32 && p->dtype != FDW_F64)) return 0;
    const int ld = pad64(p->nx), ldT = pad64(p->ny);
    size_t b = 7 * adi_plane(ld, p->ny, p->dtype);   // u, du, u0, u1, hx, hy, z
    b += 3 * adi_plane(ldT, p->nx, p->dtype);        // hyT, zT, wT
    b += adi_align(sizeof(double) * 4 * kAdiRedBlocks);
    return b;
}

int fdw_adi_init(const fdw_problem* p, double sigma, void* workspace, size_t ws_bytes, const void* u0, const void* u1,
                 const void* h1, const void* h2, void* hip_stream, fdw_adi** out)
{
    if (!out) return FDW_EINVAL;
    *out = nullptr;
    if (!p || !workspace || !u0 || !u1 || !h1) return FDW_EINVAL;
    if (((uintptr_t)workspace) % kAdiAlign) return FDW_EINVAL;
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) return FDW_EINVAL;
    if (p->nx < 3 || p->ny < 3 || !(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->tau > 0.0) || !std::isfinite(p->tau) ||
        !(p->T >= 0.0))
        return FDW_EINVAL;
    const int64_t N = (int64_t)std::llround(p->T / p->tau);
    if (std::fabs((double)N * p->tau - p->T) > 1e-9 * std::max(p->T, p->tau)) return FDW_EINVAL;
    const size_t need = fdw_adi_workspace_bytes(p);
    if (need == 0) return FDW_EINVAL;
    if (ws_bytes < need) return FDW_ENOMEM;
    fdw_adi* s = new fdw_adi();
    s->p = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->ld = pad64(p->nx);
    s->ldT = pad64(p->ny);
    s->N = N;
    s->dx = (p->x1 - p->x0) / (p->nx - 1);
    s->dy = (p->y1 - p->y0) / (p->ny - 1);
    s->sigma = sigma;
    s->stream = (hipStream_t)hip_stream;
    // a line of n unknowns is solved by one workgroup: n <= 256 chunks of line_chunk<T>() unknowns
    const int maxn = (p->dtype == FDW_F32) ? max_line_unknowns<float>() : max_line_unknowns<double>();
    if (std::max(p->nx, p->ny) - 2 > maxn) {
        delete s;
        return FDW_ENOTSUP;
    }
    char* w = (char*)workspace;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void* q = w + off;
        off += bytes;
        return q;
    };
    const size_t pn = adi_plane(s->ld, s->ny, p->dtype), pt = adi_plane(s->ldT, s->nx, p->dtype);
    s->u = take(pn);
    s->du = take(pn);
    s->u0 = take(pn);
    s->u1 = take(pn);
    s->hx = take(pn);
    s->hy = take(pn);
    s->z = take(pn);
    s->hyT = take(pt);
    s->zT = take(pt);
    s->wT = take(pt);
    s->red = (double*)take(adi_align(sizeof(double) * 4 * kAdiRedBlocks));
    // zero the state, faces and scratch (padding columns and the boundary ring stay 0)
    if (fdw::launch_fill_bytes(workspace, off, s->stream) != hipSuccess) {
        delete s;
        return FDW_EHIP;
    }
    // the line kernels' dynamic LDS (above the default limit for the longest lines)
    const int rc0 = (p->dtype == FDW_F32) ? allow_line_lds<float>(std::max(p->nx, p->ny) - 2)
                                          : allow_line_lds<double>(std::max(p->nx, p->ny) - 2);
    if (rc0 != FDW_OK) {
        delete s;
        return rc0;
    }
    const int rc = (p->dtype == FDW_F32) ? adi_setup<float>(s, u0, u1, h1, h2) : adi_setup<double>(s, u0, u1, h1, h2);
    if (rc) {
        const int code = rc;
        delete s;
        return code;
    }
    *out = s;
    return FDW_OK;
}

int fdw_adi_step_n(fdw_adi* s, int64_t n)
{
    if (!s) return FDW_EINVAL;
    if (n < 0) return adi_fail(s, FDW_EINVAL, "n must be >= 0");
    const bool f32 = s->p.dtype == FDW_F32;
    int64_t k = 0;
    while (k < n) {
        const bool start = s->n == 0;
        if (!start && n - k >= kAdiGraphSteps && !s->graph_failed) {
            // runs of kAdiGraphSteps steps are replayed from a hipGraph (the launch-bound small grids
            // gain most)
            if (!s->exec) f32 ? adi_capture<float>(s) : adi_capture<double>(s);
            if (s->exec) {
                ADICHK(s, hipGraphLaunch(s->exec, s->stream));
                s->n += kAdiGraphSteps;
                k += kAdiGraphSteps;
                continue;
            }
        }
        const int rc = f32 ? adi_step<float>(s, start, s->stream) : adi_step<double>(s, start, s->stream);
        if (rc) return rc;
        s->n += 1;
        k += 1;
    }
    return FDW_OK;
}

int fdw_adi_get_state(fdw_adi* s, void* u, void* du, int64_t* n)
{
    if (!s) return FDW_EINVAL;
    if (n) *n = s->n;
    const bool f32 = s->p.dtype == FDW_F32;
    const void* su = (s->n == 0) ? s->u0 : s->u;
    if (u) {
        if (f32)
            hipLaunchKernelGGL((k_adi_copy_out<float>), dim3(512), dim3(256), 0, s->stream, (const float*)su, s->nx,
                               s->ny, s->ld, (float*)u);
        else
            hipLaunchKernelGGL((k_adi_copy_out<double>), dim3(512), dim3(256), 0, s->stream, (const double*)su, s->nx,
                               s->ny, s->ld, (double*)u);
        ADICHK(s, hipGetLastError());
    }
    if (du) {
        if (s->n == 0) {
            ADICHK(s, fdw::launch_fill_bytes(du, (size_t)s->nx * s->ny * (f32 ? 4 : 8), s->stream));
        } else if (f32) {
            hipLaunchKernelGGL((k_adi_copy_out<float>), dim3(512), dim3(256), 0, s->stream, (const float*)s->du, s->nx,
                               s->ny, s->ld, (float*)du);
        } else {
            hipLaunchKernelGGL((k_adi_copy_out<double>), dim3(512), dim3(256), 0, s->stream, (const double*)s->du,
                               s->nx, s->ny, s->ld, (double*)du);
        }
        ADICHK(s, hipGetLastError());
    }
    return FDW_OK;
}

int fdw_adi_reset(fdw_adi* s)
{
    if (!s) return FDW_EINVAL;
    s->n = 0;
    return FDW_OK;
}

const char* fdw_adi_last_error(const fdw_adi* s) { return s ? s->err.c_str() : "null context"; }

void fdw_adi_destroy(fdw_adi* s)
{
    if (!s) return;
    if (s->exec) hipGraphExecDestroy(s->exec);
    if (s->cap) hipStreamDestroy(s->cap);
    delete s;
}

}  // extern "C"
