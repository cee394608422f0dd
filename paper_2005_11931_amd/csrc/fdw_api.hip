// fdw_api.hip - host side of libfdw: validation, workspace carving, the member table, the
// launch sequence of a step_n call (optionally captured in a hipGraph), snapshots and the
// autotuner.  The problem it solves is the regularised Cauchy problem of arXiv 2005.11931,
// Section 2 eq. (2.1), on the grid of Section 3.3 (see include/fdw.h).
#include "../../include/fdw.h"
#include "fdw_internal.h"
#include "fdw_tile.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

using namespace fdw;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
// one 8-byte value per lane and row: FP32 pairs, FP64 singles (the deepest time blocks fit)
inline int default_cols_per_lane(int dtype) { return dtype == FDW_F32 ? 2 : 1; }
// every plane carries zero rows above and below the grid (streamed rows may run past it)
inline size_t plane_alloc(int ld, int ny, size_t es)
{
    return (size_t)ld * (size_t)(kPadRowsTop + ny + kPadRowsBottom) * es;
}
inline void* plane_origin(void* base, int ld, size_t es) { return (char*)base + (size_t)kPadRowsTop * ld * es; }
inline size_t elem_size(int dtype) { return dtype == FDW_F32 ? 4 : 8; }
inline int pitch_of(int nx) { return (int)align_up((size_t)nx, 64); }
constexpr int kMinSegRows = 8;      // rows per streaming work item, at least
constexpr int kMinAdjSegRows = 16;  // ... and per reverse-sweep work item

struct HostMember {
    fdw_problem p;
    int nx = 0, ny = 0, ld = 0;
    int64_t N = 0;
    double dx = 0, dy = 0, tau = 0;
    int face = 0;
    bool coeff = false;
    int64_t n = 0;  // steps taken
    int cur = 0;    // pair holding the state (n >= 1)
    void* u[2] = {nullptr, nullptr};
    void* d[2] = {nullptr, nullptr};
    void* h = nullptr;
    void* hy = nullptr;
    void* u0 = nullptr;
    void* u1 = nullptr;
    int* rec_ij = nullptr;
    int* rowptr = nullptr;
    int* rcol = nullptr;
    int* rid = nullptr;
    double* epart = nullptr;
    int epart_stride = 0;
    int eslots = 2;  // energy-partial slots (time blocks whose energies one finalisation sums)
    int R = 0;
    int ndup = 0;  // receivers sharing a node with an earlier one (their traces are copied)
    void* traces = nullptr;
    size_t plane_bytes = 0;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct fdw_ctx {
    int count = 0;
    int dtype = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
    std::vector<HostMember> m;
    std::vector<MemberDev> tab;  // host mirror of the device table
    MemberDev* tab_dev = nullptr;
    double* red = nullptr;
    int* status = nullptr;
    int* barrier = nullptr;
    double* scal = nullptr;  // small device scalars (energies read back by fdw_energy)
    int K_cfg = 0, S_cfg = 0, use_graph = 0, batch_mode = 0, timing = 0;
    int check_energy = 1;  // fdw_step_n checks the energies it computes (FDW_CFG_CHECK_ENERGY)
    int item_order = 1;    // FDW_CFG_ITEM_ORDER: 1 walks every other launch's blocks in reverse
    int stream_policy = 0; // FDW_CFG_STREAM_POLICY: 0 automatic, 1 non-temporal, 2 cacheable
    int tile_mode = 0;     // FDW_CFG_SMALL_TILES: 0 automatic, 1 never, 2 wherever allowed
    int tile_rows = 0;     // FDW_CFG_TILE_ROWS: rows per tile (0 = automatic)
    bool tiles_now = false;  // the member table holds the tile decomposition
    int test_flag_barrier = 0;  // FDW_CFG_TEST_BARRIER_FLAG: mark the next persistent call as timed out
    bool used_persistent = false;  // the last step_n ran the persistent launch
    int C = 4;  // columns per lane of the streaming kernels
    int adjK = 2, adjC = 2;  // time block and columns per lane of the reverse sweep
    int adjS_cfg = 0;        // rows per reverse work item (0 = automatic)
    // checkpoints of the adjoint stored by the forward run of one member (member < 0: off)
    struct {
        int member = -1;
        int ck = 0;
        void* ws = nullptr;
    } rec;
    std::vector<hipEvent_t> ev_pool;  // instrumentation: start/end pairs of stencil launches
    size_t ev_used = 0;
    int S_eff = 0;
    int64_t ctx_step = 0;
    int64_t launches = 0;
    std::map<std::tuple<int64_t, int, const double*, int, int, uint64_t>, GraphEntry> graphs;
    // A family whose members do not all share one storage type is held as one child context per
    // type (member m of the family is member sub_idx[m] of child sub_of[m]); the parent itself
    // holds no state and forwards every call.
    bool mixed = false;
    fdw_ctx* sub[2] = {nullptr, nullptr};
    std::vector<int> sub_of, sub_idx;
};

namespace {

// status[8]: failure-detection word of the energy finalisation (see launch_energy_finalize);
// status[9]: error word of the persistent launch (bit 0: a grid barrier timed out)
int* health_word(fdw_ctx* c) { return c->status + 8; }
int* sync_err_word(fdw_ctx* c) { return c->status + 9; }

int fail(fdw_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                             \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail((ctx), FDW_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

bool problem_ok(const fdw_problem& p, std::string* why, int64_t* N_out)
{
    if (p.nx < 3 || p.ny < 3) return *why = "nx and ny must be >= 3", false;
    if ((int64_t)p.nx * p.ny > (int64_t)1 << 31) return *why = "grid too large", false;
    if (!(p.x1 > p.x0) || !(p.y1 > p.y0) || !std::isfinite(p.x0) || !std::isfinite(p.x1) || !std::isfinite(p.y0) ||
        !std::isfinite(p.y1))
        return *why = "domain must satisfy x0 < x1, y0 < y1 (finite)", false;
    if (!(p.tau > 0.0) || !std::isfinite(p.tau)) return *why = "tau must be finite and > 0", false;
    if (!(p.T >= 0.0) || !std::isfinite(p.T)) return *why = "T must be finite and >= 0", false;
    if (p.dtype != FDW_F32 && p.dtype != FDW_F64) return *why = "dtype must be FDW_F32 or FDW_F64", false;
    const double q = p.T / p.tau;
    const int64_t N = (int64_t)std::llround(q);
    if (std::fabs((double)N * p.tau - p.T) > 1e-9 * std::max(p.T, p.tau)) return *why = "T/tau is not an integer", false;
    if (N_out) *N_out = N;
    return true;
}

// column strips of a streaming launch with C columns per lane and time block K
int strips_for(int nx, int C, int K)
{
    const int Hx = ((K + C - 1) / C) * C;
    const int Wv = kWaveSize * C - 2 * Hx;
    return (nx + Wv - 1) / Wv;
}

// upper bound over every configuration (sizes the per-wave buffers): the narrowest strip has
// 1 column per lane and the deepest time block
int max_strips(int nx) { return strips_for(nx, 1, kMaxTimeBlock); }

// Energy-partial slots of a member: one slot holds the per-wave partials of one time block.
// The per-time-block path fills up to this many slots before one finalisation launch sums them
// all (fewer launches for small, launch-bound grids); at least the two the persistent launch
// alternates, at most 64, within about 8 MiB.
int energy_slots(const fdw_problem& p)
{
    const size_t maxw = (size_t)max_strips(p.nx) * (size_t)((p.ny + kMinSegRows - 1) / kMinSegRows);
    const size_t per = sizeof(double) * kMaxTimeBlock * std::max<size_t>(maxw, 1);
    return (int)std::max<size_t>(2, std::min<size_t>(64, ((size_t)8 << 20) / per));
}

size_t member_bytes(const fdw_problem& p)
{
    const int ld = pitch_of(p.nx);
    const size_t plane = align_up(plane_alloc(ld, p.ny, elem_size(p.dtype)), kAlign);
    const size_t maxw = (size_t)max_strips(p.nx) * (size_t)((p.ny + kMinSegRows - 1) / kMinSegRows);
    size_t b = 8 * plane;                                          // u[2], d[2], h, hy, u0, u1
    b += align_up(sizeof(int) * 2 * kMaxReceivers, kAlign);        // rec_ij
    b += align_up(sizeof(int) * (size_t)(p.ny + 1), kAlign);       // rowptr
    b += 2 * align_up(sizeof(int) * kMaxReceivers, kAlign);        // col, id
    b += align_up(sizeof(double) * (size_t)energy_slots(p) * kMaxTimeBlock * maxw, kAlign);  // energy partials
    return b;
}

size_t header_bytes(int count)
{
    size_t b = align_up(sizeof(MemberDev) * (size_t)count, kAlign);
    b += align_up(sizeof(double) * (4 * kRedBlocks + 16), kAlign);  // red
    b += align_up(sizeof(int) * 16, kAlign);                         // status
    b += align_up(sizeof(int) * kPersistentCtlInts, kAlign);         // persistent launch control
    b += align_up(sizeof(double) * (size_t)std::max(count, 1) * 2, kAlign);  // scalars
    return b;
}

void decompose(const fdw_ctx* c, const HostMember& hm, MemberDev& md, int S, int K)
{
    const int C = c->C;
    const int Hx = ((K + C - 1) / C) * C;
    const int Wv = kWaveSize * C - 2 * Hx;
    md.seg_rows = S;
    md.segs = (hm.ny + S - 1) / S;
    md.strips = (hm.nx + Wv - 1) / Wv;
    md.waves = md.strips * md.segs;
    md.blocks = (md.waves + kWavesPerBlock - 1) / kWavesPerBlock;
    // energy partials are laid out for this decomposition's waves (the allocation is sized for
    // the most waves any configuration has: fewer waves leave room for more time-block slots)
    md.epart_stride = std::max(md.waves, 1);
}

// rows per tile of the small-grid kernel (64, 48 or 32 rows: 16, 12 or 8 waves): 64 where that
// gives the launch 150..300 tiles (about one per CU), else 48 where that gives at least 150,
// else 32.  Measured (256^2 .. 1024^2, FP64 and FP32, time block 8): the per-tile time grows
// with the waves sharing a SIMD, the redundant halo work with the tile count.
int tile_rows(const fdw_ctx* c)
{
    if (c->tile_rows > 0) return c->tile_rows;
    auto tiles_of = [&](int rows) {
        int64_t tiles = 0;
        for (const HostMember& hm : c->m)
            tiles += (int64_t)((hm.nx + kTileCols - 1) / kTileCols) *
                     ((hm.ny + rows - 2 * kTileHalo - 1) / (rows - 2 * kTileHalo));
        return tiles;
    };
    const int64_t t64 = tiles_of(64);
    if (t64 >= 150 && t64 <= 300) return 64;
    return tiles_of(48) >= 150 ? 48 : 32;
}

// The small-grid decomposition: one tile per workgroup, independent of the time block (its halo
// covers the deepest one).  waves = blocks = tiles (one energy partial per tile and level).
void decompose_tile(const fdw_ctx* c, const HostMember& hm, MemberDev& md)
{
    const int rows = tile_rows(c);
    md.seg_rows = rows - 2 * kTileHalo;
    md.segs = (hm.ny + md.seg_rows - 1) / md.seg_rows;
    md.strips = (hm.nx + kTileCols - 1) / kTileCols;
    md.waves = md.strips * md.segs;
    md.blocks = md.waves;
    md.epart_stride = std::max(md.waves, 1);
}

// time blocks whose energy partials fit member i's allocation at its current decomposition
int energy_group_cap(const fdw_ctx* c, int i)
{
    const HostMember& hm = c->m[i];
    const size_t cap = (size_t)hm.eslots * (size_t)hm.epart_stride;  // per level, in waves
    return (int)std::min<size_t>(kMaxEnergySlots, cap / (size_t)std::max(c->tab[i].epart_stride, 1));
}

// reverse-sweep configurations with one 8-byte value per lane and row (time blocks up to 6)
bool adj_narrow(int dtype, int C) { return (dtype == FDW_F64) ? C == 1 : C == 2; }

int choose_K(const fdw_ctx* c)
{
    if (c->K_cfg > 0) return c->K_cfg;
    // deepest time block of the configuration (8 with one 8-byte value per lane and row)
    if (c->dtype == FDW_F32) return c->C == 4 ? 6 : 8;
    return c->C == 1 ? 8 : 4;
}

int choose_S(const fdw_ctx* c)
{
    if (c->S_cfg > 0) return c->S_cfg;
    // Segments of 16 K rows (the 2K halo rows of a segment are then 1/8 of it, and half of
    // them are usually shared with the neighbouring segment through L2), but short enough to
    // give about 4600 streaming waves (one and a half rounds of the wave slots) for the
    // largest member; at least 8 rows (small grids: more, shorter items).
    const int K = choose_K(c);
    int best = kMinSegRows;
    for (const HostMember& hm : c->m) {
        const int64_t strips = strips_for(hm.nx, c->C, K);
        int64_t S = (hm.ny * strips + 4607) / 4608;
        S = std::min<int64_t>(16 * K, std::max<int64_t>(kMinSegRows, (S + 7) / 8 * 8));
        best = std::max(best, (int)S);
    }
    return best;
}

__global__ void k_write_member(MemberDev* tab, int m, MemberDev val) { tab[m] = val; }

int push_member(fdw_ctx* c, int m, hipStream_t s = nullptr)
{
    hipLaunchKernelGGL(k_write_member, dim3(1), dim3(1), 0, s ? s : c->stream, c->tab_dev, m, c->tab[m]);
    HIPCHK(c, hipGetLastError());
    return FDW_OK;
}

// Rebuild the launch decomposition for time block K (all members) and push the table.
int layout_for_K(fdw_ctx* c, int K, int S, hipStream_t st = nullptr)
{
    int base = 0;
    for (int i = 0; i < c->count; ++i) {
        MemberDev& md = c->tab[i];
        if (c->tiles_now)
            decompose_tile(c, c->m[i], md);
        else
            decompose(c, c->m[i], md, S, K);
        md.block_base = base;
        base += md.blocks;
    }
    for (int i = 0; i < c->count; ++i) {
        int rc = push_member(c, i, st);
        if (rc) return rc;
    }
    return FDW_OK;
}

// Non-temporal streaming pays off once a member's planes (state in and out, coefficients)
// are well beyond the last-level cache; below that (a 2048^2 FP64 solve, the 4096^2 FP32
// members of a family) normal accesses keep part of the set cached from one launch to the
// next and measure faster.
bool stream_nt(const fdw_ctx* c)
{
    if (c->stream_policy) return c->stream_policy == 1 || c->stream_policy == 3;
    size_t b = 0;
    for (const HostMember& hm : c->m)
        b = std::max(b, (size_t)(hm.face ? 6 : 5) * hm.ld * hm.ny * elem_size(c->dtype));
    return b > 2 * kLastLevelCacheBytes;
}

// non-temporal loads of the state rows (float launches; the automatic policy follows the stores)
bool nt_loads(const fdw_ctx* c)
{
    if (c->stream_policy) return c->stream_policy == 1 || c->stream_policy == 4;
    return stream_nt(c);
}

void sync_member_dev(fdw_ctx* c, int i)
{
    HostMember& hm = c->m[i];
    MemberDev& md = c->tab[i];
    md.stream_nt = stream_nt(c) ? 1 : 0;
    md.cur0 = hm.cur ^ (int)(c->launches & 1);
    md.n_offset = hm.n - c->ctx_step;
    md.face = hm.face;
    md.R = hm.R;
    md.traces = hm.traces;
}

struct AdjLayout {
    size_t plane = 0, plane64 = 0;
    int64_t nck = 0;
    size_t total = 0;
};

AdjLayout adj_layout(const fdw_ctx* c, const HostMember& hm, int ck)
{
    AdjLayout L;
    L.plane = align_up(plane_alloc(hm.ld, hm.ny, elem_size(c->dtype)), kAlign);
    L.plane64 = align_up((size_t)hm.ld * hm.ny * sizeof(double), kAlign);
    L.nck = (hm.N >= 1 && ck >= 1) ? (hm.N - 1) / ck : 0;  // checkpoints at ck, 2ck, ... < N
    size_t b = align_up(sizeof(MemberDev), kAlign);
    b += 8 * L.plane + 2 * L.plane64;
    b += (size_t)(2 * L.nck) * L.plane;
    b += align_up(sizeof(int) * 2 * kMaxReceivers, kAlign);
    b += align_up(sizeof(int) * (size_t)(hm.ny + 1), kAlign);
    b += 2 * align_up(sizeof(int) * kMaxReceivers, kAlign);
    b += align_up(sizeof(int) * 16, kAlign);
    L.total = b;
    return L;
}


// Adjoint workspace: a MemberDev slot, the reverse state planes (u, du, lam, mu; two of each),
// two FP64 gradient planes, the checkpoints (u, du) at steps ck, 2ck, ... < N, and the
// receiver tables.
struct AdjPlanes {
    MemberDev* rep_dev = nullptr;
    void* planes_begin = nullptr;
    void* FU[2];
    void* FD[2];
    void* LA[2];
    void* MU[2];
    double* G1 = nullptr;
    double* G2 = nullptr;
    std::vector<void*> CU, CD;
    int* rec = nullptr;
    int* rowptr = nullptr;
    int* rcol = nullptr;
    int* rid = nullptr;
    int* status = nullptr;
};

AdjPlanes adj_carve(const fdw_ctx* c, const HostMember& hm, const AdjLayout& L, void* ws)
{
    AdjPlanes P;
    char* w = (char*)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = w + off;
        off += align_up(bytes, kAlign);
        return (void*)p;
    };
    const size_t es = elem_size(c->dtype);
    P.rep_dev = (MemberDev*)take(sizeof(MemberDev));
    P.planes_begin = w + off;
    auto plane = [&]() { return plane_origin(take(L.plane), hm.ld, es); };
    for (int k = 0; k < 2; ++k) P.FU[k] = plane();
    for (int k = 0; k < 2; ++k) P.FD[k] = plane();
    for (int k = 0; k < 2; ++k) P.LA[k] = plane();
    for (int k = 0; k < 2; ++k) P.MU[k] = plane();
    P.G1 = (double*)take(L.plane64);
    P.G2 = (double*)take(L.plane64);
    P.CU.resize(L.nck);
    P.CD.resize(L.nck);
    for (int64_t k = 0; k < L.nck; ++k) {
        P.CU[k] = plane();
        P.CD[k] = plane();
    }
    P.rec = (int*)take(sizeof(int) * 2 * kMaxReceivers);
    P.rowptr = (int*)take(sizeof(int) * (size_t)(hm.ny + 1));
    P.rcol = (int*)take(sizeof(int) * kMaxReceivers);
    P.rid = (int*)take(sizeof(int) * kMaxReceivers);
    P.status = (int*)take(sizeof(int) * 16);
    return P;
}

// Copy the state (u^n, du^n) of a member into checkpoint slot n / ck - 1.
int store_checkpoint(fdw_ctx* c, const HostMember& hm, void* cu, void* cd, const void* u, const void* d,
                     hipStream_t s)
{
    const size_t es = elem_size(c->dtype);
    const size_t pad = (size_t)kPadRowsTop * hm.ld * es;
    const size_t bytes = plane_alloc(hm.ld, hm.ny, es);
    HIPCHK(c, hipMemcpyAsync((char*)cu - pad, (const char*)u - pad, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync((char*)cd - pad, (const char*)d - pad, bytes, hipMemcpyDeviceToDevice, s));
    return FDW_OK;
}

// Forward-run hook: when the recorded member has just reached a checkpoint step, store it.
int record_hook(fdw_ctx* c, hipStream_t s)
{
    if (c->rec.member < 0) return FDW_OK;
    const HostMember& hm = c->m[c->rec.member];
    const int ck = c->rec.ck;
    if (hm.n < 1 || hm.n % ck != 0 || hm.n >= hm.N) return FDW_OK;
    const AdjLayout L = adj_layout(c, hm, ck);
    const int64_t k = hm.n / ck - 1;
    if (k >= L.nck) return FDW_OK;
    // slot addresses follow the workspace layout of the adjoint
    const size_t es = elem_size(c->dtype);
    char* base = (char*)c->rec.ws + align_up(sizeof(MemberDev), kAlign) + 8 * L.plane + 2 * L.plane64;
    void* cu = plane_origin(base + (size_t)(2 * k) * L.plane, hm.ld, es);
    void* cd = plane_origin(base + (size_t)(2 * k + 1) * L.plane, hm.ld, es);
    return store_checkpoint(c, hm, cu, cd, hm.u[hm.cur], hm.d[hm.cur], s);
}

// Checkpoint slot of the recorded member for step n (false: no checkpoint is stored there).
bool checkpoint_slot(fdw_ctx* c, const HostMember& hm, int64_t n, void** cu, void** cd)
{
    const int ck = c->rec.ck;
    if (c->rec.member < 0 || n < 1 || n % ck != 0 || n >= hm.N) return false;
    const AdjLayout L = adj_layout(c, hm, ck);
    const int64_t k = n / ck - 1;
    if (k >= L.nck) return false;
    const size_t es = elem_size(c->dtype);
    char* base = (char*)c->rec.ws + align_up(sizeof(MemberDev), kAlign) + 8 * L.plane + 2 * L.plane64;
    *cu = plane_origin(base + (size_t)(2 * k) * L.plane, hm.ld, es);
    *cd = plane_origin(base + (size_t)(2 * k + 1) * L.plane, hm.ld, es);
    return true;
}

// Steps until the recorded member's next checkpoint (a time block must not cross it).
int64_t steps_to_checkpoint(const fdw_ctx* c)
{
    if (c->rec.member < 0) return INT64_MAX;
    const int64_t n = c->m[c->rec.member].n;
    return c->rec.ck - (n % c->rec.ck);
}

template <typename T>
int do_start(fdw_ctx* c, int i, double* energy_out)
{
    HostMember& hm = c->m[i];
    MemberDev& md = c->tab[i];
    HIPCHK(c, launch_start<T>(&md, c->tab_dev + i, hm.u0, hm.u1, (T)hm.tau, energy_out != nullptr, 0, energy_out,
                              c->red, c->stream));
    hm.n = 1;
    hm.cur = 0;
    if (hm.R > 0 && hm.traces && 1 < hm.N + 1)
        HIPCHK(c, launch_gather<T>(hm.u[0], hm.ld, hm.rec_ij, hm.R, (char*)hm.traces + (size_t)hm.R * sizeof(T),
                                   c->stream));
    return record_hook(c, c->stream);
}

// One streaming launch of K steps over members [first, first + nm) (all members when nm == count).
template <typename T>
int launch_block(fdw_ctx* c, int first, int nm, int K, bool energy, bool trace, hipStream_t s, int eslot = 0)
{
    StepArgs a;
    a.eslot = eslot;
    a.table = c->tab_dev;
    a.first = first;
    a.nmembers = nm;
    a.block_offset = c->tab[first].block_base;
    int total = 0;
    for (int i = first; i < first + nm; ++i) total += c->tab[i].blocks;
    a.total_blocks = total;
    a.parity = (int)(c->launches & 1);
    a.want_energy = energy ? 1 : 0;
    a.want_trace = trace ? 1 : 0;
    a.ctx_step = c->ctx_step;
    a.stream_nt = nt_loads(c) ? 1 : 0;
    a.reverse = (c->item_order && a.parity) ? 1 : 0;
    int face_mode = c->m[first].face;
    for (int i = first; i < first + nm; ++i)
        if (c->m[i].face != face_mode) face_mode = -1;
    if (c->tiles_now && trace) return fail(c, FDW_ENOTSUP, "tile decomposition with receiver traces");
    auto launch = [&](const StepArgs& sa, int face, int grid) {
        return c->tiles_now ? launch_step_tile<T>(sa, K, face, tile_rows(c) / kTileRowsPerWave, grid, s)
                            : launch_step<T>(sa, K, c->C, face, grid, s);
    };
    if (face_mode < 0) {
        // mixed layouts in one batch: launch per member
        for (int i = first; i < first + nm; ++i) {
            a.first = i;
            a.nmembers = 1;
            a.block_offset = c->tab[i].block_base;
            a.total_blocks = c->tab[i].blocks;
            HIPCHK(c, launch(a, c->m[i].face, a.total_blocks));
        }
        return FDW_OK;
    }
    const bool timed = c->timing && s == c->stream;
    if (timed) {
        while (c->ev_pool.size() < c->ev_used + 2) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
        HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used], s));
    }
    HIPCHK(c, launch(a, face_mode, total));
    if (timed) {
        HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used + 1], s));
        c->ev_used += 2;
    }
    return FDW_OK;
}

bool any_trace(const fdw_ctx* c)
{
    for (const HostMember& hm : c->m)
        if (hm.R > 0 && hm.traces) return true;
    return false;
}

// The main loop of step_n once every member is in lock-step: `steps` steps, energies of the
// first of them land at energy_dev[m * stride + koff + ...].
template <typename T>
int run_blocks(fdw_ctx* c, int64_t steps, double* energy_dev, int64_t stride, int64_t koff, hipStream_t s)
{
    const int K = choose_K(c);
    const bool trace = any_trace(c);
    int64_t left = steps, k = koff;
    int curK = -1;
    // slots every member holds at the current decomposition
    auto group_cap = [&]() {
        int g = kMaxEnergySlots;
        for (int i = 0; i < c->count; ++i) g = std::min(g, energy_group_cap(c, i));
        return g;
    };
    int gmax = group_cap();
    int gK = 0, gcount = 0;
    int64_t gstart = 0;
    // Checkpoint recording: a launch that ends on a checkpoint step (other than the call's last)
    // writes the recorded member's state straight into the checkpoint slot, and the next launch
    // reads it from there - the member's table pointers are redirected around those launches
    // instead of copying the state after them (two planes read and written per checkpoint).
    const int rm = c->rec.member;
    void* prev_u = nullptr;
    void* prev_d = nullptr;  // slot the previous launch wrote (null: the ping-pong buffer)
    auto point_member = [&](void* in_u, void* in_d, void* out_u, void* out_d) -> int {
        HostMember& hm = c->m[rm];
        MemberDev& md = c->tab[rm];
        const int i = hm.cur;
        if (md.u[i] == in_u && md.d[i] == in_d && md.u[i ^ 1] == out_u && md.d[i ^ 1] == out_d) return FDW_OK;
        md.u[i] = in_u;
        md.d[i] = in_d;
        md.u[i ^ 1] = out_u;
        md.d[i ^ 1] = out_d;
        return push_member(c, rm, s);
    };
    while (left > 0) {
        const int Kb = (int)std::min<int64_t>(std::min<int64_t>(K, left), steps_to_checkpoint(c));
        // energies: consecutive time blocks of one length write their partials into successive
        // slots; one finalisation sums a full group (or the group before a change of length,
        // and the last one).  It runs before the table is laid out for a new length: the sums
        // run over the waves of the decomposition that wrote the partials.
        if (energy_dev && gcount > 0 && (Kb != gK || gcount == gmax)) {
            HIPCHK(c, launch_energy_finalize<T>(c->tab_dev, 0, c->count, gK, energy_dev, stride, gstart,
                                                health_word(c), s, 0, gcount));
            gcount = 0;
        }
        if (Kb != curK) {
            int rc = layout_for_K(c, Kb, c->S_eff, s);
            if (rc) return rc;
            curK = Kb;
            gmax = group_cap();
        }
        if (energy_dev && gcount == 0) {
            gK = Kb;
            gstart = k;
        }
        bool direct = false;
        if (rm >= 0) {
            const HostMember& hm = c->m[rm];
            void* su = nullptr;
            void* sd = nullptr;
            direct = left > Kb && checkpoint_slot(c, hm, hm.n + Kb, &su, &sd);
            int rc = point_member(prev_u ? prev_u : hm.u[hm.cur], prev_d ? prev_d : hm.d[hm.cur],
                                  direct ? su : hm.u[hm.cur ^ 1], direct ? sd : hm.d[hm.cur ^ 1]);
            if (rc) return rc;
            prev_u = direct ? su : nullptr;
            prev_d = direct ? sd : nullptr;
        }
        int rc = launch_block<T>(c, 0, c->count, Kb, energy_dev != nullptr, trace, s, energy_dev ? gcount : 0);
        if (rc) return rc;
        if (energy_dev) ++gcount;
        c->ctx_step += Kb;
        c->launches += 1;
        for (HostMember& hm : c->m) {
            hm.n += Kb;
            hm.cur ^= 1;
        }
        if (!direct) {
            rc = record_hook(c, s);  // a copy, where the state is in the ping-pong buffer
            if (rc) return rc;
        }
        left -= Kb;
        k += Kb;
    }
    if (energy_dev && gcount > 0)
        HIPCHK(c, launch_energy_finalize<T>(c->tab_dev, 0, c->count, gK, energy_dev, stride, gstart, health_word(c), s,
                                            0, gcount));
    if (rm >= 0) {
        // the call's last launch wrote the ping-pong buffer: the table points at the member's own
        // buffers again
        const HostMember& hm = c->m[rm];
        int rc = point_member(hm.u[hm.cur], hm.d[hm.cur], hm.u[hm.cur ^ 1], hm.d[hm.cur ^ 1]);
        if (rc) return rc;
    }
    if (curK != K) {
        // leave the table in the main configuration
        int rc = layout_for_K(c, K, c->S_eff, s);
        if (rc) return rc;
    }
    return FDW_OK;
}

// Time block of the persistent kernel (instantiated for 1, 2, 4, 8).
int persistent_K(const fdw_ctx* c)
{
    const int Kc = choose_K(c);
    return Kc >= 8 ? 8 : (Kc >= 4 ? 4 : (Kc >= 2 ? 2 : 1));
}

// The main loop of step_n as one cooperative launch per kPersistentPhases time blocks (then the
// remaining steps as ordinary launches).  Energies as in run_blocks: the launch sums the
// energies of all but its last time block itself; that one is summed by k_energy_finalize.
template <typename T>
int run_persistent(fdw_ctx* c, int64_t steps, double* energy_dev, int64_t stride, int64_t koff, hipStream_t s)
{
    const int K = persistent_K(c);
    int face_mode = c->m[0].face;
    for (const HostMember& hm : c->m)
        if (hm.face != face_mode) return fail(c, FDW_ENOTSUP, "persistent batch needs one coefficient layout");
    int rc = layout_for_K(c, K, c->S_eff, s);
    if (rc) return rc;
    const int64_t phases = steps / K;
    const int64_t tail = steps - phases * K;
    int total = 0;
    for (const MemberDev& md : c->tab) total += md.blocks;
    int grid = std::min(total, persistent_max_blocks<T>(K, c->C, face_mode, energy_dev != nullptr));
    if (grid < 1) return fail(c, FDW_EHIP, "persistent launch: no resident blocks");
    int64_t k = koff;
    for (int64_t done = 0; done < phases;) {
        const int ph = (int)std::min<int64_t>(kPersistentPhases, phases - done);
        HIPCHK(c, launch_fill_bytes(c->barrier, (size_t)kPersistentCtlInts * sizeof(int), s));
        StepArgs a;
        a.eslot = 0;
        a.table = c->tab_dev;
        a.first = 0;
        a.nmembers = c->count;
        a.block_offset = 0;
        a.total_blocks = total;
        a.parity = (int)(c->launches & 1);
        a.want_energy = energy_dev ? 1 : 0;
        a.want_trace = 0;
        a.ctx_step = c->ctx_step;
        a.stream_nt = nt_loads(c) ? 1 : 0;
        a.reverse = 0;
        PersistentExtra x;
        x.energy_base = energy_dev;
        x.energy_stride = stride;
        x.energy_offset = k;
        x.health = health_word(c);
        x.err = sync_err_word(c);
        HIPCHK(c, launch_step_persistent<T>(a, K, c->C, face_mode, ph, grid, c->barrier, x, s));
        if (energy_dev)
            HIPCHK(c, launch_energy_finalize<T>(c->tab_dev, 0, c->count, K, energy_dev, stride, k + (int64_t)(ph - 1) * K,
                                                health_word(c), s, (ph - 1) & 1));
        c->ctx_step += (int64_t)ph * K;
        c->launches += ph;
        for (HostMember& hm : c->m) {
            hm.n += (int64_t)ph * K;
            if (ph & 1) hm.cur ^= 1;
        }
        done += ph;
        k += (int64_t)ph * K;
    }
    if (tail > 0) return run_blocks<T>(c, tail, energy_dev, stride, k, s);
    if (choose_K(c) != K) return layout_for_K(c, choose_K(c), c->S_eff, s);
    return FDW_OK;
}

// Host bookkeeping of a replayed launch sequence (what run_blocks / run_persistent update).
void replay_bookkeeping(fdw_ctx* c, int64_t steps, bool persistent)
{
    int64_t l = steps;
    if (persistent) {
        const int K = persistent_K(c);
        const int64_t phases = l / K;
        c->ctx_step += phases * K;
        c->launches += phases;
        for (HostMember& hm : c->m) {
            hm.n += phases * K;
            if (phases & 1) hm.cur ^= 1;
        }
        l -= phases * K;
    }
    const int K = choose_K(c);
    while (l > 0) {
        const int Kb = (int)std::min<int64_t>(K, l);
        c->ctx_step += Kb;
        c->launches += 1;
        for (HostMember& hm : c->m) {
            hm.n += Kb;
            hm.cur ^= 1;
        }
        l -= Kb;
    }
}

// Whether a step_n call runs the small-grid tile kernel: not with receiver traces (the streaming
// kernel records them) or the persistent launch; automatically where every member has at most
// kTileAutoNodes nodes (there the streaming kernel's few, long work items leave much of the
// device idle: measured faster from 256^2 to 1024^2 - at 1024^2 by 7% in FP64, 14% in FP32).
constexpr int64_t kTileAutoNodes = (int64_t)1024 * 1024;
bool want_tiles(const fdw_ctx* c)
{
    if (c->tile_mode == 1 || c->batch_mode == 1 || any_trace(c)) return false;
    if (c->tile_mode == 2) return true;
    for (const HostMember& hm : c->m)
        if ((int64_t)hm.nx * hm.ny > kTileAutoNodes) return false;
    return true;
}

template <typename T>
int step_n_impl(fdw_ctx* c, int64_t n, double* energy_dev)
{
    for (int i = 0; i < c->count; ++i)
        if (!c->m[i].coeff) return fail(c, FDW_ESTATE, "fdw_set_coeff has not been called for member " + std::to_string(i));
    if (n == 0) return FDW_OK;
    {
        // both kernels produce the same states bit for bit: the choice may change between calls
        const bool tiles = want_tiles(c);
        if (tiles != c->tiles_now) {
            c->tiles_now = tiles;
            const int rc = layout_for_K(c, choose_K(c), c->S_eff);
            if (rc) return rc;
        }
    }
    bool any0 = false, any1 = false;
    for (const HostMember& hm : c->m) (hm.n == 0 ? any0 : any1) = true;
    int64_t done = 0;
    if (any0 || any1) {
        if (any0) {
            // members at n = 0 take the start step; the others one single-member step, so that
            // all are in lock-step afterwards
            for (int i = 0; i < c->count; ++i) {
                HostMember& hm = c->m[i];
                double* e = energy_dev ? energy_dev + (int64_t)c->tab[i].energy_row * n : nullptr;
                if (hm.n == 0) {
                    int rc = do_start<T>(c, i, e);
                    if (rc) return rc;
                } else {
                    int rc = layout_for_K(c, 1, c->S_eff);
                    if (rc) return rc;
                    rc = launch_block<T>(c, i, 1, 1, e != nullptr, any_trace(c), c->stream);
                    if (rc) return rc;
                    if (e)
                        HIPCHK(c, launch_energy_finalize<T>(c->tab_dev, i, 1, 1, energy_dev, n, 0, health_word(c),
                                                            c->stream));
                    // this member alone advanced: its parity and offset move relative to the context
                    hm.n += 1;
                    hm.cur ^= 1;
                }
            }
            done = 1;
            for (int i = 0; i < c->count; ++i) sync_member_dev(c, i);
            int rc = layout_for_K(c, choose_K(c), c->S_eff);
            if (rc) return rc;
        }
    }
    const int64_t left = n - done;
    if (left <= 0) return FDW_OK;
    const bool recording = c->rec.member >= 0;
    // traces and checkpoint recording need the per-time-block launches
    const bool persistent = c->batch_mode == 1 && !any_trace(c) && !recording;
    c->used_persistent = persistent;
    if (c->use_graph && !any_trace(c) && !recording) {
        // The launch sequence of the main loop depends only on (steps, K, energy pointer and
        // offset, launch parity, batch mode); capture it once and replay it.
        // The captured sequence rewrites the member table with the pair index each member's
        // state sits in (cur0); with up to 64 members these are part of the key, so a graph is
        // replayed only where they match and returning a member to step 0 need not drop graphs.
        uint64_t pairs = 0;
        if (c->count <= 64)
            for (int i = 0; i < c->count; ++i) pairs |= (uint64_t)(c->tab[i].cur0 & 1) << i;
        const auto key = std::make_tuple(left, choose_K(c) + 16 * (int)persistent + 32 * (int)c->tiles_now,
                                         (const double*)energy_dev,
                                         (int)(c->launches & 1), (int)done, pairs);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = persistent ? run_persistent<T>(c, left, energy_dev, n, done, c->cap_stream)
                                : run_blocks<T>(c, left, energy_dev, n, done, c->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) {
                if (g) hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(c, FDW_EHIP, std::string("capture: ") + hipGetErrorString(e));
            GraphEntry ge;
            e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return fail(c, FDW_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
            it = c->graphs.emplace(key, ge).first;
        } else {
            replay_bookkeeping(c, left, persistent);
        }
        HIPCHK(c, hipGraphLaunch(it->second.exec, c->stream));
        return FDW_OK;
    }
    if (persistent) return run_persistent<T>(c, left, energy_dev, n, done, c->stream);
    return run_blocks<T>(c, left, energy_dev, n, done, c->stream);
}

}  // namespace

// ---- families that mix storage types (one child context per type) --------------------------
bool mixed_types(const fdw_problem* p, int count)
{
    for (int i = 1; i < count; ++i)
        if (p[i].dtype != p[0].dtype) return true;
    return false;
}

// the members of one storage type, in family order
void members_of_type(const fdw_problem* p, int count, int dtype, std::vector<fdw_problem>* ps, std::vector<int>* idx)
{
    for (int i = 0; i < count; ++i)
        if (p[i].dtype == dtype) {
            ps->push_back(p[i]);
            idx->push_back(i);
        }
}

// a child's status, with its message, as the parent's
int fwd(fdw_ctx* c, const fdw_ctx* child, int rc)
{
    if (rc) c->err = child->err;
    return rc;
}

// =============================================================================================
// C-ABI
// =============================================================================================
extern "C" {

const char* fdw_status_string(int s)
{
    switch (s) {
    case FDW_OK: return "ok";
    case FDW_EINVAL: return "invalid argument";
    case FDW_ECFL: return "time step above the stability bound";
    case FDW_ESTATE: return "call out of order";
    case FDW_ENOMEM: return "workspace too small";
    case FDW_EHIP: return "HIP runtime error";
    case FDW_EUNSTABLE: return "non-finite energy";
    case FDW_ENOTSUP: return "not supported";
    case FDW_ESYNC: return "grid barrier timed out";
    default: return "unknown status";
    }
}

const char* fdw_last_error(const fdw_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t fdw_workspace_bytes(const fdw_problem* problems, int32_t count)
{
    if (!problems || count < 1) return 0;
    if (mixed_types(problems, count)) {
        // one child context per storage type, each in its own (aligned) part of the workspace
        size_t b = 0;
        for (int t = FDW_F32; t <= FDW_F64; ++t) {
            std::vector<fdw_problem> ps;
            std::vector<int> idx;
            members_of_type(problems, count, t, &ps, &idx);
            const size_t bt = ps.empty() ? 0 : fdw_workspace_bytes(ps.data(), (int)ps.size());
            if (!ps.empty() && bt == 0) return 0;
            b += align_up(bt, kAlign);
        }
        for (int i = 0; i < count; ++i)
            if (problems[i].dtype != FDW_F32 && problems[i].dtype != FDW_F64) return 0;
        return b;
    }
    size_t b = header_bytes(count);
    std::string why;
    for (int i = 0; i < count; ++i) {
        if (!problem_ok(problems[i], &why, nullptr)) return 0;
        if (problems[i].dtype != problems[0].dtype) return 0;
        b += member_bytes(problems[i]);
    }
    return b;
}

int fdw_init(const fdw_problem* problems, int32_t count, void* workspace, size_t ws_bytes, const void* const* u0,
             const void* const* u1, void* hip_stream, fdw_ctx** out)
{
    if (!out) return FDW_EINVAL;
    *out = nullptr;
    if (!problems || count < 1 || !workspace || !u0 || !u1) return FDW_EINVAL;
    if (((uintptr_t)workspace) % kAlign) return FDW_EINVAL;
    std::string why;
    if (mixed_types(problems, count)) {
        const size_t need = fdw_workspace_bytes(problems, count);
        if (need == 0) return FDW_EINVAL;
        if (ws_bytes < need) return FDW_ENOMEM;
        for (int i = 0; i < count; ++i)
            if (!u0[i] || !u1[i]) return FDW_EINVAL;
        fdw_ctx* c = new fdw_ctx();
        c->mixed = true;
        c->count = count;
        c->dtype = -1;
        c->stream = (hipStream_t)hip_stream;
        c->sub_of.assign(count, 0);
        c->sub_idx.assign(count, 0);
        size_t off = 0;
        for (int t = FDW_F32; t <= FDW_F64; ++t) {
            std::vector<fdw_problem> ps;
            std::vector<int> idx;
            members_of_type(problems, count, t, &ps, &idx);
            std::vector<const void*> a0, a1;
            for (size_t j = 0; j < idx.size(); ++j) {
                c->sub_of[idx[j]] = t;
                c->sub_idx[idx[j]] = (int)j;
                a0.push_back(u0[idx[j]]);
                a1.push_back(u1[idx[j]]);
            }
            const size_t bt = fdw_workspace_bytes(ps.data(), (int)ps.size());
            int rc = fdw_init(ps.data(), (int)ps.size(), (char*)workspace + off, bt, a0.data(), a1.data(), hip_stream,
                              &c->sub[t]);
            if (rc) {
                fdw_destroy(c);
                return rc;
            }
            off += align_up(bt, kAlign);
            // energies go to the family's row of each member
            fdw_ctx* ch = c->sub[t];
            for (size_t j = 0; j < idx.size(); ++j) {
                ch->tab[j].energy_row = idx[j];
                rc = push_member(ch, (int)j);
                if (rc) {
                    fdw_destroy(c);
                    return rc;
                }
            }
        }
        *out = c;
        return FDW_OK;
    }
    for (int i = 0; i < count; ++i) {
        if (!problem_ok(problems[i], &why, nullptr)) return FDW_EINVAL;
        if (!u0[i] || !u1[i]) return FDW_EINVAL;
    }
    const size_t need = fdw_workspace_bytes(problems, count);
    if (need == 0) return FDW_EINVAL;
    if (ws_bytes < need) return FDW_ENOMEM;

    fdw_ctx* c = new fdw_ctx();
    c->count = count;
    c->dtype = problems[0].dtype;
    c->C = default_cols_per_lane(c->dtype);
    c->adjC = (c->dtype == FDW_F64) ? 1 : 2;
    c->adjK = 6;  // the deepest reverse blocks at two waves per SIMD (the default lane layouts allow it)
    c->stream = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return FDW_EHIP;
    }
    char* w = (char*)workspace;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = w + off;
        off += align_up(bytes, kAlign);
        return (void*)p;
    };
    c->tab_dev = (MemberDev*)take(sizeof(MemberDev) * (size_t)count);
    c->red = (double*)take(sizeof(double) * (4 * kRedBlocks + 16));
    c->status = (int*)take(sizeof(int) * 16);
    c->barrier = (int*)take(sizeof(int) * kPersistentCtlInts);
    c->scal = (double*)take(sizeof(double) * (size_t)std::max(count, 1) * 2);
    c->m.resize(count);
    c->tab.resize(count);
    for (int i = 0; i < count; ++i) {
        HostMember& hm = c->m[i];
        const fdw_problem& p = problems[i];
        hm.p = p;
        hm.nx = p.nx;
        hm.ny = p.ny;
        hm.ld = pitch_of(p.nx);
        problem_ok(p, &why, &hm.N);
        hm.dx = (p.x1 - p.x0) / (p.nx - 1);
        hm.dy = (p.y1 - p.y0) / (p.ny - 1);
        hm.tau = p.tau;
        const size_t es = elem_size(c->dtype);
        hm.plane_bytes = align_up(plane_alloc(hm.ld, p.ny, es), kAlign);
        auto plane = [&]() { return plane_origin(take(hm.plane_bytes), hm.ld, es); };
        for (int k = 0; k < 2; ++k) hm.u[k] = plane();
        for (int k = 0; k < 2; ++k) hm.d[k] = plane();
        hm.h = plane();
        hm.hy = plane();
        hm.u0 = plane();
        hm.u1 = plane();
        hm.rec_ij = (int*)take(sizeof(int) * 2 * kMaxReceivers);
        hm.rowptr = (int*)take(sizeof(int) * (size_t)(p.ny + 1));
        hm.rcol = (int*)take(sizeof(int) * kMaxReceivers);
        hm.rid = (int*)take(sizeof(int) * kMaxReceivers);
        hm.epart_stride = max_strips(p.nx) * ((p.ny + kMinSegRows - 1) / kMinSegRows);
        hm.eslots = energy_slots(p);
        hm.epart = (double*)take(sizeof(double) * (size_t)hm.eslots * kMaxTimeBlock * (size_t)hm.epart_stride);

        MemberDev& md = c->tab[i];
        std::memset(&md, 0, sizeof(md));
        md.energy_row = i;
        md.nx = hm.nx;
        md.ny = hm.ny;
        md.ld = hm.ld;
        md.trace_rows = hm.N + 1;
        md.ax = 0.5 * p.tau * p.tau / (hm.dx * hm.dx);
        md.ay = 0.5 * p.tau * p.tau / (hm.dy * hm.dy);
        md.escale = hm.dx * hm.dy / (p.tau * p.tau);
        for (int k = 0; k < 2; ++k) {
            md.u[k] = hm.u[k];
            md.d[k] = hm.d[k];
        }
        md.h = hm.h;
        md.hy = hm.hy;
        md.rec_rowptr = hm.rowptr;
        md.rec_col = hm.rcol;
        md.rec_id = hm.rid;
        md.epart = hm.epart;
        md.epart_stride = hm.epart_stride;
    }
    if (off > ws_bytes) {
        fdw_destroy(c);
        return FDW_ENOMEM;
    }
    int rc = FDW_OK;
    // zero everything, then bring in the initial data (boundary ring zeroed)
    if (launch_fill_bytes(workspace, off, c->stream) != hipSuccess) rc = FDW_EHIP;
    for (int i = 0; i < count && rc == FDW_OK; ++i) {
        HostMember& hm = c->m[i];
        hipError_t e = (c->dtype == FDW_F32) ? launch_copy_in<float>(u0[i], hm.nx, hm.ny, hm.u0, hm.ld, 1, c->stream)
                                             : launch_copy_in<double>(u0[i], hm.nx, hm.ny, hm.u0, hm.ld, 1, c->stream);
        if (e == hipSuccess)
            e = (c->dtype == FDW_F32) ? launch_copy_in<float>(u1[i], hm.nx, hm.ny, hm.u1, hm.ld, 1, c->stream)
                                      : launch_copy_in<double>(u1[i], hm.nx, hm.ny, hm.u1, hm.ld, 1, c->stream);
        if (e != hipSuccess) rc = FDW_EHIP;
    }
    if (rc == FDW_OK) {
        c->S_eff = choose_S(c);
        for (int i = 0; i < count; ++i) sync_member_dev(c, i);
        rc = layout_for_K(c, choose_K(c), c->S_eff);
    }
    if (rc != FDW_OK) {
        fdw_destroy(c);
        return rc;
    }
    *out = c;
    return FDW_OK;
}

void fdw_destroy(fdw_ctx* c)
{
    if (!c) return;
    for (fdw_ctx*& ch : c->sub) {
        fdw_destroy(ch);
        ch = nullptr;
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    for (auto& kv : c->graphs)
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

static int check_member(fdw_ctx* c, int32_t m)
{
    if (!c) return FDW_EINVAL;
    if (m < 0 || m >= c->count) return fail(c, FDW_EINVAL, "member index out of range");
    return FDW_OK;
}

static void invalidate_graphs(fdw_ctx* c)
{
    for (auto& kv : c->graphs)
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    c->graphs.clear();
}

int fdw_set_coeff(fdw_ctx* c, int32_t m, const void* h1, const void* h2)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed) return fwd(c, c->sub[c->sub_of[m]], fdw_set_coeff(c->sub[c->sub_of[m]], c->sub_idx[m], h1, h2));
    if (!h1) return fail(c, FDW_EINVAL, "h1 is NULL");
    HostMember& hm = c->m[m];
    const int face = h2 ? 1 : 0;
    MemberDev tmp = c->tab[m];
    tmp.face = face;
    hipError_t e = (c->dtype == FDW_F32) ? launch_prepare_coeff<float>(&tmp, h1, h2, face, c->red, c->stream)
                                         : launch_prepare_coeff<double>(&tmp, h1, h2, face, c->red, c->stream);
    HIPCHK(c, e);
    double st[4];
    HIPCHK(c, hipMemcpyAsync(st, c->red + 4 * kRedBlocks, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hm.coeff = false;
    if (st[3] != 0.0) return fail(c, FDW_EINVAL, "h contains non-finite values");
    const bool allow0 = (hm.p.flags & FDW_ALLOW_ZERO_H) != 0;
    if (allow0 ? !(st[0] >= 0.0) : !(st[0] > 0.0))
        return fail(c, FDW_EINVAL, allow0 ? "h must be >= 0" : "h must be > 0 (set FDW_ALLOW_ZERO_H to allow 0)");
    const double bound = hm.tau * hm.tau * (4.0 * st[1] / (hm.dx * hm.dx) + 4.0 * st[2] / (hm.dy * hm.dy));
    if (!(hm.p.flags & FDW_ALLOW_UNSTABLE) && bound > 4.0 * (1.0 + 1e-12)) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "tau^2 (4 max hx/dx^2 + 4 max hy/dy^2) = %.6g > 4 (max hx %.6g, max hy %.6g)",
                      bound, st[1], st[2]);
        return fail(c, FDW_ECFL, buf);
    }
    hm.face = face;
    hm.coeff = true;
    hm.n = 0;
    hm.cur = 0;
    if (c->rec.member == m) c->rec.member = -1;
    sync_member_dev(c, m);
    invalidate_graphs(c);
    return push_member(c, m);
}

int fdw_step_n(fdw_ctx* c, int64_t n, double* energy_dev)
{
    if (!c) return FDW_EINVAL;
    if (n < 0) return fail(c, FDW_EINVAL, "n must be >= 0");
    if (c->mixed) {
        // one launch sequence per storage type, one after the other on the stream; each writes
        // the energy rows of its own members
        for (fdw_ctx* ch : c->sub) {
            const int rc = fdw_step_n(ch, n, energy_dev);
            if (rc) return fwd(c, ch, rc);
        }
        return FDW_OK;
    }
    std::vector<int64_t> n_before;
    for (const HostMember& hm : c->m) n_before.push_back(hm.n);
    const bool check = energy_dev && c->check_energy && n > 0;
    // both words (failure detection, barrier timeout) start at zero; a test can mark the
    // barrier word as if the persistent launch had timed out (no kernel waits on it)
    HIPCHK(c, launch_fill_bytes(health_word(c), 2 * sizeof(int), c->stream));
    if (c->test_flag_barrier) HIPCHK(c, launch_set_int(sync_err_word(c), 1, c->stream));
    c->used_persistent = false;
    const int rc = (c->dtype == FDW_F32) ? step_n_impl<float>(c, n, energy_dev) : step_n_impl<double>(c, n, energy_dev);
    if (rc) return rc;
    // coincident receivers: the kernels recorded the first of each run; copy the others
    for (size_t i = 0; i < c->m.size(); ++i) {
        const HostMember& hm = c->m[i];
        if (hm.R <= 0 || !hm.traces || hm.ndup <= 0) continue;
        const int64_t lo = n_before[i] + 1, hi = std::min<int64_t>(hm.n, hm.N);
        HIPCHK(c, launch_trace_dups(hm.traces, (int)elem_size(c->dtype), hm.R, hm.rec_ij, hm.rid, lo, hi, c->stream));
    }
    if (check || c->used_persistent || c->test_flag_barrier) {
        // failure detection (the energies of this call) and the persistent launch's barrier word:
        // two words read back, the stream synchronised
        int h[2] = {0, 0};
        HIPCHK(c, hipMemcpyAsync(h, health_word(c), 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->test_flag_barrier = 0;
        if (h[1] & 1)
            return fail(c, FDW_ESYNC, "a grid barrier of the persistent launch timed out: the steps of this call are "
                                      "not valid");
        if (check && (h[0] & 1)) return fail(c, FDW_EUNSTABLE, "a non-finite energy was computed (the solution blew up)");
        if (check && (h[0] & 2)) return fail(c, FDW_EUNSTABLE, "the energy grew beyond 10x its first value in the call");
    }
    return FDW_OK;
}

int fdw_energy(fdw_ctx* c, double* energy_host)
{
    if (!c || !energy_host) return FDW_EINVAL;
    if (c->mixed) {
        std::vector<double> part[2];
        for (int t = 0; t < 2; ++t) {
            part[t].assign(c->sub[t]->count, 0.0);
            const int rc = fdw_energy(c->sub[t], part[t].data());
            if (rc) return fwd(c, c->sub[t], rc);
        }
        for (int i = 0; i < c->count; ++i) energy_host[i] = part[c->sub_of[i]][c->sub_idx[i]];
        return FDW_OK;
    }
    for (int i = 0; i < c->count; ++i)
        if (c->m[i].n < 1) return fail(c, FDW_ESTATE, "energy needs at least one step");
    for (int i = 0; i < c->count; ++i) {
        HostMember& hm = c->m[i];
        MemberDev md = c->tab[i];
        hipError_t e = (c->dtype == FDW_F32) ? launch_state_energy<float>(&md, hm.cur, c->red, c->scal + i, c->stream)
                                             : launch_state_energy<double>(&md, hm.cur, c->red, c->scal + i, c->stream);
        HIPCHK(c, e);
    }
    HIPCHK(c, hipMemcpyAsync(energy_host, c->scal, sizeof(double) * c->count, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->count; ++i)
        if (!std::isfinite(energy_host[i])) return fail(c, FDW_EUNSTABLE, "non-finite energy");
    return FDW_OK;
}

int fdw_record_traces(fdw_ctx* c, int32_t m, const int32_t* recv_ij, int32_t R, void* traces)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed)
        return fwd(c, c->sub[c->sub_of[m]], fdw_record_traces(c->sub[c->sub_of[m]], c->sub_idx[m], recv_ij, R, traces));
    HostMember& hm = c->m[m];
    if (R < 0 || R > kMaxReceivers) return fail(c, FDW_EINVAL, "R out of range");
    if (R == 0 || !traces) {
        hm.R = 0;
        hm.ndup = 0;
        hm.traces = nullptr;
        sync_member_dev(c, m);
        invalidate_graphs(c);
        return push_member(c, m);
    }
    if (!recv_ij) return fail(c, FDW_EINVAL, "recv_ij is NULL");
    HIPCHK(c, hipMemcpyAsync(hm.rec_ij, recv_ij, sizeof(int) * 2 * (size_t)R, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_receivers_csr(hm.rec_ij, R, hm.nx, hm.ny, hm.rowptr, hm.rcol, hm.rid, c->status, c->stream));
    int st[2] = {-1, 0};
    HIPCHK(c, hipMemcpyAsync(st, c->status, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (st[0] != 0) {
        hm.R = 0;
        hm.ndup = 0;
        hm.traces = nullptr;
        sync_member_dev(c, m);
        push_member(c, m);
        return fail(c, FDW_EINVAL, "receivers must be interior nodes (1 <= i <= nx-2, 1 <= j <= ny-2)");
    }
    hm.R = R;
    hm.ndup = st[1];
    hm.traces = traces;
    sync_member_dev(c, m);
    invalidate_graphs(c);
    rc = push_member(c, m);
    if (rc) return rc;
    if (hm.n <= hm.N) {
        const void* u = (hm.n == 0) ? hm.u0 : hm.u[hm.cur];
        const size_t es = elem_size(c->dtype);
        void* row = (char*)traces + (size_t)hm.n * R * es;
        HIPCHK(c, (c->dtype == FDW_F32) ? launch_gather<float>(u, hm.ld, hm.rec_ij, R, row, c->stream)
                                        : launch_gather<double>(u, hm.ld, hm.rec_ij, R, row, c->stream));
    }
    return FDW_OK;
}

int fdw_misfit(fdw_ctx* c, int32_t m, const void* traces, const double* d, int64_t rows, int32_t R, double* J_dev,
               double* trace_grad)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed)
        return fwd(c, c->sub[c->sub_of[m]],
                   fdw_misfit(c->sub[c->sub_of[m]], c->sub_idx[m], traces, d, rows, R, J_dev, trace_grad));
    if (!traces || !d || !J_dev || rows < 0 || R < 0) return fail(c, FDW_EINVAL, "bad misfit arguments");
    const int64_t n = rows * (int64_t)R;
    HIPCHK(c, (c->dtype == FDW_F32) ? launch_misfit<float>(traces, d, n, J_dev, trace_grad, c->red, c->stream)
                                    : launch_misfit<double>(traces, d, n, J_dev, trace_grad, c->red, c->stream));
    return FDW_OK;
}

int fdw_get_state(fdw_ctx* c, int32_t m, void* u, void* du, int64_t* n)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed) return fwd(c, c->sub[c->sub_of[m]], fdw_get_state(c->sub[c->sub_of[m]], c->sub_idx[m], u, du, n));
    HostMember& hm = c->m[m];
    if (n) *n = hm.n;
    const void* su = (hm.n == 0) ? hm.u0 : hm.u[hm.cur];
    if (u)
        HIPCHK(c, (c->dtype == FDW_F32) ? launch_copy_out<float>(su, hm.ld, hm.nx, hm.ny, u, c->stream)
                                        : launch_copy_out<double>(su, hm.ld, hm.nx, hm.ny, u, c->stream));
    if (du) {
        if (hm.n == 0)
            HIPCHK(c, launch_fill_bytes(du, (size_t)hm.nx * hm.ny * elem_size(c->dtype), c->stream));
        else
            HIPCHK(c, (c->dtype == FDW_F32) ? launch_copy_out<float>(hm.d[hm.cur], hm.ld, hm.nx, hm.ny, du, c->stream)
                                            : launch_copy_out<double>(hm.d[hm.cur], hm.ld, hm.nx, hm.ny, du, c->stream));
    }
    return FDW_OK;
}

int fdw_set_state(fdw_ctx* c, int32_t m, const void* u, const void* du, int64_t n)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed) return fwd(c, c->sub[c->sub_of[m]], fdw_set_state(c->sub[c->sub_of[m]], c->sub_idx[m], u, du, n));
    if (!u || !du || n < 1) return fail(c, FDW_EINVAL, "set_state needs u, du and n >= 1");
    HostMember& hm = c->m[m];
    if (!hm.coeff) return fail(c, FDW_ESTATE, "fdw_set_coeff first");
    HIPCHK(c, (c->dtype == FDW_F32) ? launch_copy_in<float>(u, hm.nx, hm.ny, hm.u[hm.cur], hm.ld, 1, c->stream)
                                    : launch_copy_in<double>(u, hm.nx, hm.ny, hm.u[hm.cur], hm.ld, 1, c->stream));
    HIPCHK(c, (c->dtype == FDW_F32) ? launch_copy_in<float>(du, hm.nx, hm.ny, hm.d[hm.cur], hm.ld, 1, c->stream)
                                    : launch_copy_in<double>(du, hm.nx, hm.ny, hm.d[hm.cur], hm.ld, 1, c->stream));
    hm.n = n;
    if (c->rec.member == m) c->rec.member = -1;
    sync_member_dev(c, m);
    invalidate_graphs(c);
    return push_member(c, m);
}

int fdw_member_distance(fdw_ctx* c, int32_t a, int32_t b, double* dist_host)
{
    int rc = check_member(c, a);
    if (rc) return rc;
    rc = check_member(c, b);
    if (rc) return rc;
    if (c->mixed) {
        if (c->sub_of[a] != c->sub_of[b]) return fail(c, FDW_ENOTSUP, "members of different storage types");
        fdw_ctx* ch = c->sub[c->sub_of[a]];
        return fwd(c, ch, fdw_member_distance(ch, c->sub_idx[a], c->sub_idx[b], dist_host));
    }
    if (!dist_host) return fail(c, FDW_EINVAL, "dist_host is NULL");
    const HostMember& A = c->m[a];
    const HostMember& B = c->m[b];
    if (A.nx != B.nx || A.ny != B.ny || A.p.x0 != B.p.x0 || A.p.x1 != B.p.x1 || A.p.y0 != B.p.y0 ||
        A.p.y1 != B.p.y1)
        return fail(c, FDW_EINVAL, "members differ in grid or domain");
    const void* ua = (A.n == 0) ? A.u0 : A.u[A.cur];
    const void* ub = (B.n == 0) ? B.u0 : B.u[B.cur];
    const double scale = A.dx * A.dy;
    HIPCHK(c, (c->dtype == FDW_F32) ? launch_diff_norm<float>(ua, ub, A.ld, A.nx, A.ny, scale, c->red, c->scal, c->stream)
                                    : launch_diff_norm<double>(ua, ub, A.ld, A.nx, A.ny, scale, c->red, c->scal, c->stream));
    double sq = 0.0;
    HIPCHK(c, hipMemcpyAsync(&sq, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *dist_host = std::sqrt(sq);
    return FDW_OK;
}

int fdw_reset(fdw_ctx* c, int32_t m)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed) return fwd(c, c->sub[c->sub_of[m]], fdw_reset(c->sub[c->sub_of[m]], c->sub_idx[m]));
    c->m[m].n = 0;
    c->m[m].cur = 0;
    if (c->rec.member == m) c->rec.member = -1;
    sync_member_dev(c, m);
    // graphs stay valid: their key holds every member's pair index (families of up to 64)
    if (c->count > 64) invalidate_graphs(c);
    return push_member(c, m);
}

int64_t fdw_steps_taken(const fdw_ctx* c, int32_t m)
{
    if (!c || m < 0 || m >= c->count) return -1;
    if (c->mixed) return fdw_steps_taken(c->sub[c->sub_of[m]], c->sub_idx[m]);
    return c->m[m].n;
}

int fdw_configure(fdw_ctx* c, int32_t key, int64_t v)
{
    if (!c) return FDW_EINVAL;
    if (c->mixed) {
        // applied to both storage types (a value must be valid for both)
        for (fdw_ctx* ch : c->sub) {
            const int rc = fdw_configure(ch, key, v);
            if (rc) return fwd(c, ch, rc);
        }
        return FDW_OK;
    }
    switch (key) {
    case FDW_CFG_TIME_BLOCK:
        if (v < 0 || v > kMaxTimeBlock || (c->dtype == FDW_F64 && c->C == 2 && v > 4) || (c->C == 4 && v > 6))
            return fail(c, FDW_EINVAL, "time block must be 0..8 (float with 2 columns per lane, double with 1), "
                                       "0..6 (float, 4 columns) or 0..4 (double, 2 columns)");
        c->K_cfg = (int)v;
        break;
    case FDW_CFG_SEGMENT_ROWS:
        if (v != 0 && (v < kMinSegRows || v > 4096)) return fail(c, FDW_EINVAL, "segment rows must be 0 or 8..4096");
        c->S_cfg = (int)v;
        c->S_eff = choose_S(c);
        break;
    case FDW_CFG_USE_GRAPH:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "use_graph must be 0 or 1");
        c->use_graph = (int)v;
        break;
    case FDW_CFG_BATCH_MODE:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "batch mode must be 0 or 1");
        c->batch_mode = (int)v;
        break;
    case FDW_CFG_TIMING:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "timing must be 0 or 1");
        c->timing = (int)v;
        break;
    case FDW_CFG_LANE_COLUMNS:
        if (v == 0) v = default_cols_per_lane(c->dtype);
        if (!(v == 2 || (v == 4 && c->dtype == FDW_F32) || (v == 1 && c->dtype == FDW_F64)))
            return fail(c, FDW_EINVAL, "lane columns must be 2 or 4 (float) / 1 or 2 (double)");
        if (v == 4 && c->K_cfg > 6) return fail(c, FDW_EINVAL, "4 columns per lane supports time blocks up to 6");
        if (v == 2 && c->dtype == FDW_F64 && c->K_cfg > 4)
            return fail(c, FDW_EINVAL, "double with 2 columns per lane supports time blocks up to 4");
        c->C = (int)v;
        break;
    case FDW_CFG_ADJ_TIME_BLOCK:
        if (v == 0) v = adj_narrow(c->dtype, c->adjC) ? 6 : 4;
        if (v < 1 || v > 6 || (v > 4 && !adj_narrow(c->dtype, c->adjC)))
            return fail(c, FDW_EINVAL, "adjoint time block must be 1..6 (double with 1 column per lane, float with 2) "
                                       "or 1..4");
        c->adjK = (int)v;
        break;
    case FDW_CFG_ADJ_LANE_COLUMNS:
        if (v == 0) v = (c->dtype == FDW_F64) ? 1 : 2;
        if (!(v == 2 || (v == 4 && c->dtype == FDW_F32) || (v == 1 && c->dtype == FDW_F64)))
            return fail(c, FDW_EINVAL, "adjoint lane columns must be 2 or 4 (float) / 1 or 2 (double)");
        if (c->adjK > 4 && !adj_narrow(c->dtype, (int)v))
            return fail(c, FDW_EINVAL, "adjoint time blocks above 4 need 1 (double) or 2 (float) columns per lane");
        c->adjC = (int)v;
        break;
    case FDW_CFG_ADJ_SEGMENT_ROWS:
        if (v != 0 && (v < kMinAdjSegRows || v > 4096)) return fail(c, FDW_EINVAL, "adjoint segment rows must be 0 or 16..4096");
        c->adjS_cfg = (int)v;
        break;
    case FDW_CFG_CHECK_ENERGY:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "check_energy must be 0 or 1");
        c->check_energy = (int)v;
        return FDW_OK;
    case FDW_CFG_TEST_BARRIER_FLAG:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "test_barrier_flag must be 0 or 1");
        c->test_flag_barrier = (int)v;
        return FDW_OK;
    case FDW_CFG_ITEM_ORDER:
        if (v != 0 && v != 1) return fail(c, FDW_EINVAL, "item order must be 0 or 1");
        c->item_order = (int)v;
        break;
    case FDW_CFG_STREAM_POLICY:
        if (v < 0 || v > 4) return fail(c, FDW_EINVAL, "stream policy must be 0..4");
        c->stream_policy = (int)v;
        break;
    case FDW_CFG_SMALL_TILES:
        if (v < 0 || v > 2) return fail(c, FDW_EINVAL, "small-grid tiles must be 0 (automatic), 1 (off) or 2 (on)");
        c->tile_mode = (int)v;
        break;
    case FDW_CFG_TILE_ROWS:
        if (v != 0 && v != 32 && v != 48 && v != 64) return fail(c, FDW_EINVAL, "tile rows must be 0, 32, 48 or 64");
        c->tile_rows = (int)v;
        break;
    default: return fail(c, FDW_EINVAL, "unknown configuration key");
    }
    invalidate_graphs(c);
    c->S_eff = choose_S(c);  // the automatic segment length depends on the time block
    for (int i = 0; i < c->count; ++i) sync_member_dev(c, i);
    return layout_for_K(c, choose_K(c), c->S_eff);
}

int fdw_kernel_time(fdw_ctx* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return FDW_EINVAL;
    if (c->mixed) {
        double tot = 0.0;
        int64_t nl = 0;
        for (fdw_ctx* ch : c->sub) {
            double t = 0.0;
            int64_t k = 0;
            const int rc = fdw_kernel_time(ch, &t, &k);
            if (rc) return fwd(c, ch, rc);
            tot += t;
            nl += k;
        }
        *ms = tot;
        *launches = nl;
        return FDW_OK;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[k], c->ev_pool[k + 1]));
        tot += t;
    }
    *ms = tot;
    *launches = (int64_t)(c->ev_used / 2);
    c->ev_used = 0;
    return FDW_OK;
}

int64_t fdw_get_config(const fdw_ctx* c, int32_t key)
{
    if (!c) return -1;
    if (c->mixed) return fdw_get_config(c->sub[FDW_F32], key);  // the FP32 members' configuration
    switch (key) {
    case FDW_CFG_TIME_BLOCK: return choose_K(c);
    case FDW_CFG_SEGMENT_ROWS: return c->S_eff;
    case FDW_CFG_USE_GRAPH: return c->use_graph;
    case FDW_CFG_BATCH_MODE: return c->batch_mode;
    case FDW_CFG_TIMING: return c->timing;
    case FDW_CFG_LANE_COLUMNS: return c->C;
    case FDW_CFG_ADJ_TIME_BLOCK: return c->adjK;
    case FDW_CFG_ADJ_LANE_COLUMNS: return c->adjC;
    case FDW_CFG_ADJ_SEGMENT_ROWS: return c->adjS_cfg;
    case FDW_CFG_CHECK_ENERGY: return c->check_energy;
    case FDW_CFG_TEST_BARRIER_FLAG: return c->test_flag_barrier;
    case FDW_CFG_ITEM_ORDER: return c->item_order;
    case FDW_CFG_STREAM_POLICY: return c->stream_policy;
    case FDW_CFG_SMALL_TILES: return c->tile_mode;
    case FDW_CFG_TILE_ROWS: return tile_rows(c);
    default: return -1;
    }
}

}  // extern "C"

// =============================================================================================
// Adjoint driver: forward replay with checkpoints, reverse sweep
// =============================================================================================
namespace {

int adjoint_K(const fdw_ctx* c) { return c->adjK; }

// Rows per reverse work item: 4K, at least 16 (measured best at 2048^2: 16 rows at K = 4,
// 24 at K = 6); short items keep many waves in flight for this register-heavy kernel, and the
// 2K halo rows of an item are largely shared with its neighbours through L2.
void adj_decompose(const fdw_ctx* c, const HostMember& hm, int K, int S, AdjArgs& a)
{
    const int C = c->adjC;
    const int Hx = ((K + C - 1) / C) * C;
    const int Wv = kWaveSize * C - 2 * Hx;
    a.seg_rows = S;
    a.segs = (hm.ny + S - 1) / S;
    a.strips = (hm.nx + Wv - 1) / Wv;
    a.waves = a.strips * a.segs;
}

// Rows per reverse work item.  The default is 4K (at least 16): every item recomputes 2K halo
// rows, so shorter items waste more, longer ones leave fewer items to fill the device.  When
// the 4K-row items of a small grid need a second round of resident waves (the reverse kernel
// holds two per SIMD), that round is mostly idle and costs a whole item time; the items are
// then lengthened, in steps of 8 rows up to 16K, until they fit in one round.
template <typename T>
int choose_adj_S(const fdw_ctx* c, const HostMember& hm, int K, bool split)
{
    if (c->adjS_cfg > 0) return c->adjS_cfg;
    const int cap = std::max(kMinAdjSegRows, (int)align_up((size_t)hm.ny, 8));
    const int S0 = std::min(std::max(kMinAdjSegRows, (4 * K + 7) / 8 * 8), cap);
    const int resident = adjoint_resident_waves<T>(K, c->adjC, hm.face != 0, split);
    AdjArgs a;
    adj_decompose(c, hm, K, S0, a);
    if (resident <= 0 || a.waves <= resident) return S0;
    for (int S = S0 + 8; S <= std::min(16 * K, cap); S += 8) {
        adj_decompose(c, hm, K, S, a);
        if (a.waves <= resident) return S;
    }
    return S0;
}

template <typename T>
int adjoint_impl(fdw_ctx* c, int m, const int32_t* recv_ij, int R, const double* tg, int ck, void* ws, size_t wsb,
                 double* g1_out, double* g2_out)
{
    HostMember& hm = c->m[m];
    const AdjLayout L = adj_layout(c, hm, ck);
    if (wsb < L.total) return fail(c, FDW_ENOMEM, "adjoint workspace too small");
    const AdjPlanes P = adj_carve(c, hm, L, ws);
    void* const* FU = P.FU;
    void* const* FD = P.FD;
    void* const* LA = P.LA;
    void* const* MU = P.MU;
    double* G1 = P.G1;
    double* G2 = P.G2;
    const std::vector<void*>& CU = P.CU;
    const std::vector<void*>& CD = P.CD;
    int* rec = P.rec;
    int* rowptr = P.rowptr;
    int* rcol = P.rcol;
    int* rid = P.rid;
    int* status = P.status;
    MemberDev* rep_dev = P.rep_dev;
    hipStream_t s = c->stream;
    const int64_t N = hm.N;
    // The forward run of this member stored every checkpoint into this workspace and stopped
    // at step N: reverse from its final state without a replay.
    const bool recorded = c->rec.member == m && c->rec.ws == ws && c->rec.ck == ck && hm.n == N && N >= 1;

    // zero the reverse state planes (boundary ring and padding must be 0) and the accumulators
    HIPCHK(c, launch_fill_bytes(P.planes_begin, 8 * L.plane + 2 * L.plane64, s));
    if (R > 0) {
        HIPCHK(c, hipMemcpyAsync(rec, recv_ij, sizeof(int) * 2 * (size_t)R, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, launch_receivers_csr(rec, R, hm.nx, hm.ny, rowptr, rcol, rid, status, s));
        int st = -1;
        HIPCHK(c, hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (st != 0) return fail(c, FDW_EINVAL, "receivers must be interior nodes (1 <= i <= nx-2, 1 <= j <= ny-2)");
    }
    if (N == 0) {
        HIPCHK(c, launch_grad_out(G1, hm.ld, hm.nx, hm.ny, g1_out, s));
        if (g2_out) HIPCHK(c, launch_grad_out(G2, hm.ld, hm.nx, hm.ny, g2_out, s));
        return FDW_OK;
    }

    MemberDev rep = c->tab[m];
    int cur = 0;
    const void* top_u = nullptr;
    const void* top_d = nullptr;
    if (recorded) {
        top_u = hm.u[hm.cur];
        top_d = hm.d[hm.cur];
    } else {
        // ---- forward replay from the initial data, storing (u, du) every ck steps
        for (int k = 0; k < 2; ++k) {
            rep.u[k] = FU[k];
            rep.d[k] = FD[k];
        }
        rep.R = 0;
        rep.traces = nullptr;
        rep.cur0 = 0;
        rep.n_offset = 0;
        rep.block_base = 0;
        HIPCHK(c, launch_start<T>(&rep, rep_dev, hm.u0, hm.u1, (T)hm.tau, 0, 0, nullptr, c->red, s));
        int64_t n = 1;
        const int Kf = choose_K(c);
        int pushedK = -1;
        auto store_ckpt = [&](int64_t step) -> int {
            const int64_t k = step / ck - 1;
            return store_checkpoint(c, hm, CU[k], CD[k], FU[cur], FD[cur], s);
        };
        if (n % ck == 0 && n < N) {
            int rc = store_ckpt(n);
            if (rc) return rc;
        }
        while (n < N) {
            const int64_t next = std::min<int64_t>(N, (n / ck + 1) * ck);
            const int Kb = (int)std::min<int64_t>(Kf, next - n);
            if (Kb != pushedK) {
                decompose(c, hm, rep, c->S_eff, Kb);
                hipLaunchKernelGGL(k_write_member, dim3(1), dim3(1), 0, s, rep_dev, 0, rep);
                HIPCHK(c, hipGetLastError());
                pushedK = Kb;
            }
            StepArgs a;
            a.eslot = 0;
            a.table = rep_dev;
            a.first = 0;
            a.nmembers = 1;
            a.block_offset = 0;
            a.total_blocks = rep.blocks;
            a.parity = cur;
            a.want_energy = 0;
            a.want_trace = 0;
            a.ctx_step = 0;
            a.stream_nt = rep.stream_nt;
            a.reverse = 0;
            HIPCHK(c, launch_step<T>(a, Kb, c->C, hm.face, rep.blocks, s));
            cur ^= 1;
            n += Kb;
            if (n % ck == 0 && n < N) {
                int rc = store_ckpt(n);
                if (rc) return rc;
            }
        }
        top_u = FU[cur];
        top_d = FD[cur];
    }

    // ---- reverse sweep
    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.nx = hm.nx;
    A.ny = hm.ny;
    A.ld = hm.ld;
    A.face = hm.face;
    A.ax = rep.ax;
    A.ay = rep.ay;
    A.h = hm.h;
    A.hy = hm.hy;
    A.g1 = G1;
    A.g2 = g2_out ? G2 : G1;
    A.R = R;
    A.trace_grad = tg;
    // reverse launch: u, du, lam, mu in and out, h (and hy), the FP64 accumulator in and out
    A.stream_nt = ((size_t)(hm.face ? 10 : 9) * elem_size(c->dtype) + 2 * sizeof(double)) * hm.ld * hm.ny >
                  2 * kLastLevelCacheBytes ? 1 : 0;
    // seed lam^N = mu^N = s_N (planes are zero)
    A.lout = LA[0];
    A.mout = MU[0];
    A.rec_col = rec;
    if (R > 0) HIPCHK(c, launch_adjoint_seed<T>(A, N, s));
    A.rec_rowptr = rowptr;
    A.rec_col = rcol;
    A.rec_id = rid;
    const void* fu_in = top_u;
    const void* fd_in = top_d;
    int fcur = recorded ? 1 : cur;  // the first reverse output goes to the other state plane
    int lcur = 0;
    const int Kr = adjoint_K(c);
    const int Sr = choose_adj_S<T>(c, hm, Kr, g2_out != nullptr);
    int64_t mtop = N;
    while (mtop > 0) {
        if (mtop < N && mtop % ck == 0) {
            // re-anchor the time reversal on the exact stored state
            const int64_t k = mtop / ck - 1;
            fu_in = CU[k];
            fd_in = CD[k];
        }
        const int64_t seg_bot = ((mtop - 1) / ck) * ck;
        const int Kb = (int)std::min<int64_t>(Kr, mtop - seg_bot);
        adj_decompose(c, hm, Kb, Sr, A);
        const int outk = fcur ^ 1;
        A.uin = fu_in;
        A.din = fd_in;
        A.uout = FU[outk];
        A.dout = FD[outk];
        A.lin = LA[lcur];
        A.min = MU[lcur];
        A.lout = LA[lcur ^ 1];
        A.mout = MU[lcur ^ 1];
        A.n_top = mtop;
        const int grid = (A.waves + kWavesPerBlock - 1) / kWavesPerBlock;
        HIPCHK(c, launch_adjoint_block<T>(A, Kb, c->adjC, grid, s));
        fu_in = FU[outk];
        fd_in = FD[outk];
        fcur = outk;
        lcur ^= 1;
        mtop -= Kb;
    }
    HIPCHK(c, launch_grad_out(G1, hm.ld, hm.nx, hm.ny, g1_out, s));
    if (g2_out) HIPCHK(c, launch_grad_out(G2, hm.ld, hm.nx, hm.ny, g2_out, s));
    return FDW_OK;
}

}  // namespace

extern "C" {

size_t fdw_adjoint_workspace_bytes(const fdw_ctx* c, int32_t m, int32_t ckpt_every)
{
    if (!c || m < 0 || m >= c->count || ckpt_every < 1) return 0;
    if (c->mixed) return fdw_adjoint_workspace_bytes(c->sub[c->sub_of[m]], c->sub_idx[m], ckpt_every);
    return adj_layout(c, c->m[m], ckpt_every).total;
}

int fdw_record_checkpoints(fdw_ctx* c, int32_t m, int32_t ckpt_every, void* adj_ws, size_t adj_ws_bytes)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed)
        return fwd(c, c->sub[c->sub_of[m]],
                   fdw_record_checkpoints(c->sub[c->sub_of[m]], c->sub_idx[m], ckpt_every, adj_ws, adj_ws_bytes));
    if (!adj_ws) {
        if (c->rec.member == m) c->rec.member = -1;
        return FDW_OK;
    }
    HostMember& hm = c->m[m];
    if (!hm.coeff) return fail(c, FDW_ESTATE, "fdw_set_coeff first");
    if (hm.n != 0) return fail(c, FDW_ESTATE, "checkpoint recording starts at step 0 (fdw_reset or fdw_set_coeff first)");
    if (ckpt_every < 1) return fail(c, FDW_EINVAL, "ckpt_every must be >= 1");
    if (((uintptr_t)adj_ws) % kAlign) return fail(c, FDW_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (adj_ws_bytes < adj_layout(c, hm, ckpt_every).total) return fail(c, FDW_ENOMEM, "adjoint workspace too small");
    c->rec.member = m;
    c->rec.ck = ckpt_every;
    c->rec.ws = adj_ws;
    return FDW_OK;
}

int fdw_adjoint(fdw_ctx* c, int32_t m, const int32_t* recv_ij, int32_t R, const double* trace_grad, int32_t ckpt_every,
                void* adj_ws, size_t adj_ws_bytes, double* grad_h1, double* grad_h2)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed)
        return fwd(c, c->sub[c->sub_of[m]],
                   fdw_adjoint(c->sub[c->sub_of[m]], c->sub_idx[m], recv_ij, R, trace_grad, ckpt_every, adj_ws,
                               adj_ws_bytes, grad_h1, grad_h2));
    HostMember& hm = c->m[m];
    if (!hm.coeff) return fail(c, FDW_ESTATE, "fdw_set_coeff first");
    if (R < 0 || R > kMaxReceivers) return fail(c, FDW_EINVAL, "R out of range");
    if (R > 0 && (!recv_ij || !trace_grad)) return fail(c, FDW_EINVAL, "recv_ij and trace_grad are required");
    if (ckpt_every < 1) return fail(c, FDW_EINVAL, "ckpt_every must be >= 1");
    if (!adj_ws || ((uintptr_t)adj_ws) % kAlign) return fail(c, FDW_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!grad_h1) return fail(c, FDW_EINVAL, "grad_h1 is NULL");
    if (grad_h2 && !hm.face)
        return fail(c, FDW_EINVAL, "separate dL/dh2 needs a coefficient set with a separate h2");
    return (c->dtype == FDW_F32)
               ? adjoint_impl<float>(c, m, recv_ij, R, trace_grad, ckpt_every, adj_ws, adj_ws_bytes, grad_h1, grad_h2)
               : adjoint_impl<double>(c, m, recv_ij, R, trace_grad, ckpt_every, adj_ws, adj_ws_bytes, grad_h1, grad_h2);
}

}  // extern "C"

// =============================================================================================
// Autotuner
// =============================================================================================
namespace {

std::string tune_key(const fdw_ctx* c)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    std::ostringstream os;
    os << arch << " " << (c->dtype == FDW_F32 ? "f32" : "f64") << " " << c->count;
    for (const HostMember& hm : c->m) os << " " << hm.nx << "x" << hm.ny << (hm.face ? "f" : "n");
    // the launch mode the candidates were timed in
    os << " g" << c->use_graph << "b" << c->batch_mode;
    return os.str();
}

bool cache_lookup(const std::string& key, int* K, int* S, int* C, int* P)
{
    const char* path = std::getenv("FDW_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.rfind('|');
        if (bar == std::string::npos) continue;
        if (line.substr(0, bar) != key) continue;
        std::istringstream is(line.substr(bar + 1));
        int k = 0, sr = 0, cc = 0, pp = 0;
        if (is >> k >> sr >> cc) {
            if (!(is >> pp)) pp = 0;  // the stream policy (absent: automatic)
            *K = k;
            *S = sr;
            *C = cc;
            *P = pp;
            found = true;  // last entry wins
        }
    }
    return found;
}

void cache_store(const std::string& key, int K, int S, int C, int P)
{
    const char* path = std::getenv("FDW_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << "|" << K << " " << S << " " << C << " " << P << "\n";
}

}  // namespace

extern "C" int fdw_autotune(fdw_ctx* c, int32_t steps, int64_t* best_out)
{
    if (!c) return FDW_EINVAL;
    if (c->mixed) {
        // each storage type is tuned on its own; best_out reports the FP32 members' choice
        for (int t = FDW_F64; t >= FDW_F32; --t) {
            const int rc = fdw_autotune(c->sub[t], steps, t == FDW_F32 ? best_out : nullptr);
            if (rc) return fwd(c, c->sub[t], rc);
        }
        return FDW_OK;
    }
    for (const HostMember& hm : c->m) {
        if (!hm.coeff) return fail(c, FDW_ESTATE, "fdw_set_coeff first");
        if (hm.n != 0) return fail(c, FDW_ESTATE, "autotune runs from step 0 (call fdw_reset first)");
    }
    c->rec.member = -1;  // the candidate runs overwrite any checkpoint recording
    const std::string key = tune_key(c);
    int bestK = 0, bestS = 0, bestC_out = c->C, bestP_out = 0;
    if (!cache_lookup(key, &bestK, &bestS, &bestC_out, &bestP_out)) {
        int maxny = 0;
        int64_t points = 0;
        for (const HostMember& hm : c->m) {
            maxny = std::max(maxny, hm.ny);
            points += (int64_t)hm.nx * hm.ny;
        }
        int nsteps = steps > 0 ? steps : (int)std::max<int64_t>(16, std::min<int64_t>(256, (int64_t)4e9 / std::max<int64_t>(points, 1)));
        nsteps = std::max(nsteps, 2 * kMaxTimeBlock);
        // candidates: (columns per lane, time block) pairs the kernels support, x segment rows
        std::vector<std::pair<int, int>> CK;
        if (c->dtype == FDW_F32) {
            for (int K = 1; K <= 8; ++K) CK.push_back({2, K});
            for (int K = 1; K <= 6; ++K) CK.push_back({4, K});
        } else {
            for (int K = 1; K <= 4; ++K) CK.push_back({2, K});
            for (int K = 1; K <= 8; ++K) CK.push_back({1, K});
        }
        const int Ss[] = {8, 16, 32, 48, 64, 96, 128};
        // stream policies: the automatic one, and non-temporal stores with cacheable loads
        // (where that differs from it): which is faster depends on the grids (measured both
        // ways: the 16384^2 float grid gains 18% from cacheable loads, the 8192^2 one loses 5%)
        c->stream_policy = 0;
        std::vector<int> Ps = {0};
        if (!(c->dtype == FDW_F64 && stream_nt(c))) Ps.push_back(3);
        // candidates run in the context's own launch mode (graph replay, persistent launch), so
        // the choice is the best for the way the caller steps; the energy check is off meanwhile
        const int saveCheck = c->check_energy;
        c->check_energy = 0;
        // the search times the streaming kernel (the small-grid tiles have no such parameters)
        const int saveTiles = c->tile_mode;
        c->tile_mode = 1;
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        float best = 1e30f;
        int bestC = c->C, bestP = 0;
        for (int P : Ps)
        for (const auto& ck : CK) {
            for (int S : Ss) {
                if (S > 2 * maxny && S != 32) continue;
                const int Kc = ck.second;
                // the persistent launch runs time blocks of 1, 2, 4 or 8 only
                if (c->batch_mode == 1 && (Kc & (Kc - 1)) != 0) continue;
                c->C = ck.first;
                c->K_cfg = Kc;
                c->S_cfg = S;
                c->S_eff = S;
                c->stream_policy = P;
                invalidate_graphs(c);  // a graph holds the decomposition it was captured with
                int rc = layout_for_K(c, Kc, S);
                if (rc) return rc;
                float med = 0.f;
                std::vector<float> ts;
                for (int rep = 0; rep < 3; ++rep) {
                    for (int i = 0; i < c->count; ++i) {
                        c->m[i].n = 0;
                        c->m[i].cur = 0;
                        sync_member_dev(c, i);
                    }
                    rc = layout_for_K(c, Kc, S);
                    if (rc) return rc;
                    rc = fdw_step_n(c, 1, nullptr);  // start step, outside the timed region
                    if (rc) return rc;
                    HIPCHK(c, hipEventRecord(e0, c->stream));
                    rc = fdw_step_n(c, nsteps, nullptr);
                    if (rc) return rc;
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    HIPCHK(c, hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                    ts.push_back(ms);
                }
                std::sort(ts.begin(), ts.end());
                med = ts[1];
                // candidates come in increasing time block; a later one must be 2% faster
                if (med < best * 0.98f || (med < best && Kc == bestK)) {
                    best = med;
                    bestK = Kc;
                    bestS = S;
                    bestC = ck.first;
                    bestP = P;
                }
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        c->check_energy = saveCheck;
        c->tile_mode = saveTiles;
        bestC_out = bestC;
        bestP_out = bestP;
        cache_store(key, bestK, bestS, bestC, bestP);
    }
    c->C = bestC_out;
    c->K_cfg = bestK;
    c->S_cfg = bestS;
    c->S_eff = bestS;
    c->stream_policy = bestP_out;
    for (int i = 0; i < c->count; ++i) {
        c->m[i].n = 0;
        c->m[i].cur = 0;
        sync_member_dev(c, i);
    }
    invalidate_graphs(c);
    int rc = layout_for_K(c, choose_K(c), c->S_eff);
    if (rc) return rc;
    if (best_out) {
        best_out[0] = bestK;
        best_out[1] = bestS;
        best_out[2] = c->C;
    }
    return FDW_OK;
}

// =============================================================================================
// Autotuner of the reverse sweep
// =============================================================================================
extern "C" int fdw_autotune_adjoint(fdw_ctx* c, int32_t m, const int32_t* recv_ij, int32_t R, const double* trace_grad,
                                    int32_t ckpt_every, void* adj_ws, size_t adj_ws_bytes, double* grad_scratch,
                                    int64_t* best_out)
{
    int rc = check_member(c, m);
    if (rc) return rc;
    if (c->mixed) {
        fdw_ctx* ch = c->sub[c->sub_of[m]];
        return fwd(c, ch, fdw_autotune_adjoint(ch, c->sub_idx[m], recv_ij, R, trace_grad, ckpt_every, adj_ws,
                                               adj_ws_bytes, grad_scratch, best_out));
    }
    if (!grad_scratch) return fail(c, FDW_EINVAL, "grad_scratch is NULL");
    const HostMember& hm = c->m[m];
    std::ostringstream key;
    key << tune_key(c) << " adj m" << m << " c" << ckpt_every << " R" << R;
    int bestK = c->adjK, bestC = c->adjC, bestS = c->adjS_cfg;
    int cK = 0, cS = 0, cC = 0;
    int cP = 0;
    if (cache_lookup(key.str(), &cK, &cS, &cC, &cP)) {
        bestK = cK;
        bestS = cS;
        bestC = cC;
    } else {
        // (columns per lane, reverse time block) pairs the kernels support, x rows per item (0: automatic)
        std::vector<std::pair<int, int>> CK;
        if (c->dtype == FDW_F64) {
            for (int K = 2; K <= 6; ++K) CK.push_back({1, K});
            for (int K = 2; K <= 4; ++K) CK.push_back({2, K});
        } else {
            for (int K = 2; K <= 6; ++K) CK.push_back({2, K});
            for (int K = 2; K <= 4; ++K) CK.push_back({4, K});
        }
        const int Ss[] = {0, 16, 32, 64};
        const int saveK = c->adjK, saveC = c->adjC, saveS = c->adjS_cfg;
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        float best = 1e30f;
        for (const auto& ck : CK) {
            for (int S : Ss) {
                if (S > 0 && (S < 4 * ck.second || S > hm.ny)) continue;
                c->adjC = ck.first;
                c->adjK = ck.second;
                c->adjS_cfg = S;
                std::vector<float> ts;
                for (int rep = 0; rep < 2; ++rep) {
                    HIPCHK(c, hipEventRecord(e0, c->stream));
                    rc = fdw_adjoint(c, m, recv_ij, R, trace_grad, ckpt_every, adj_ws, adj_ws_bytes, grad_scratch,
                                     nullptr);
                    if (rc) {
                        c->adjK = saveK;
                        c->adjC = saveC;
                        c->adjS_cfg = saveS;
                        hipEventDestroy(e0);
                        hipEventDestroy(e1);
                        return rc;
                    }
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    HIPCHK(c, hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                    ts.push_back(ms);
                }
                const float t = std::min(ts[0], ts[1]);
                if (t < best) {
                    best = t;
                    bestK = ck.second;
                    bestC = ck.first;
                    bestS = S;
                }
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        cache_store(key.str(), bestK, bestS, bestC, 0);
    }
    c->adjK = bestK;
    c->adjC = bestC;
    c->adjS_cfg = bestS;
    if (best_out) {
        best_out[0] = bestK;
        best_out[1] = bestS;
        best_out[2] = bestC;
    }
    return FDW_OK;
}
