// fdw_internal.h - device data layout and kernel launchers of libfdw (gfx950).
//
// Layout in HBM: every field of a member is a pitched plane [ny][ld] in the storage type
// (float or double), x fastest, ld = nx rounded up to a multiple of 64 elements so that
// every row starts on a 256-byte boundary and a wave's C-element lane vectors are aligned.
// Columns nx..ld-1 and the boundary ring hold 0 at all times.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

constexpr int kMaxTimeBlock = 8;      // time steps fused in one streaming launch
constexpr int kMaxEnergySlots = 64;   // time blocks whose energy partials one finalisation sums
constexpr int kWaveSize = 64;         // CDNA wavefront
constexpr int kWavesPerBlock = 4;     // independent streaming waves per workgroup
constexpr int kMaxReceivers = 16384;  // per member
constexpr int kRedBlocks = 1024;      // blocks of the generic two-stage reductions
// persistent batched launch: at most this many time blocks per launch; its control words are
// the grid barrier (16 ints) and one work counter per (time block, XCD)
constexpr int kPersistentPhases = 1024;
// last-level (Infinity) cache of the MI355X; working sets above it are streamed non-temporally
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
constexpr int kPersistentCtlInts = 16 + 8 * kPersistentPhases;
constexpr int kPadRowsTop = 0;        // rows reserved above / below each plane (none needed: the
constexpr int kPadRowsBottom = 0;     // streaming kernel's buffer loads return 0 outside the grid)

// Static description of one member, resident in device memory (the member table).
struct MemberDev {
    int nx, ny, ld;
    int face;        // 0: nodal h (h1 == h2) in plane h; 1: face sums FX = h1_i + h1_{i+1} in h, FY in hy
    int strips;      // streaming work decomposition of the current launch configuration
    int segs;
    int seg_rows;
    int waves;       // strips * segs
    int blocks;      // ceil(waves / kWavesPerBlock)
    int block_base;  // first block of this member in an all-member launch
    int cur0;        // buffer pair holding the state when the launch parity is 0
    int energy_row;  // row of this member in the caller's [count][n] energy array (its index in the
                     // family; differs from the index in this table when the family mixes storage types)
    int R;           // receivers (0: no trace recording)
    int64_t n_offset;    // member step = context step + n_offset
    int64_t trace_rows;  // N + 1
    double ax, ay;   // 0.5 tau^2/dx^2, 0.5 tau^2/dy^2 (cast to the storage type in kernels)
    double escale;   // dx dy / tau^2 (energy)
    void* u[2];
    void* d[2];
    void* h;
    void* hy;
    const int* rec_rowptr;  // [ny + 1] CSR of receivers by row
    const int* rec_col;     // [R] column of each receiver, sorted by (row, column)
    const int* rec_id;      // [R] position of the receiver in the caller's list
    void* traces;           // [trace_rows][R]
    double* epart;          // energy partials [2][kMaxTimeBlock][max waves] (two slots: the persistent
                            // launch alternates them between time blocks)
    int epart_stride;       // max waves
    int stream_nt;          // 1: the launch's planes exceed the last-level cache; stream them
                            // with non-temporal accesses (0: keep them cacheable)
};

// Per-launch arguments of the streaming stencil.
struct StepArgs {
    const MemberDev* table;
    int nmembers;      // members covered by this launch (table[first .. first+nmembers-1])
    int first;
    int block_offset;  // added to blockIdx.x before the member lookup
    int total_blocks;  // blocks of the launch (for the XCD-aware remap)
    int parity;        // launch parity: member state pair = cur0 ^ parity
    int want_energy;
    int want_trace;
    int64_t ctx_step;  // context step before this launch
    int stream_nt;     // 1: non-temporal loads of the state rows (float; see MemberDev for the stores)
    int reverse;       // 1: walk the launch's blocks in reverse order (alternating item order)
    int eslot;         // energy-partial slot the launch writes (time block within a finalisation group)
};

// Extra arguments of the persistent launch: where its energies go (as for
// launch_energy_finalize) and its error words.
struct PersistentExtra {
    double* energy_base;    // energy of member m, step k of the call: energy_base[row_m * energy_stride + k]
    int64_t energy_stride;
    int64_t energy_offset;  // step of the call the launch's first time block starts at
    int* health;            // failure detection, as for launch_energy_finalize
    int* err;               // bit 0: a grid barrier timed out (results invalid)
};

// ---- launchers (fdw_kernels.hip) ---------------------------------------------------------
// All return hipError_t of the launch.
// C = columns per lane (float: 2 or 4; double: 2)
template <typename T>
hipError_t launch_step(const StepArgs& a, int K, int C, int face_mode, int grid, hipStream_t s);
template <typename T>
hipError_t launch_step_persistent(const StepArgs& a, int K, int C, int face_mode, int phases, int grid, int* barrier,
                                  const PersistentExtra& x, hipStream_t s);
// resident workgroups of the persistent launch variant (with or without energies)
template <typename T>
int persistent_max_blocks(int K, int C, int face_mode, bool energy);

template <typename T>
// health (may be null): bit 0 set when an energy is non-finite, bit 1 when one exceeds 10x the
// first energy of the call (energy_base[row * energy_stride], row = MemberDev::energy_row)
// slot: the partial slot holding the first time block; nslots time blocks of `levels` steps
// each, in slots slot .. slot + nslots - 1, their energies at energy_offset + j * levels + t
hipError_t launch_energy_finalize(const MemberDev* table, int first, int nmembers, int levels, double* energy_base,
                                  int64_t energy_stride, int64_t energy_offset, int* health, hipStream_t s,
                                  int slot = 0, int nslots = 1);

template <typename T>
hipError_t launch_prepare_coeff(const MemberDev* m_host, const void* h1, const void* h2, int face, double* red,
                                hipStream_t s);
template <typename T>
hipError_t launch_start(const MemberDev* m_host, const MemberDev* m_dev, const void* u0, const void* u1, T tau,
                        int want_energy, int want_trace, double* energy_out, double* red, hipStream_t s);
template <typename T>
hipError_t launch_state_energy(const MemberDev* m_host, int cur, double* red, double* out, hipStream_t s);
template <typename T>
hipError_t launch_gather(const void* u, int ld, const int* rec_ij, int R, void* out_row, hipStream_t s);
template <typename T>
hipError_t launch_misfit(const void* traces, const double* d, int64_t n, double* J, double* grad, double* red,
                         hipStream_t s);
template <typename T>
hipError_t launch_copy_in(const void* src, int nx, int ny, void* dst, int ld, int zero_ring, hipStream_t s);
template <typename T>
hipError_t launch_copy_out(const void* src, int ld, int nx, int ny, void* dst, hipStream_t s);
hipError_t launch_fill_bytes(void* p, size_t bytes, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);  // *p = v, stream-ordered (a kernel, not a memset)
template <typename T>
hipError_t launch_diff_norm(const void* a, const void* b, int ld, int nx, int ny, double scale, double* red,
                            double* out, hipStream_t s);
// copies the trace columns of coincident receivers (rows lo..hi of a [rows][R] trace array)
hipError_t launch_trace_dups(void* traces, int es, int R, const int* rec_ij, const int* id, int64_t lo, int64_t hi,
                             hipStream_t s);
hipError_t launch_receivers_csr(const int* rec_ij, int R, int nx, int ny, int* rowptr, int* col, int* id,
                                int* status, hipStream_t s);

// ---- adjoint (fdw_adjoint.hip) ---------------------------------------------------------
struct AdjArgs {
    int nx, ny, ld, face;
    double ax, ay;
    const void* h;
    const void* hy;
    // state pairs: forward (u, du) and adjoint (lam, mu), in and out
    const void* uin;
    const void* din;
    void* uout;
    void* dout;
    const void* lin;
    const void* min;
    void* lout;
    void* mout;
    double* g1;  // dL/dh1 accumulator (nodal), [ny][ld] double
    double* g2;  // dL/dh2 accumulator, or equal to g1 when the two are summed
    const int* rec_rowptr;
    const int* rec_col;
    const int* rec_id;
    int R;
    const double* trace_grad;  // [N+1][R]
    int64_t n_top;             // forward step index of the input state u (level n_top)
    int strips, segs, seg_rows, waves;
    int stream_nt;             // 1: write the outputs with non-temporal stores (planes exceed the cache)
};
template <typename T>
hipError_t launch_adjoint_block(const AdjArgs& a, int K, int C, int grid, hipStream_t s);
// waves of the reverse kernel (K, C, layout) the device holds at once (0 if unknown)
template <typename T>
int adjoint_resident_waves(int K, int C, bool face, bool split);
template <typename T>
hipError_t launch_adjoint_seed(const AdjArgs& a, int64_t N, hipStream_t s);
hipError_t launch_grad_out(const double* g, int ld, int nx, int ny, double* out, hipStream_t s);

}  // namespace fdw
