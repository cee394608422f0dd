// fdw_tile.h - the small-grid kernel's decomposition and launcher (fdw_tile.hip).
//
// One workgroup of `waves` waves per tile of kWaveSize columns (kTileCols owned) and
// kTileRowsPerWave * waves rows (kTileHalo halo rows above and below); the member table holds
// strips = tile columns, seg_rows = owned rows per tile, waves = blocks = tiles.  Time blocks
// 1..8, no receiver traces.
#pragma once

#include "fdw_internal.h"

namespace fdw {

constexpr int kTileRowsPerWave = 4;
constexpr int kTileHalo = kMaxTimeBlock;
constexpr int kTileCols = kWaveSize - 2 * kTileHalo;
constexpr int kMaxTileWaves = 16;

template <typename T>
hipError_t launch_step_tile(const StepArgs& a, int K, int face_mode, int waves, int grid, hipStream_t s);

}  // namespace fdw
