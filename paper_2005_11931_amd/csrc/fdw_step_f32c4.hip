// fdw_step_f32c4.hip - instantiation unit of the streaming stencil: float storage, 4 grid
// columns per lane, time blocks K = 1..6.
#include "fdw_stream.h"

namespace fdw {

hipError_t launch_step_f32c4(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s)
{
    return launch_step_c<float, 4, 6>(a, K, face_mode, grid, s);
}
hipError_t launch_persistent_f32c4(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s)
{
    return launch_persistent_c<float, 4, 6>(a, K, face_mode, phases, grid, bar, x, s);
}
int persistent_max_f32c4(int K, int face_mode, bool energy) { return persistent_max_c<float, 4, 6>(K, face_mode, energy); }

}  // namespace fdw
