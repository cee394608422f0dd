// fdw_step_f64c2.hip - instantiation unit of the streaming stencil: double storage, 2 grid
// columns per lane, time blocks K = 1..4.
#include "fdw_stream.h"

namespace fdw {

hipError_t launch_step_f64c2(const StepArgs& a, int K, int face_mode, int grid, hipStream_t s)
{
    return launch_step_c<double, 2, 4>(a, K, face_mode, grid, s);
}
hipError_t launch_persistent_f64c2(const StepArgs& a, int K, int face_mode, int phases, int grid, int* bar,
                                   const PersistentExtra& x, hipStream_t s)
{
    return launch_persistent_c<double, 2, 4>(a, K, face_mode, phases, grid, bar, x, s);
}
int persistent_max_f64c2(int K, int face_mode, bool energy) { return persistent_max_c<double, 2, 4>(K, face_mode, energy); }

}  // namespace fdw
