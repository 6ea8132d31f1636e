// Dispatch of the persistent solve kernel over the MR degree l (one
// instance per l, compiled in its own translation unit).
#include "kernels.h"

namespace msb {

template <typename T, int L> int persistent_grid_l(int device);
template <typename T, int L> hipError_t launch_persistent_l(hipStream_t st, const PersistArgs &pa, int grid);

template <typename T>
int persistent_grid(int device, int l) {
    switch (l) {
    case 1: return persistent_grid_l<T, 1>(device);
    case 2: return persistent_grid_l<T, 2>(device);
    case 3: return persistent_grid_l<T, 3>(device);
    case 4: return persistent_grid_l<T, 4>(device);
    case 5: return persistent_grid_l<T, 5>(device);
    case 6: return persistent_grid_l<T, 6>(device);
    default: return 0;
    }
}

template <typename T>
hipError_t launch_persistent(hipStream_t st, const PersistArgs &pa, int grid, int l) {
    switch (l) {
    case 1: return launch_persistent_l<T, 1>(st, pa, grid);
    case 2: return launch_persistent_l<T, 2>(st, pa, grid);
    case 3: return launch_persistent_l<T, 3>(st, pa, grid);
    case 4: return launch_persistent_l<T, 4>(st, pa, grid);
    case 5: return launch_persistent_l<T, 5>(st, pa, grid);
    case 6: return launch_persistent_l<T, 6>(st, pa, grid);
    default: return hipErrorInvalidValue;
    }
}

template int persistent_grid<double>(int, int);
template int persistent_grid<float>(int, int);
template hipError_t launch_persistent<double>(hipStream_t, const PersistArgs &, int, int);
template hipError_t launch_persistent<float>(hipStream_t, const PersistArgs &, int, int);

}  // namespace msb
