// Instances of the level kernel k_level<double, L> for levels 1 .. kFastLevels.
#include "pc_level.h"

namespace pcg {

hipError_t launch_level_fast_f64(hipStream_t s, const Batch &b, int level, int R, int lds, int grid) {
    return LevelRange<double, 1, kFastLevels>::launch(s, b, level, R, lds, grid);
}

int occupancy_level_fast_f64(int level, int lds_bytes) {
    return LevelRange<double, 1, kFastLevels>::occupancy(level, lds_bytes);
}

}  // namespace pcg
