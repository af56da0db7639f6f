// Instances of the deep-level kernel k_level_deep<T, L> for levels kFastLevels + 1 .. PC_MAX_LEVEL.
#include "pc_level.h"

namespace pcg {

hipError_t launch_level_deep(hipStream_t s, const Batch &b, int level, int R, int lds, int grid) {
    if (b.prec == PC_PREC_FP64)
        return LevelRange<double, kFastLevels + 1, PC_MAX_LEVEL>::launch(s, b, level, R, lds, grid);
    return LevelRange<float, kFastLevels + 1, PC_MAX_LEVEL>::launch(s, b, level, R, lds, grid);
}

int occupancy_level_deep(int prec, int level) {
    if (prec == PC_PREC_FP64) return LevelRange<double, kFastLevels + 1, PC_MAX_LEVEL>::occupancy(level, 0);
    return LevelRange<float, kFastLevels + 1, PC_MAX_LEVEL>::occupancy(level, 0);
}

}  // namespace pcg
