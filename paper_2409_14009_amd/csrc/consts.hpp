// Constants shared by the schedule builder (host) and the kernels.
#pragma once

namespace spchol {

constexpr int kSiSeg = 256;  // selected inversion: most rows of B per Y task (split K)
constexpr int kSiTasksMax = 1024;  // Y launches: segments are halved (down to 64 rows) while
                                   // the launch stays within this many tasks

}  // namespace spchol
