// Constants shared by the schedule builder (host) and the kernels.
#pragma once

namespace spchol {

constexpr int kSiSeg = 256;  // selected inversion: most rows of B per Y task (split K)
constexpr int kSiTasksMax = 1024;  // Y launches: segments are halved (down to 64 rows) while
                                   // the launch stays within this many tasks
// An internal update tile over a range of panels (task field c: first panel
// | count << 16 | kPanelRange), its adds atomic: a column block entering the
// window of the one-launch panel rounds takes all finished panels at once,
// split over tasks of at most kRangePanels panels each.
constexpr int kPanelRange = 1 << 30;
constexpr int kRangePanels = 4;
// The window: panel p - 2's update tiles in round p go to column blocks p ..
// p + kRoundWindow - 1; the block after them enters (40^3 x 3, 111-panel
// root: windows of 2 / 3-4 / 8 / 16 blocks 24.1 / 23.8-23.9 / 24.8 / 25.1 ms
// against 25.7 ms without; ranges of 2 / 8 / 16 panels instead of 4:
// 24.1 / 24.7 / 28.3 ms).
constexpr int kRoundWindow = 4;

}  // namespace spchol
