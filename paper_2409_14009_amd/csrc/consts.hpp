// Constants shared by the schedule builder (host) and the kernels.
#pragma once

namespace spchol {

constexpr int kSiSeg = 256;  // selected inversion: rows of B per Y task (split K)

}  // namespace spchol
