// Sizes shared by the network's kernels (mlp.hip) and the API that allocates for
// them (api.hip).
#pragma once

namespace mc {

// Blocks of the feature statistics' first pass, and the doubles of its buffer:
// 4 means and 4 standard deviations, then 4 partial sums per block.
constexpr int kStatBlocks = 256;
constexpr int kFeatStatsDoubles = 8 + 4 * kStatBlocks;

}  // namespace mc
