// Constants shared by the host and GPU forms of k-means.
#pragma once

namespace csc {

// k-means++ seeding: the cumulative D^2 weights are summed in blocks of this
// many points (a block's offset plus the running sum inside it), on the host
// and on the GPU alike.
constexpr int kSeedBlock = 32;

}  // namespace csc
