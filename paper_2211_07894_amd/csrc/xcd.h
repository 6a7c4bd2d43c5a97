// Workgroup -> work mapping aware of the MI355X's 8 accelerator dies (XCDs).
//
// The dispatcher hands workgroups to the XCDs round-robin by linear id, and each
// XCD has its own L2.  Work items that share operands (the tiles of one split of
// one projected matrix read the same rows of Psi; the directions of one block of
// grid points read the same slice of Psi) should run on one XCD at about the same
// time.  With `groups` groups of `per_group` items, linear id L is mapped so that
// XCD L % 8 takes whole groups, their items in consecutive order.  When groups
// is not a multiple of 8 the groups are simply laid out one after another.
#pragma once

#include <hip/hip_runtime.h>

namespace lrdm {

constexpr int kXcds = 8;

__device__ inline void xcd_map(int L, int groups, int per_group, int& group, int& item) {
  if (groups % kXcds == 0) {
    const int j = L / kXcds;
    group = L % kXcds + kXcds * (j / per_group);
    item = j % per_group;
  } else {
    group = L / per_group;
    item = L % per_group;
  }
}

}  // namespace lrdm
