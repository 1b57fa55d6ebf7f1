// Device code shared by the kernel translation units (included only by the
// .hip files; the host translation units see common.h alone).
#pragma once

#include "common.h"

namespace lbmib {

__device__ inline int wrap_index(int a, int b) {
  const int r = a % b;
  return r < 0 ? r + b : r;
}

// Mark the stream-collide blocks holding any node of [lo - 2, hi + 2] (per
// axis, periodic) of box `box` as near at step v, listing each newly marked
// block once (the flag exchange decides which marker lists it).  Called by
// one workgroup per bead.
__device__ inline void mark_near_blocks(const Dev& d, const Box& B, int box, const int* lo, const int* hi,
                                        int64_t v) {
  const int p = (int)(v & 1), pf = near_slot(v);
  const int first = d.nboxes == 1 ? 0 : d.sc_box_block0[box];
  const int x0 = lo[0] - 2, nxs = hi[0] - lo[0] + 5;
  const int ny_r = min(hi[1] - lo[1] + 5, B.ny), nz_r = min(hi[2] - lo[2] + 5, B.nz);
  for (int r = threadIdx.x; r < ny_r * nz_r; r += blockDim.x) {
    const int y = wrap_index(lo[1] - 2 + r % ny_r, B.ny), z = wrap_index(lo[2] - 2 + r / ny_r, B.nz);
    const int row = (z * B.ny + y) * B.nx;  // box-local id of node (0, y, z)
    int seg[2][2] = {{0, B.nx - 1}, {0, -1}};
    if (nxs < B.nx) {
      const int xs = wrap_index(x0, B.nx), xe = xs + nxs - 1;
      seg[0][0] = xs;
      seg[0][1] = min(xe, B.nx - 1);
      if (xe >= B.nx) seg[1][1] = xe - B.nx;
    }
    for (int sgi = 0; sgi < 2; ++sgi) {
      if (seg[sgi][1] < seg[sgi][0]) continue;
      for (int blk = first + (row + seg[sgi][0]) / d.sc_bs; blk <= first + (row + seg[sgi][1]) / d.sc_bs; ++blk) {
        if (atomicExch(&d.near[pf * d.nsc + blk], (int)v) != (int)v) {
          const int i = atomicAdd(&d.near_count[p], 1);
          if (i < d.max_near)
            d.near_list[p * d.max_near + i] = blk;
          else
            atomicOr(d.overflow, 2);
        }
      }
    }
  }
}

}  // namespace lbmib
