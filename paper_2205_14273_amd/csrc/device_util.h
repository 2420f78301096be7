// Device helpers shared by the kernel files.
#pragma once

#include "ssamg_impl.h"

namespace ssamg {
namespace dev {

__device__ __forceinline__ void cell_ijk(int c, int nx, int ny, int &i, int &j, int &k) {
  i = c % nx;
  const int t = c / nx;
  j = t % ny;
  k = t / ny;
}

// bit0: the -1 neighbour exists, bit1: the 0 neighbour (always), bit2: +1
__device__ __forceinline__ unsigned nb_mask(int i, int n) {
  return (i > 0 ? 1u : 0u) | 2u | (i < n - 1 ? 4u : 0u);
}

__device__ __forceinline__ bool nb_ok(unsigned mx, unsigned my, unsigned mz, int code) {
  return ((mx >> (code & 3)) & (my >> ((code >> 2) & 3)) & (mz >> ((code >> 4) & 3)) & 1u) != 0;
}

// XCD-aware block order: consecutive chunks of one part land on one XCD (the
// hardware deals blocks round-robin over the 8 XCDs), so the neighbour planes a
// block re-reads sit in that XCD's L2.
__device__ __forceinline__ int chunk_index() {
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  if ((nblk & 7) != 0) return b;
  return (b & 7) * (nblk >> 3) + (b >> 3);
}

}  // namespace dev
}  // namespace ssamg
