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

// Load through a pointer known to address global memory. Pointers read from
// device-side tables (part descriptors) are generic to the compiler, which
// then emits flat loads; a flat load counts against the scalar-load counter as
// well, so each wait for a table entry would also wait for it.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> G(const T *p) {
  return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ T gload(const T *p) {
  return *G(p);
}

template <typename T>
using gptr_w = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr_w<T> Gw(T *p) {
  return (gptr_w<T>)p;
}

// v through an empty asm statement, so that the optimiser cannot see how it
// was formed: an index chosen by a select (a neighbour's offset or 0) then
// keeps its load unconditional instead of being folded into a branch around
// the load, where the load would wait for the one before it.
__device__ __forceinline__ int opaque(int v) {
  __asm__("" : "+v"(v));
  return v;
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

// Tiled block order for a sweep whose blocks cover whole z-planes bp blocks at
// a time: the 8 XCD ranges are as in chunk_index, and inside its range an XCD
// walks strips of sb blocks of one plane, every plane of the range for one
// strip before the next strip. The planes above and below a block are then read
// again while they still sit in the XCD's L2. A bijection on [0, gridDim.x).
__device__ __forceinline__ int chunk_index_tiled(int bp, int sb) {
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  if ((nblk & 7) != 0) return b;
  const int r = nblk >> 3, xcd = b & 7, k = b >> 3;
  if (sb <= 0 || bp <= 0 || sb >= bp || r % bp != 0) return xcd * r + k;
  const int pz = r / bp;
  const int full = bp / sb;
  const int span = sb * pz;
  int z, pb;
  if (k < full * span) {
    const int s = k / span, q = k - s * span;
    z = q / sb;
    pb = s * sb + (q - z * sb);
  } else {
    const int w = bp - full * sb, q = k - full * span;
    z = q / w;
    pb = full * sb + (q - z * w);
  }
  return xcd * r + z * bp + pb;
}

}  // namespace dev
}  // namespace ssamg
