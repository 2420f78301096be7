// Krylov (PCG, Section 4 protocol) and vector kernels (gfx950): deterministic
// dot products, the fused x/r and p updates, casts, fills and copies.
// Vectors are [cell][rhs] with nrhs = 1 << lg right-hand sides interleaved.
#include "ssamg_impl.h"

namespace ssamg {

namespace {

__global__ __launch_bounds__(kBlock) void k_cast_d2f(const double *__restrict__ in,
                                                     float *__restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    out[i] = (float)in[i];
}

__global__ __launch_bounds__(kBlock) void k_cast_f2d(const float *__restrict__ in,
                                                     double *__restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    out[i] = (double)in[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ x, double v, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    x[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_copy(const double *__restrict__ in,
                                                 double *__restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    out[i] = in[i];
}

// ---------------------------------------------------------------- reductions
// Deterministic: a fixed grid of kRedBlocks blocks, each thread accumulating a
// fixed stride-set of elements, a fixed LDS tree per block, and a single-block
// final pass in fixed order.  With nrhs interleaved right-hand sides, lanes
// that share (tid mod nrhs) share a right-hand side, and every tree step keeps
// that invariant (strides are multiples of nrhs).

__device__ __forceinline__ void block_tree(double *sh, int nr) {
  for (int s = kBlock / 2; s >= nr; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(const double *__restrict__ a,
                                                        const double *__restrict__ b, long long nel,
                                                        int lg, double *__restrict__ partial) {
  __shared__ double sh[kBlock];
  const int nr = 1 << lg;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock)
    acc = fma(a[i], b[i], acc);
  sh[threadIdx.x] = acc;
  block_tree(sh, nr);
  if ((int)threadIdx.x < nr) partial[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
}

// a.b and b.c in one pass over the three vectors (the same per-thread sums
// and trees as two k_dot_partial launches, so the same values); the second
// set of partials goes to partial + kRedBlocks * kMaxRhs
__global__ __launch_bounds__(kBlock) void k_dot2_partial(const double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         const double *__restrict__ c, long long nel,
                                                         int lg, double *__restrict__ partial) {
  __shared__ double sh[kBlock], sh2[kBlock];
  const int nr = 1 << lg;
  double acc = 0.0, acc2 = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock) {
    const double bi = b[i];
    acc = fma(a[i], bi, acc);
    acc2 = fma(bi, c[i], acc2);
  }
  sh[threadIdx.x] = acc;
  sh2[threadIdx.x] = acc2;
  for (int s = kBlock / 2; s >= nr; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) {
      sh[threadIdx.x] += sh[threadIdx.x + s];
      sh2[threadIdx.x] += sh2[threadIdx.x + s];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    partial[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
    partial[(kRedBlocks + blockIdx.x) * kMaxRhs + threadIdx.x] = sh2[threadIdx.x];
  }
}

// slot <- sum of partials; shift_rz: first move S_RZN to S_RZ (PCG bookkeeping).
// kFinalThreads threads; each requests its first four partials of its
// right-hand side at once (then four at a time), adds them in a fixed order,
// and the sums of one right-hand side are combined by a fixed tree of
// cross-lane exchanges inside each wave and a fixed pairwise tree over the
// waves.
constexpr int kFinalThreads = 1024;
constexpr int kFinalWaves = kFinalThreads / 64;

// Block b of the grid reduces the partials at partial + b * kRedBlocks * kMaxRhs
// into slot + b * (slot2 - slot): one launch finishes one or two dot products.
__global__ __launch_bounds__(kFinalThreads) void k_dot_final(const double *__restrict__ partial, int nblk,
                                                             int lg, double *__restrict__ scal, int slot,
                                                             int shift_rz, int slot2) {
  __shared__ double sh[kFinalWaves * kMaxRhs];
  if (blockIdx.x == 1) {
    partial += (size_t)kRedBlocks * kMaxRhs;
    slot = slot2;
    shift_rz = 0;
  }
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  const int step = kFinalThreads >> lg;
  int bidx = threadIdx.x >> lg;
  double a[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    // out-of-range slots load partial 0 (always present) and add nothing
    const int bb = bidx + u * step;
    const double t = partial[(long long)(bb < nblk ? bb : 0) * kMaxRhs + kr];
    a[u] = bb < nblk ? t : 0.0;
  }
  for (bidx += 4 * step; bidx + 3 * step < nblk; bidx += 4 * step) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] += partial[(long long)(bidx + u * step) * kMaxRhs + kr];
  }
  for (; bidx < nblk; bidx += step) a[0] += partial[(long long)bidx * kMaxRhs + kr];
  double v = (a[0] + a[1]) + (a[2] + a[3]);
  // lanes l and l ^ off hold the same right-hand side for every off >= nr
  for (int off = 32; off >= nr; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < nr) sh[wave * nr + lane] = v;
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    double w[kFinalWaves];
#pragma unroll
    for (int q = 0; q < kFinalWaves; ++q) w[q] = sh[q * nr + threadIdx.x];
#pragma unroll
    for (int h = kFinalWaves / 2; h >= 1; h >>= 1) {
#pragma unroll
      for (int q = 0; q < h; ++q) w[q] += w[q + h];
    }
    if (shift_rz) scal[S_RZ * kMaxRhs + threadIdx.x] = scal[S_RZN * kMaxRhs + threadIdx.x];
    scal[slot * kMaxRhs + threadIdx.x] = w[0];
  }
}

// r -= alpha q with alpha = rz/pq per right-hand side (0 when frozen), plus
// the partial sums of r.r; alpha is kept in S_ALPHA for the x update, which
// waits for the next p update (k_pcg_xp) or the end of the solve (k_pcg_x), so
// that p is read once per iteration
// TX (one column only): also the finest level's first sweep from zero of the
// next cycle, x0 = w r with the level's smoother factors w (k_smooth_zero's
// arithmetic), so that the cycle need not read r again for it
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_pcg_r(long long nel, int lg, double *__restrict__ scal,
                                                  const int *__restrict__ active, double *__restrict__ r,
                                                  const double *__restrict__ q,
                                                  double *__restrict__ partial, const TX *__restrict__ w,
                                                  TX *__restrict__ x0) {
  __shared__ double sh[kBlock];
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  const bool act = active[kr] != 0;
  const double alpha = act ? scal[S_RZN * kMaxRhs + kr] / scal[S_PQ * kMaxRhs + kr] : 0.0;
  if (blockIdx.x == 0 && (int)threadIdx.x < nr) scal[S_ALPHA * kMaxRhs + kr] = alpha;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock) {
    double ri = r[i];
    if (act) {
      ri = fma(-alpha, q[i], ri);
      r[i] = ri;
    }
    acc = fma(ri, ri, acc);
    if (x0) x0[i] = w[i] * (TX)ri;
  }
  sh[threadIdx.x] = acc;
  block_tree(sh, nr);
  if ((int)threadIdx.x < nr) partial[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
}

// x += alpha p (alpha of the last r update, 0 for a right-hand side that was
// frozen then), then p = z + beta p; beta = rz_new/rz_old, or -(z.q)/(p.q) for
// flexible CG, 0 for a frozen right-hand side
__global__ __launch_bounds__(kBlock) void k_pcg_xp(long long nel, int lg,
                                                   const double *__restrict__ scal,
                                                   const int *__restrict__ active, int flexible,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ p, double *__restrict__ x) {
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  const double alpha = scal[S_ALPHA * kMaxRhs + kr];
  double beta = flexible ? -scal[S_ZQ * kMaxRhs + kr] / scal[S_PQ * kMaxRhs + kr]
                         : scal[S_RZN * kMaxRhs + kr] / scal[S_RZ * kMaxRhs + kr];
  if (!active[kr]) beta = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock) {
    const double pi = p[i];
    x[i] = fma(alpha, pi, x[i]);
    p[i] = fma(beta, pi, z[i]);
  }
}

// the last x += alpha p of a solve
__global__ __launch_bounds__(kBlock) void k_pcg_x(long long nel, int lg, const double *__restrict__ scal,
                                                  const double *__restrict__ p, double *__restrict__ x) {
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  const double alpha = scal[S_ALPHA * kMaxRhs + kr];
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock)
    x[i] = fma(alpha, p[i], x[i]);
}

// partial sums of (b - Ax)^2
__global__ __launch_bounds__(kBlock) void k_resid_partial(const double *__restrict__ b,
                                                          const double *__restrict__ ax,
                                                          long long nel, int lg,
                                                          double *__restrict__ partial) {
  __shared__ double sh[kBlock];
  const int nr = 1 << lg;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock) {
    const double t = b[i] - ax[i];
    acc = fma(t, t, acc);
  }
  sh[threadIdx.x] = acc;
  block_tree(sh, nr);
  if ((int)threadIdx.x < nr) partial[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
}

// Layout change between [nrhs][N] (one vector per right-hand side) and the
// library's [N][nrhs]: a block moves a tile of kTrCells cells x nrhs columns
// through LDS, so both the read and the write are unit-stride across lanes.
constexpr int kTrCells = 128;
__global__ __launch_bounds__(kBlock) void k_transpose(const double *__restrict__ in,
                                                      double *__restrict__ out, long long n, int lg,
                                                      int to_cell_major) {
  __shared__ double tile[kMaxRhs][kTrCells + 1];
  const int nrhs = 1 << lg;
  const long long c0 = (long long)blockIdx.x * kTrCells;
  const int nc = (int)min((long long)kTrCells, n - c0);
  const int tot = nrhs * kTrCells;
  for (int t = threadIdx.x; t < tot; t += kBlock) {
    // column-major side: [nrhs][N], cells fastest
    const int k = t / kTrCells, cc = t % kTrCells;
    // cell-major side: [N][nrhs], right-hand sides fastest
    const int cm = t >> lg, km = t & (nrhs - 1);
    if (to_cell_major) {
      if (cc < nc) tile[k][cc] = in[(long long)k * n + c0 + cc];
    } else {
      if (cm < nc) tile[km][cm] = in[(c0 + cm) * nrhs + km];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tot; t += kBlock) {
    const int k = t / kTrCells, cc = t % kTrCells;
    const int cm = t >> lg, km = t & (nrhs - 1);
    if (to_cell_major) {
      if (cm < nc) out[(c0 + cm) * nrhs + km] = tile[km][cm];
    } else {
      if (cc < nc) out[(long long)k * n + c0 + cc] = tile[k][cc];
    }
  }
}

inline unsigned grid_stream(long long n) {
  long long nb = (n + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  return (unsigned)(nb > 0 ? nb : 1);
}

inline unsigned red_blocks(long long nel) {
  long long nb = (nel + kBlock - 1) / kBlock;
  if (nb > kRedBlocks) nb = kRedBlocks;
  return (unsigned)(nb > 0 ? nb : 1);
}

}  // namespace

// ---------------------------------------------------------------- launchers

void launch_transpose(const double *in, double *out, int64_t n, int lg, int to_cell_major, hipStream_t st) {
  if (n > 0)
    k_transpose<<<(unsigned)((n + kTrCells - 1) / kTrCells), kBlock, 0, st>>>(in, out, n, lg, to_cell_major);
}

void launch_cast_d2f(const double *in, float *out, int64_t n, hipStream_t st) {
  if (n > 0) k_cast_d2f<<<grid_stream(n), kBlock, 0, st>>>(in, out, n);
}
void launch_cast_f2d(const float *in, double *out, int64_t n, hipStream_t st) {
  if (n > 0) k_cast_f2d<<<grid_stream(n), kBlock, 0, st>>>(in, out, n);
}
void launch_fill(double *x, double v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill<<<grid_stream(n), kBlock, 0, st>>>(x, v, n);
}
void launch_copy(const double *in, double *out, int64_t n, hipStream_t st) {
  if (n > 0) k_copy<<<grid_stream(n), kBlock, 0, st>>>(in, out, n);
}

void launch_dot(const double *a, const double *b, int64_t nel, int lg, double *partial, double *scal,
                int slot, int shift_rz, hipStream_t st) {
  const unsigned nb = red_blocks(nel);
  k_dot_partial<<<nb, kBlock, 0, st>>>(a, b, nel, lg, partial);
  k_dot_final<<<1, kFinalThreads, 0, st>>>(partial, (int)nb, lg, scal, slot, shift_rz, slot);
}

void launch_dot_final(const double *partial, int nblk, int lg, double *scal, int slot, hipStream_t st) {
  k_dot_final<<<1, kFinalThreads, 0, st>>>(partial, nblk, lg, scal, slot, 0, slot);
}

void launch_dot_final2(const double *partial, int nblk, int lg, double *scal, int slot_a, int shift_rz,
                       int slot_b, int nset, hipStream_t st) {
  k_dot_final<<<nset, kFinalThreads, 0, st>>>(partial, nblk, lg, scal, slot_a, shift_rz, slot_b);
}

void launch_dot2(const double *a, const double *b, const double *c, int64_t nel, int lg, double *partial,
                 double *scal, int slot_ab, int shift_rz, int slot_bc, hipStream_t st) {
  const unsigned nb = red_blocks(nel);
  k_dot2_partial<<<nb, kBlock, 0, st>>>(a, b, c, nel, lg, partial);
  k_dot_final<<<2, kFinalThreads, 0, st>>>(partial, (int)nb, lg, scal, slot_ab, shift_rz, slot_bc);
}

void launch_pcg_r(int64_t nel, int lg, double *scal, const int *active, double *r, const double *q,
                  double *partial, hipStream_t st, const float *w32, float *x32, const double *w64, double *x64) {
  const unsigned nb = red_blocks(nel);
  if (x64)
    k_pcg_r<double><<<nb, kBlock, 0, st>>>(nel, lg, scal, active, r, q, partial, w64, x64);
  else
    k_pcg_r<float><<<nb, kBlock, 0, st>>>(nel, lg, scal, active, r, q, partial, w32, x32);
  k_dot_final<<<1, kFinalThreads, 0, st>>>(partial, (int)nb, lg, scal, S_RR, 0, S_RR);
}

void launch_pcg_xp(int64_t nel, int lg, const double *scal, const int *active, int flexible,
                   const double *z, double *p, double *x, hipStream_t st) {
  k_pcg_xp<<<grid_stream(nel), kBlock, 0, st>>>(nel, lg, scal, active, flexible, z, p, x);
}

void launch_pcg_x(int64_t nel, int lg, const double *scal, const double *p, double *x, hipStream_t st) {
  k_pcg_x<<<grid_stream(nel), kBlock, 0, st>>>(nel, lg, scal, p, x);
}

void launch_resid_norm(const double *b, const double *ax, int64_t nel, int lg, double *partial,
                       double *scal, int slot, hipStream_t st) {
  const unsigned nb = red_blocks(nel);
  k_resid_partial<<<nb, kBlock, 0, st>>>(b, ax, nel, lg, partial);
  k_dot_final<<<1, kFinalThreads, 0, st>>>(partial, (int)nb, lg, scal, slot, 0, slot);
}

}  // namespace ssamg
