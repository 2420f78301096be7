// Exact solve of a coarse level as a dense FP64 inverse (gfx950): the hybrid
// coarse tail of Section 3.5, where the multigrid hierarchy stops at a chosen
// level and that level's operator is solved directly.
//
// The operator A_k (n cells, stencils + couplings) is written into a dense
// matrix padded to np = 64 * ceil(n / 64) with identity rows, then inverted in
// place by blocked Gauss-Jordan elimination without pivoting (A_k is SPD, so
// every pivot block is SPD).  Step K (64 columns):
//   D^{-1}          one workgroup, in LDS
//   A[K, J] = D^{-1} A[K, J]          (row panel, J != K)
//   A[I, J] -= A[I, K] A[K, J]        (rank-64 update, I, J != K: FP64 MFMA)
//   A[I, K] = -A[I, K] D^{-1},  A[K, K] = D^{-1}
// The rank-64 update carries almost all of the 2 np^3 flops; it runs on the
// v_mfma_f64_16x16x4 matrix cores with the column panel in a transposed copy so
// that every operand load is unit-stride across the lanes.
// Applying the inverse is a matrix-vector (or matrix-matrix, several
// right-hand sides) product split over column chunks: partial sums per chunk,
// then a fixed-order sum over the chunks.
#include "device_util.h"
#include "ssamg_impl.h"

namespace ssamg {

namespace {

constexpr int kNb = 64;          // Gauss-Jordan block
constexpr int kApplyRows = 256;  // rows of one apply block (one per thread)
constexpr int kApplyCols = 256;  // columns (inner index) of one apply chunk

// ---- dense operator of one level

__global__ __launch_bounds__(kBlock) void k_dense_fill(double *__restrict__ a, long long npad, long long n) {
  const long long total = npad * npad;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const long long i = t / npad, j = t - i * npad;
    a[t] = (i == j && i >= n) ? 1.0 : 0.0;
  }
}

// row c of the level's stencil part (one thread per cell)
__global__ __launch_bounds__(kBlock) void k_dense_stencil(const PartDesc<double> *__restrict__ desc,
                                                          double *__restrict__ a, long long npad) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.ncell) return;
  const int i = (int)(c % d.n[0]);
  const int j = (int)((c / d.n[0]) % d.n[1]);
  const int k = (int)(c / ((long long)d.n[0] * d.n[1]));
  const long long row = d.off + c;
  for (int s = 0; s < d.nent; ++s) {
    const int dx = (d.code[s] & 3) - 1, dy = ((d.code[s] >> 2) & 3) - 1, dz = ((d.code[s] >> 4) & 3) - 1;
    if (i + dx < 0 || i + dx >= d.n[0] || j + dy < 0 || j + dy >= d.n[1] || k + dz < 0 || k + dz >= d.n[2])
      continue;
    const double v = dev::G(d.coef)[(long long)s * d.ncell + c];
    a[row * npad + row + d.lin[s]] += v;
  }
}

// the couplings U (one thread per stored row)
__global__ __launch_bounds__(kBlock) void k_dense_coupling(int nrow, const int *__restrict__ urow,
                                                           const int *__restrict__ uptr,
                                                           const int *__restrict__ ucol,
                                                           const double *__restrict__ uval,
                                                           double *__restrict__ a, long long npad) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrow) return;
  const long long row = urow[r];
  for (int q = uptr[r]; q < uptr[r + 1]; ++q) a[row * npad + ucol[q]] += uval[q];
}

// ---- blocked Gauss-Jordan inversion

// D^{-1} of the pivot block K (64 x 64), unpivoted Gauss-Jordan in LDS; flag 2
// when a pivot is not positive (the operator is not positive definite).
__global__ __launch_bounds__(kBlock) void k_gj_diag(const double *__restrict__ a, long long npad, int kb,
                                                    double *__restrict__ dinv, int *__restrict__ flag) {
  __shared__ double m[kNb][kNb + 1];
  __shared__ double colp[kNb], rowp[kNb];
  const long long k0 = (long long)kb * kNb;
  for (int t = threadIdx.x; t < kNb * kNb; t += kBlock) {
    const int r = t / kNb, c = t % kNb;
    m[r][c] = a[(k0 + r) * npad + k0 + c];
  }
  __syncthreads();
  for (int p = 0; p < kNb; ++p) {
    const double piv = m[p][p];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) flag[0] = 2;
      return;   // block-uniform: every thread read the same pivot
    }
    const double inv = 1.0 / piv;
    if (threadIdx.x < kNb) {
      colp[threadIdx.x] = m[threadIdx.x][p];
      rowp[threadIdx.x] = m[p][threadIdx.x] * inv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kNb * kNb; t += kBlock) {
      const int r = t / kNb, c = t % kNb;
      if (r == p && c == p)
        m[r][c] = inv;
      else if (r == p)
        m[r][c] = rowp[c];
      else if (c == p)
        m[r][c] = -colp[r] * inv;
      else
        m[r][c] = m[r][c] - colp[r] * rowp[c];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < kNb * kNb; t += kBlock) dinv[t] = m[t / kNb][t % kNb];
}

// Row panel A[K, j] = D^{-1} A[K, j] for j outside K (one thread per column),
// and the transposed copy pt[m][i] = A[i][K0 + m] of the column panel (all i),
// which the update and the column step read.
__global__ __launch_bounds__(kBlock) void k_gj_panels(double *__restrict__ a, long long npad, int kb,
                                                      const double *__restrict__ dinv,
                                                      double *__restrict__ pt) {
  __shared__ double dv[kNb][kNb + 1];
  for (int t = threadIdx.x; t < kNb * kNb; t += kBlock) dv[t / kNb][t % kNb] = dinv[t];
  __syncthreads();
  const long long k0 = (long long)kb * kNb;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= npad) return;
  // transposed column panel: thread j copies row j's 64 entries of columns K
  for (int m = 0; m < kNb; ++m) pt[(long long)m * npad + j] = a[j * npad + k0 + m];
  if (j >= k0 && j < k0 + kNb) return;
  double col[kNb];
#pragma unroll
  for (int m = 0; m < kNb; ++m) col[m] = a[(k0 + m) * npad + j];
#pragma unroll 4
  for (int r = 0; r < kNb; ++r) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kNb; ++m) s = fma(dv[r][m], col[m], s);
    a[(k0 + r) * npad + j] = s;
  }
}

// Rank-64 update of every 64 x 64 tile (I, J) outside block row and column K:
// A[I, J] -= A[I, K] A[K, J], with A[I, K] read from the transposed copy pt and
// A[K, J] (already the row panel) from the matrix.  Four waves per tile, each a
// 32 x 32 quarter as 2 x 2 products of 16 x 16 on v_mfma_f64_16x16x4: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] of each 16 x 4 x 16 step and
// holds D[l / 16 + 4 v][l % 16], v = 0..3 (the FP64 form keeps one row per
// register group: rows of one lane are 4 apart, unlike the FP32 16 x 16 forms).
__global__ __launch_bounds__(kBlock) void k_gj_update(double *__restrict__ a, long long npad, int kb,
                                                      const double *__restrict__ pt) {
  const int nbk = (int)(npad / kNb);
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi == kb || bj == kb || bi >= nbk || bj >= nbk) return;   // block-uniform
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long r0 = (long long)bi * kNb + (w >> 1) * 32, c0 = (long long)bj * kNb + (w & 1) * 32;
  const long long k0 = (long long)kb * kNb;
  const int li = lane & 15, lk = lane >> 4;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[ti][tj][v] = a[(r0 + ti * 16 + lk + 4 * v) * npad + c0 + tj * 16 + li];
#pragma unroll 4
  for (int s = 0; s < kNb / 4; ++s) {
    const long long kk = 4 * s + lk;
    double av[2], bv[2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) av[ti] = -pt[kk * npad + r0 + ti * 16 + li];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) bv[tj] = a[(k0 + kk) * npad + c0 + tj * 16 + li];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) a[(r0 + ti * 16 + lk + 4 * v) * npad + c0 + tj * 16 + li] = acc[ti][tj][v];
}

// Column panel A[i, K] = -A[i, K] D^{-1} for i outside K (one thread per row,
// the old values from pt), and A[K, K] = D^{-1}.
__global__ __launch_bounds__(kBlock) void k_gj_column(double *__restrict__ a, long long npad, int kb,
                                                      const double *__restrict__ dinv,
                                                      const double *__restrict__ pt) {
  __shared__ double dv[kNb][kNb + 1];
  for (int t = threadIdx.x; t < kNb * kNb; t += kBlock) dv[t / kNb][t % kNb] = dinv[t];
  __syncthreads();
  const long long k0 = (long long)kb * kNb;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= npad) return;
  if (i >= k0 && i < k0 + kNb) {
    const int r = (int)(i - k0);
    for (int c = 0; c < kNb; ++c) a[i * npad + k0 + c] = dv[r][c];
    return;
  }
  double old[kNb];
#pragma unroll
  for (int m = 0; m < kNb; ++m) old[m] = pt[(long long)m * npad + i];
#pragma unroll 4
  for (int c = 0; c < kNb; ++c) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kNb; ++m) s = fma(old[m], dv[m][c], s);
    a[i * npad + k0 + c] = -s;
  }
}

// ---- applying the inverse: vt = M vb for 1 << lg right-hand sides

// partial[chunk][row][k] = sum over the chunk's inner indices j of M[j][row] vb[j][k]
// (M is symmetric; reading it by columns makes the loads unit-stride across rows)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_apply_part(const double *__restrict__ m, long long npad,
                                                            long long n, int lg, const T *__restrict__ vb,
                                                            double *__restrict__ part) {
  __shared__ double bs[kApplyCols * 4];
  const int nr = 1 << lg;
  const long long row = (long long)blockIdx.x * kApplyRows + threadIdx.x;
  const long long j0 = (long long)blockIdx.y * kApplyCols;
  const long long j1 = j0 + kApplyCols < n ? j0 + kApplyCols : n;
  // right-hand sides in groups of 4: the chunk's b values of the group in LDS
  for (int k0 = 0; k0 < nr; k0 += 4) {
    const int kn = nr - k0 < 4 ? nr - k0 : 4;
    __syncthreads();
    for (int t = threadIdx.x; t < kApplyCols * 4; t += kBlock) {
      const long long j = j0 + t / 4;
      const int kk = t % 4;
      bs[t] = (j < j1 && kk < kn) ? (double)vb[(j << lg) + k0 + kk] : 0.0;
    }
    __syncthreads();
    if (row >= n) continue;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long j = j0; j < j1; ++j) {
      const double mv = m[j * npad + row];
      const double *bj = bs + (j - j0) * 4;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc[kk] = fma(mv, bj[kk], acc[kk]);
    }
    for (int kk = 0; kk < kn; ++kk) part[(((long long)blockIdx.y * n + row) << lg) + k0 + kk] = acc[kk];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_apply_sum(const double *__restrict__ part, int nchunk,
                                                           long long nel, T *__restrict__ vt) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nel) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(long long)c * nel + e];
  vt[e] = (T)s;
}

inline unsigned nblk(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

int64_t dense_pad(int64_t n) { return ((n + kNb - 1) / kNb) * kNb; }

int64_t dense_apply_chunks(int64_t n) { return (n + kApplyCols - 1) / kApplyCols; }

void launch_dense_inverse(const PartDesc<double> *desc, int nparts, int maxcell, int64_t n, int nrow,
                          const int *urow, const int *uptr, const int *ucol, const double *uval, double *a,
                          double *pt, double *dinv, int *flag, hipStream_t st) {
  const int64_t npad = dense_pad(n);
  const long long total = npad * npad;
  const unsigned fb = (unsigned)std::min<long long>((total + kBlock - 1) / kBlock, 65536);
  k_dense_fill<<<fb, kBlock, 0, st>>>(a, npad, n);
  k_dense_stencil<<<dim3(nblk(maxcell), nparts), kBlock, 0, st>>>(desc, a, npad);
  if (nrow > 0) k_dense_coupling<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, ucol, uval, a, npad);
  const int nbk = (int)(npad / kNb);
  for (int kb = 0; kb < nbk; ++kb) {
    k_gj_diag<<<1, kBlock, 0, st>>>(a, npad, kb, dinv, flag);
    k_gj_panels<<<nblk(npad), kBlock, 0, st>>>(a, npad, kb, dinv, pt);
    if (nbk > 1) k_gj_update<<<dim3(nbk, nbk), kBlock, 0, st>>>(a, npad, kb, pt);
    k_gj_column<<<nblk(npad), kBlock, 0, st>>>(a, npad, kb, dinv, pt);
  }
}

template <typename T>
void launch_dense_apply(const double *m, int64_t n, int lg, const T *vb, T *vt, double *part, hipStream_t st) {
  const int64_t npad = dense_pad(n);
  const unsigned nchunk = (unsigned)dense_apply_chunks(n);
  const unsigned nrb = (unsigned)((n + kApplyRows - 1) / kApplyRows);
  k_dense_apply_part<T><<<dim3(nrb, nchunk), kBlock, 0, st>>>(m, npad, n, lg, vb, part);
  k_dense_apply_sum<T><<<nblk(n << lg), kBlock, 0, st>>>(part, (int)nchunk, n << lg, vt);
}

template void launch_dense_apply<double>(const double *, int64_t, int, const double *, double *, double *,
                                         hipStream_t);
template void launch_dense_apply<float>(const double *, int64_t, int, const float *, float *, double *,
                                        hipStream_t);

}  // namespace ssamg
