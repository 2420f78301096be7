// V-cycle and Krylov kernels (gfx950).
//
// Every grid-over-cells kernel runs one block row per part (blockIdx.y = part)
// and reads that part's PartDesc, so box extents, stencil offsets and pointers
// are wave-uniform and live in scalar registers.  Vectors are [cell][rhs] with
// nrhs = 1 << lg right-hand sides interleaved (rhs fastest): consecutive lanes
// touch consecutive addresses for any nrhs, and a stencil coefficient is read
// once per cell for all right-hand sides.
//
// The operations are those of Section 3.4 (weighted Jacobi, eq:relax0 with
// M = D / omega_p), the Galerkin transfers of Sections 3.2/3.3 (restriction
// R = P^T, interpolation by the two-point stencil of eq:prolEx) and the
// structured + unstructured matrix-vector product of Section 2 (A = S + U).
#include "ssamg_impl.h"

namespace ssamg {

namespace {

__device__ __forceinline__ void cell_ijk(int c, int nx, int ny, int &i, int &j, int &k) {
  i = c % nx;
  int t = c / nx;
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

// XCD-aware block order: consecutive chunks of one part land on one XCD, so
// the neighbour planes a block re-reads sit in that XCD's L2.
__device__ __forceinline__ int chunk_index() {
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  if ((nblk & 7) != 0) return b;
  return (b & 7) * (nblk >> 3) + (b >> 3);
}

// y = S x (APPLY), r = b - S x (RESID) or x' = x + omega (b - S x) / a_C
// (JACOBI) over every cell of every part.  T: coefficients and x; TB: b; TO:
// output.  FINE marks the launches on the finest level (own instantiation: in
// a mixed-precision cycle they read the FP64 PCG residual and write the FP64
// correction directly).
template <typename T, int MODE, typename TB, typename TO, int FINE>
__global__ __launch_bounds__(kBlock) void k_stencil(const PartDesc<T> *__restrict__ desc, int lg,
                                                    const T *__restrict__ x,
                                                    const TB *__restrict__ b, TO *__restrict__ y) {
  __shared__ int urow_of[kBlock];
  const PartDesc<T> &d = desc[blockIdx.y];
  const int chunk = chunk_index();
  const long long e = (long long)chunk * kBlock + threadIdx.x;
  const long long nel = d.ncell << lg;
  if ((long long)chunk * kBlock >= nel) return;      // whole block past the part's end
  const bool valid = e < nel;
  const int c = valid ? (int)(e >> lg) : 0;
  const int kr = (int)(e & ((1 << lg) - 1));
  int i, j, k;
  cell_ijk(c, d.n[0], d.n[1], i, j, k);
  const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const long long o = ((d.off + c) << lg) + kr;
  const T *xp = x + o;
  const T *cf = d.coef + c;
  T acc = T(0);
  if (valid) {
    for (int s = 0; s < d.nent; ++s) {
      const T a = cf[(long long)s * d.ncell];
      const T xv = nb_ok(mx, my, mz, d.code[s]) ? xp[(long long)d.lin[s] << lg] : T(0);
      acc = fma(a, xv, acc);
    }
  }
  // couplings of the cells of this block (part-boundary blocks only): map each
  // stored row to its cell slot in LDS, then each lane adds its row of U x
  const int u0 = d.ublk[lg][chunk], u1 = d.ublk[lg][chunk + 1];
  if (u0 < u1) {
    const int cpb = kBlock >> lg;
    const int cell0 = (int)d.off + chunk * cpb;
    if ((int)threadIdx.x < cpb) urow_of[threadIdx.x] = -1;
    __syncthreads();
    for (int t = u0 + (int)threadIdx.x; t < u1; t += kBlock) urow_of[d.urow[t] - cell0] = t;
    __syncthreads();
    const int r = urow_of[threadIdx.x >> lg];
    if (valid && r >= 0)
      for (int q = d.uptr[r]; q < d.uptr[r + 1]; ++q)
        acc = fma(d.uval[q], x[((long long)d.ucol[q] << lg) + kr], acc);
  }
  if (!valid) return;
  if (MODE == MODE_APPLY) {
    y[o] = (TO)acc;
  } else if (MODE == MODE_RESID) {
    y[o] = (TO)((T)b[o] - acc);
  } else {
    const T ac = cf[(long long)d.center * d.ncell];
    y[o] = (TO)(xp[0] + d.omega * ((T)b[o] - acc) / ac);
  }
}

// x = omega D^{-1} b: the first sweep of eq:relax0 from a zero guess
template <typename T, typename TB, int FINE>
__global__ __launch_bounds__(kBlock) void k_smooth_zero(const PartDesc<T> *__restrict__ desc, int lg,
                                                        const TB *__restrict__ b, T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  const int c = (int)(e >> lg);
  const long long o = ((d.off + c) << lg) + (e & ((1 << lg) - 1));
  x[o] = d.omega * (T)b[o] / d.coef[(long long)d.center * d.ncell + c];
}

// Coarsest level of a mixed-precision cycle: one sweep from zero computed in
// FP64 from the FP64 coarse operator, with FP32 input and output.
__global__ __launch_bounds__(kBlock) void k_coarse_mixed(const PartDesc<double> *__restrict__ desc,
                                                         int lg, const float *__restrict__ b,
                                                         float *__restrict__ x) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  const int c = (int)(e >> lg);
  const long long o = ((d.off + c) << lg) + (e & ((1 << lg) - 1));
  x[o] = (float)(d.omega * (double)b[o] / d.coef[(long long)d.center * d.ncell + c]);
}

// b_c = P^T r.  Coarse cell I (fine 2I along d*) gathers r(2I), the F cell
// 2I-1 through its +d* weight and the F cell 2I+1 through its -d* weight.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const PartDesc<T> *__restrict__ desc, int lg,
                                                     const T *__restrict__ r, T *__restrict__ bc) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.cncell << lg)) return;
  const int cc = (int)(e >> lg);
  const int kr = (int)(e & ((1 << lg) - 1));
  const long long oc = ((d.coff + cc) << lg) + kr;
  if (d.dstar < 0) {
    bc[oc] = r[((d.off + cc) << lg) + kr];
    return;
  }
  int ci[3];
  cell_ijk(cc, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  const int ds = d.dstar;
  int fi[3] = {ci[0], ci[1], ci[2]};
  fi[ds] = 2 * ci[ds];
  const int f0 = fi[0] + d.n[0] * (fi[1] + d.n[1] * fi[2]);
  const int stride = ds == 0 ? 1 : (ds == 1 ? d.n[0] : d.n[0] * d.n[1]);
  const T *rp = r + ((d.off + f0) << lg) + kr;
  T v = rp[0];
  int g[3] = {ci[0], ci[1], ci[2]};
  if (fi[ds] - 1 >= 0) {
    g[ds] = ci[ds] - 1;
    const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
    v = fma(d.wp[fl], rp[-((long long)stride << lg)], v);
  }
  if (fi[ds] + 1 <= d.n[ds] - 1) {
    g[ds] = ci[ds];
    const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
    v = fma(d.wm[fl], rp[(long long)stride << lg], v);
  }
  bc[oc] = v;
}

// x += P x_c: even cells along d* copy their coarse value, odd cells combine
// their two coarse neighbours with the F-box weights.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp_add(const PartDesc<T> *__restrict__ desc, int lg,
                                                       const T *__restrict__ xc,
                                                       T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  const int c = (int)(e >> lg);
  const int kr = (int)(e & ((1 << lg) - 1));
  const long long o = ((d.off + c) << lg) + kr;
  if (d.dstar < 0) {
    x[o] += xc[((d.coff + c) << lg) + kr];
    return;
  }
  int f[3];
  cell_ijk(c, d.n[0], d.n[1], f[0], f[1], f[2]);
  const int ds = d.dstar;
  const int id = f[ds];
  int g[3] = {f[0], f[1], f[2]};
  if ((id & 1) == 0) {
    g[ds] = id >> 1;
    x[o] += xc[((d.coff + g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2])) << lg) + kr];
    return;
  }
  g[ds] = (id - 1) >> 1;
  const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
  const int cm = g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2]);
  T v = d.wm[fl] * xc[((d.coff + cm) << lg) + kr];
  if (id + 1 <= d.n[ds] - 1) {
    const int cstride = ds == 0 ? 1 : (ds == 1 ? d.cn[0] : d.cn[0] * d.cn[1]);
    v = fma(d.wp[fl], xc[((d.coff + cm + cstride) << lg) + kr], v);
  }
  x[o] += v;
}

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

// slot <- sum of partials; shift_rz: first move S_RZN to S_RZ (PCG bookkeeping)
__global__ __launch_bounds__(kBlock) void k_dot_final(const double *__restrict__ partial, int nblk,
                                                      int lg, double *__restrict__ scal, int slot,
                                                      int shift_rz) {
  __shared__ double sh[kBlock];
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  double acc = 0.0;
  for (int bidx = threadIdx.x >> lg; bidx < nblk; bidx += kBlock >> lg)
    acc += partial[bidx * kMaxRhs + kr];
  sh[threadIdx.x] = acc;
  block_tree(sh, nr);
  if ((int)threadIdx.x < nr) {
    if (shift_rz) scal[S_RZ * kMaxRhs + threadIdx.x] = scal[S_RZN * kMaxRhs + threadIdx.x];
    scal[slot * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
  }
}

// x += alpha p, r -= alpha q with alpha = rz/pq per right-hand side (0 when
// frozen), plus the partial sums of r.r
__global__ __launch_bounds__(kBlock) void k_pcg_xr(long long nel, int lg,
                                                   const double *__restrict__ scal,
                                                   const int *__restrict__ active,
                                                   double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ partial) {
  __shared__ double sh[kBlock];
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  const bool act = active[kr] != 0;
  const double alpha = act ? scal[S_RZN * kMaxRhs + kr] / scal[S_PQ * kMaxRhs + kr] : 0.0;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock) {
    double ri = r[i];
    if (act) {
      x[i] = fma(alpha, p[i], x[i]);
      ri = fma(-alpha, q[i], ri);
      r[i] = ri;
    }
    acc = fma(ri, ri, acc);
  }
  sh[threadIdx.x] = acc;
  block_tree(sh, nr);
  if ((int)threadIdx.x < nr) partial[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
}

// p = z + beta p; beta = rz_new/rz_old, or -(z.q)/(p.q) for flexible CG
__global__ __launch_bounds__(kBlock) void k_pcg_p(long long nel, int lg,
                                                  const double *__restrict__ scal,
                                                  const int *__restrict__ active, int flexible,
                                                  const double *__restrict__ z,
                                                  double *__restrict__ p) {
  const int nr = 1 << lg;
  const int kr = threadIdx.x & (nr - 1);
  double beta = flexible ? -scal[S_ZQ * kMaxRhs + kr] / scal[S_PQ * kMaxRhs + kr]
                         : scal[S_RZN * kMaxRhs + kr] / scal[S_RZ * kMaxRhs + kr];
  if (!active[kr]) beta = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nel;
       i += (long long)gridDim.x * kBlock)
    p[i] = fma(beta, p[i], z[i]);
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

inline unsigned grid_cells(long long n, int lg) {
  long long nb = ((n << lg) + kBlock - 1) / kBlock;
  return (unsigned)(nb > 0 ? nb : 1);
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

template <typename T, typename TB, typename TO>
void launch_stencil(int mode, int fine, const PartDesc<T> *desc, int nparts, int maxcell, int lg,
                    const T *x, const TB *b, TO *y, hipStream_t st) {
  dim3 grid(grid_cells(maxcell, lg), nparts);
#define SSAMG_ST(M, F) k_stencil<T, M, TB, TO, F><<<grid, kBlock, 0, st>>>(desc, lg, x, b, y)
  if (fine) {
    if (mode == MODE_APPLY) SSAMG_ST(MODE_APPLY, 1);
    else if (mode == MODE_RESID) SSAMG_ST(MODE_RESID, 1);
    else SSAMG_ST(MODE_JACOBI, 1);
  } else {
    if (mode == MODE_APPLY) SSAMG_ST(MODE_APPLY, 0);
    else if (mode == MODE_RESID) SSAMG_ST(MODE_RESID, 0);
    else SSAMG_ST(MODE_JACOBI, 0);
  }
#undef SSAMG_ST
}

template <typename T, typename TB>
void launch_smooth_zero(int fine, const PartDesc<T> *desc, int nparts, int maxcell, int lg, const TB *b,
                        T *x, hipStream_t st) {
  if (fine)
    k_smooth_zero<T, TB, 1><<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
  else
    k_smooth_zero<T, TB, 0><<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
}

template <typename T>
void launch_restrict(const PartDesc<T> *desc, int nparts, int maxcoarse, int lg, const T *r, T *bc,
                     hipStream_t st) {
  k_restrict<T><<<dim3(grid_cells(maxcoarse, lg), nparts), kBlock, 0, st>>>(desc, lg, r, bc);
}

template <typename T>
void launch_interp_add(const PartDesc<T> *desc, int nparts, int maxcell, int lg, const T *xc, T *x,
                       hipStream_t st) {
  k_interp_add<T><<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, xc, x);
}

void launch_coarse_mixed(const PartDesc<double> *desc, int nparts, int maxcell, int lg, const float *b,
                         float *x, hipStream_t st) {
  k_coarse_mixed<<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
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
  k_dot_final<<<1, kBlock, 0, st>>>(partial, (int)nb, lg, scal, slot, shift_rz);
}

void launch_pcg_xr(int64_t nel, int lg, const double *scal, const int *active, double *x, double *r,
                   const double *p, const double *q, double *partial, double *scal_out,
                   hipStream_t st) {
  const unsigned nb = red_blocks(nel);
  k_pcg_xr<<<nb, kBlock, 0, st>>>(nel, lg, scal, active, x, r, p, q, partial);
  k_dot_final<<<1, kBlock, 0, st>>>(partial, (int)nb, lg, scal_out, S_RR, 0);
}

void launch_pcg_p(int64_t nel, int lg, const double *scal, const int *active, int flexible,
                  const double *z, double *p, hipStream_t st) {
  k_pcg_p<<<grid_stream(nel), kBlock, 0, st>>>(nel, lg, scal, active, flexible, z, p);
}

void launch_resid_norm(const double *b, const double *ax, int64_t nel, int lg, double *partial,
                       double *scal, int slot, hipStream_t st) {
  const unsigned nb = red_blocks(nel);
  k_resid_partial<<<nb, kBlock, 0, st>>>(b, ax, nel, lg, partial);
  k_dot_final<<<1, kBlock, 0, st>>>(partial, (int)nb, lg, scal, slot, 0);
}

template void launch_stencil<double, double, double>(int, int, const PartDesc<double> *, int, int, int,
                                                     const double *, const double *, double *, hipStream_t);
template void launch_stencil<float, float, float>(int, int, const PartDesc<float> *, int, int, int,
                                                  const float *, const float *, float *, hipStream_t);
template void launch_stencil<float, double, float>(int, int, const PartDesc<float> *, int, int, int,
                                                   const float *, const double *, float *, hipStream_t);
template void launch_stencil<float, double, double>(int, int, const PartDesc<float> *, int, int, int,
                                                    const float *, const double *, double *, hipStream_t);
template void launch_smooth_zero<double, double>(int, const PartDesc<double> *, int, int, int,
                                                 const double *, double *, hipStream_t);
template void launch_smooth_zero<float, float>(int, const PartDesc<float> *, int, int, int, const float *,
                                               float *, hipStream_t);
template void launch_smooth_zero<float, double>(int, const PartDesc<float> *, int, int, int,
                                                const double *, float *, hipStream_t);
template void launch_restrict<double>(const PartDesc<double> *, int, int, int, const double *, double *,
                                      hipStream_t);
template void launch_restrict<float>(const PartDesc<float> *, int, int, int, const float *, float *,
                                     hipStream_t);
template void launch_interp_add<double>(const PartDesc<double> *, int, int, int, const double *, double *,
                                        hipStream_t);
template void launch_interp_add<float>(const PartDesc<float> *, int, int, int, const float *, float *,
                                       hipStream_t);

}  // namespace ssamg
