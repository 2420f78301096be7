// V(1,1)-cycle kernels (gfx950): stencil sweeps with the couplings U fused in,
// the first smoothing sweep from zero, restriction and interpolation, and a
// one-workgroup kernel that runs the whole coarse end of the cycle.
//
// Every grid-over-cells kernel runs one block row per part (blockIdx.y = part)
// and reads that part's PartDesc, so box extents, stencil offsets and pointers
// are wave-uniform.  Vectors are [cell][rhs] with nrhs = 1 << lg right-hand
// sides interleaved (rhs fastest): consecutive lanes touch consecutive
// addresses for any nrhs, and a coefficient is read once per cell for all of
// them.
//
// Operations: weighted Jacobi or weighted L1-Jacobi sweeps (Section 3.4,
// eq:relax0), restriction R = P^T and interpolation by the two-point stencil
// of eq:prolEx (Sections 3.2, 3.3), and the semi-structured product
// A x = S x + U x (Section 2).
#include "device_util.h"
#include "ssamg_impl.h"

namespace ssamg {

namespace {

using dev::cell_ijk;
using dev::chunk_index;
using dev::nb_mask;
using dev::nb_ok;

constexpr int kTailThreads = 1024;

// smoother factor of cell c: omega_p / a_ii (Jacobi) or factor / sum|a_ij| (L1)
template <typename T>
__device__ __forceinline__ T smooth_factor(const PartDesc<T> &d, long long c) {
  return d.rs ? d.rs[c] : d.omega / d.coef[(long long)d.center * d.ncell + c];
}

// sum_s a_s(c) x(c + s) over the part's stencil; all loads are issued before
// the first multiply (entries s >= nent are masked off)
template <typename T, int NENT>
__device__ __forceinline__ T stencil_acc(const PartDesc<T> &d, int c, int lg, const T *xp) {
  int i, j, k;
  cell_ijk(c, d.n[0], d.n[1], i, j, k);
  const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const T *cf = d.coef + c;
  T a[NENT], xv[NENT];
#pragma unroll
  for (int s = 0; s < NENT; ++s) {
    const bool act = s < d.nent;
    a[s] = act ? cf[(long long)s * d.ncell] : T(0);
    xv[s] = (act && nb_ok(mx, my, mz, d.code[s])) ? xp[(long long)d.lin[s] << lg] : T(0);
  }
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < NENT; ++s) acc = fma(a[s], xv[s], acc);
  return acc;
}

// row r of U times x, four entries in flight at a time
template <typename T>
__device__ __forceinline__ T coupling_row(const int *__restrict__ uptr, const int *__restrict__ ucol,
                                         const T *__restrict__ uval, int r, int lg, int kr,
                                         const T *__restrict__ x) {
  const int q0 = uptr[r], q1 = uptr[r + 1];
  T acc = T(0);
  for (int q = q0; q < q1; q += 4) {
    int cc[4];
    T vv[4], xx[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool in = q + t < q1;
      cc[t] = in ? ucol[q + t] : 0;
      vv[t] = in ? uval[q + t] : T(0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) xx[t] = q + t < q1 ? x[((long long)cc[t] << lg) + kr] : T(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = fma(vv[t], xx[t], acc);
  }
  return acc;
}

// b_c = P^T r for coarse cell cc: r(2I) + wp(2I-1) r(2I-1) + wm(2I+1) r(2I+1)
template <typename T>
__device__ __forceinline__ void restrict_one(const PartDesc<T> &d, int cc, int kr, int lg,
                                             const T *__restrict__ r, T *__restrict__ bc) {
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

// x(c) += (P x_c)(c): even cells along d* take their coarse value, odd cells
// combine their two coarse neighbours with the F-box weights
template <typename T>
__device__ __forceinline__ void interp_one(const PartDesc<T> &d, int c, int kr, int lg,
                                           const T *__restrict__ xc, T *__restrict__ x) {
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

// y = S x + U x (APPLY), r = b - A x (RESID) or x' = x + w (b - A x) (JACOBI,
// w the smoother factor) over every cell of every part.  T: coefficients and
// x; TB: b; TO: output.  NENT bounds the entries of the level's stencils.
// FINE marks finest-level launches (own instantiation: in a mixed-precision
// cycle they read the FP64 residual and write the FP64 correction directly).
// Blocks that hold rows of U map those rows to their cell slots in LDS.
template <typename T, int MODE, typename TB, typename TO, int FINE, int NENT>
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
  const long long o = ((d.off + c) << lg) + kr;
  const T *xp = x + o;
  T acc = valid ? stencil_acc<T, NENT>(d, c, lg, xp) : T(0);
  const int u0 = d.ublk[lg][chunk], u1 = d.ublk[lg][chunk + 1];
  if (u0 < u1) {
    const int cpb = kBlock >> lg;
    const int cell0 = (int)d.off + chunk * cpb;
    if ((int)threadIdx.x < cpb) urow_of[threadIdx.x] = -1;
    __syncthreads();
    for (int t = u0 + (int)threadIdx.x; t < u1; t += kBlock) urow_of[d.urow[t] - cell0] = t;
    __syncthreads();
    const int r = urow_of[threadIdx.x >> lg];
    if (valid && r >= 0) acc += coupling_row<T>(d.uptr, d.ucol, d.uval, r, lg, kr, x);
  }
  if (!valid) return;
  if (MODE == MODE_APPLY) {
    y[o] = (TO)acc;
  } else if (MODE == MODE_RESID) {
    y[o] = (TO)((T)b[o] - acc);
  } else {
    y[o] = (TO)(xp[0] + smooth_factor(d, c) * ((T)b[o] - acc));
  }
}

// The first sweep of eq:relax0 from a zero guess, x = w b, fused with the
// residual r = b - A x: the iterate at a neighbour is formed there from its
// own factor and right-hand side, so x and b are each read once.
template <typename T, typename TB, int FINE, int NENT>
__global__ __launch_bounds__(kBlock) void k_smooth_resid(const PartDesc<T> *__restrict__ desc, int lg,
                                                         const TB *__restrict__ b,
                                                         T *__restrict__ x, T *__restrict__ r) {
  __shared__ int urow_of[kBlock];
  const PartDesc<T> &d = desc[blockIdx.y];
  const int chunk = chunk_index();
  const long long e = (long long)chunk * kBlock + threadIdx.x;
  const long long nel = d.ncell << lg;
  if ((long long)chunk * kBlock >= nel) return;
  const bool valid = e < nel;
  const int c = valid ? (int)(e >> lg) : 0;
  const int kr = (int)(e & ((1 << lg) - 1));
  const long long o = ((d.off + c) << lg) + kr;
  const TB *bp = b + o;
  const T *wp = d.rs + c;
  T acc = T(0);
  if (valid) {
    int i, j, k;
    cell_ijk(c, d.n[0], d.n[1], i, j, k);
    const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
    const T *cf = d.coef + c;
    T a[NENT], bv[NENT], wv[NENT];
#pragma unroll
    for (int s = 0; s < NENT; ++s) {
      const bool act = s < d.nent;
      const bool ok = act && nb_ok(mx, my, mz, d.code[s]);
      a[s] = act ? cf[(long long)s * d.ncell] : T(0);
      bv[s] = ok ? (T)bp[(long long)d.lin[s] << lg] : T(0);
      wv[s] = ok ? wp[d.lin[s]] : T(0);
    }
#pragma unroll
    for (int s = 0; s < NENT; ++s) acc = fma(a[s], wv[s] * bv[s], acc);
  }
  const int u0 = d.ublk[lg][chunk], u1 = d.ublk[lg][chunk + 1];
  if (u0 < u1) {
    const int cpb = kBlock >> lg;
    const int cell0 = (int)d.off + chunk * cpb;
    if ((int)threadIdx.x < cpb) urow_of[threadIdx.x] = -1;
    __syncthreads();
    for (int t = u0 + (int)threadIdx.x; t < u1; t += kBlock) urow_of[d.urow[t] - cell0] = t;
    __syncthreads();
    const int rr = urow_of[threadIdx.x >> lg];
    if (valid && rr >= 0) {
      const T *wl = d.rs - d.off;   // factors of the whole level
      const int q0 = d.uptr[rr], q1 = d.uptr[rr + 1];
      for (int q = q0; q < q1; q += 4) {
        int cc[4];
        T vv[4], xx[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool in = q + t < q1;
          cc[t] = in ? d.ucol[q + t] : 0;
          vv[t] = in ? d.uval[q + t] : T(0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
          xx[t] = q + t < q1 ? wl[cc[t]] * (T)b[((long long)cc[t] << lg) + kr] : T(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = fma(vv[t], xx[t], acc);
      }
    }
  }
  if (!valid) return;
  const T b0 = (T)bp[0];
  x[o] = wp[0] * b0;
  r[o] = b0 - acc;
}

// x = w b: the first sweep of eq:relax0 from a zero guess
template <typename T, typename TB, int FINE>
__global__ __launch_bounds__(kBlock) void k_smooth_zero(const PartDesc<T> *__restrict__ desc, int lg,
                                                        const TB *__restrict__ b, T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  const int c = (int)(e >> lg);
  const long long o = ((d.off + c) << lg) + (e & ((1 << lg) - 1));
  x[o] = smooth_factor(d, c) * (T)b[o];
}

// One sweep from zero on the coarsest level computed in FP64 from the FP64
// operator, FP32 input and output (mixed-precision cycle, single level case).
__global__ __launch_bounds__(kBlock) void k_coarse_mixed(const PartDesc<double> *__restrict__ desc,
                                                         int lg, const float *__restrict__ b,
                                                         float *__restrict__ x) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  const int c = (int)(e >> lg);
  const long long o = ((d.off + c) << lg) + (e & ((1 << lg) - 1));
  x[o] = (float)(smooth_factor(d, c) * (double)b[o]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const PartDesc<T> *__restrict__ desc, int lg,
                                                     const T *__restrict__ r, T *__restrict__ bc) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.cncell << lg)) return;
  restrict_one(d, (int)(e >> lg), (int)(e & ((1 << lg) - 1)), lg, r, bc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp_add(const PartDesc<T> *__restrict__ desc, int lg,
                                                       const T *__restrict__ xc,
                                                       T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lg)) return;
  interp_one(d, (int)(e >> lg), (int)(e & ((1 << lg) - 1)), lg, xc, x);
}

// The coarse end of one V(1,1) cycle, levels tl[0] .. tl[nl-1] (the last one
// the coarsest), in a single workgroup: the same operations as the grid
// kernels, one phase at a time with a workgroup barrier between phases.  The
// couplings are applied as a separate phase over the rows of U.
template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailLevel<T> *__restrict__ tl, int nl,
                                                       int lg) {
  const int tid = threadIdx.x;
  const int mask = (1 << lg) - 1;
  for (int i = 0; i + 1 < nl; ++i) {
    const TailLevel<T> &v = tl[i];
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<T> &d = v.desc[p];
      for (long long e = tid; e < (d.ncell << lg); e += kTailThreads) {
        const int c = (int)(e >> lg);
        const long long o = ((d.off + c) << lg) + (e & mask);
        v.vx[o] = smooth_factor(d, c) * v.vb[o];
      }
    }
    __syncthreads();
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<T> &d = v.desc[p];
      for (long long e = tid; e < (d.ncell << lg); e += kTailThreads) {
        const int c = (int)(e >> lg);
        const long long o = ((d.off + c) << lg) + (e & mask);
        v.vt[o] = v.vb[o] - stencil_acc<T, kMaxEnt>(d, c, lg, v.vx + o);
      }
    }
    __syncthreads();
    for (long long e = tid; e < ((long long)v.nrow << lg); e += kTailThreads) {
      const int r = (int)(e >> lg), kr = (int)(e & mask);
      v.vt[((long long)v.urow[r] << lg) + kr] -= coupling_row<T>(v.uptr, v.ucol, v.uval, r, lg, kr, v.vx);
    }
    __syncthreads();
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<T> &d = v.desc[p];
      for (long long e = tid; e < (d.cncell << lg); e += kTailThreads)
        restrict_one(d, (int)(e >> lg), (int)(e & mask), lg, v.vt, tl[i + 1].vb);
    }
    __syncthreads();
  }
  {
    const TailLevel<T> &v = tl[nl - 1];
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<double> &d = v.desc64[p];
      for (long long e = tid; e < (d.ncell << lg); e += kTailThreads) {
        const int c = (int)(e >> lg);
        const long long o = ((d.off + c) << lg) + (e & mask);
        v.vt[o] = (T)(smooth_factor(d, c) * (double)v.vb[o]);
      }
    }
    __syncthreads();
  }
  for (int i = nl - 2; i >= 0; --i) {
    const TailLevel<T> &v = tl[i];
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<T> &d = v.desc[p];
      for (long long e = tid; e < (d.ncell << lg); e += kTailThreads)
        interp_one(d, (int)(e >> lg), (int)(e & mask), lg, tl[i + 1].vt, v.vx);
    }
    __syncthreads();
    for (int p = 0; p < v.np; ++p) {
      const PartDesc<T> &d = v.desc[p];
      for (long long e = tid; e < (d.ncell << lg); e += kTailThreads) {
        const int c = (int)(e >> lg);
        const long long o = ((d.off + c) << lg) + (e & mask);
        const T acc = stencil_acc<T, kMaxEnt>(d, c, lg, v.vx + o);
        v.vt[o] = v.vx[o] + smooth_factor(d, c) * (v.vb[o] - acc);
      }
    }
    __syncthreads();
    for (long long e = tid; e < ((long long)v.nrow << lg); e += kTailThreads) {
      const int r = (int)(e >> lg), kr = (int)(e & mask);
      const int cell = v.urow[r];
      int p = 0;
      while (p + 1 < v.np && v.desc[p + 1].off <= cell) ++p;
      const PartDesc<T> &d = v.desc[p];
      const T w = smooth_factor(d, cell - d.off);
      v.vt[((long long)cell << lg) + kr] -= w * coupling_row<T>(v.uptr, v.ucol, v.uval, r, lg, kr, v.vx);
    }
    __syncthreads();
  }
}

inline unsigned grid_cells(long long n, int lg) {
  long long nb = ((n << lg) + kBlock - 1) / kBlock;
  return (unsigned)(nb > 0 ? nb : 1);
}

template <typename T, typename TB, typename TO, int FINE, int NENT>
void stencil_mode(int mode, dim3 grid, const PartDesc<T> *desc, int lg, const T *x, const TB *b, TO *y,
                  hipStream_t st) {
  if (mode == MODE_APPLY)
    k_stencil<T, MODE_APPLY, TB, TO, FINE, NENT><<<grid, kBlock, 0, st>>>(desc, lg, x, b, y);
  else if (mode == MODE_RESID)
    k_stencil<T, MODE_RESID, TB, TO, FINE, NENT><<<grid, kBlock, 0, st>>>(desc, lg, x, b, y);
  else
    k_stencil<T, MODE_JACOBI, TB, TO, FINE, NENT><<<grid, kBlock, 0, st>>>(desc, lg, x, b, y);
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T, typename TB, typename TO>
void launch_stencil(int mode, int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell,
                    int lg, const T *x, const TB *b, TO *y, hipStream_t st) {
  dim3 grid(grid_cells(maxcell, lg), nparts);
  if (fine) {
    if (maxent <= 7)
      stencil_mode<T, TB, TO, 1, 7>(mode, grid, desc, lg, x, b, y, st);
    else if (maxent <= 15)
      stencil_mode<T, TB, TO, 1, 15>(mode, grid, desc, lg, x, b, y, st);
    else
      stencil_mode<T, TB, TO, 1, 27>(mode, grid, desc, lg, x, b, y, st);
  } else {
    if (maxent <= 7)
      stencil_mode<T, TB, TO, 0, 7>(mode, grid, desc, lg, x, b, y, st);
    else if (maxent <= 15)
      stencil_mode<T, TB, TO, 0, 15>(mode, grid, desc, lg, x, b, y, st);
    else
      stencil_mode<T, TB, TO, 0, 27>(mode, grid, desc, lg, x, b, y, st);
  }
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

template <typename T, typename TB>
void launch_smooth_resid(int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell, int lg,
                         const TB *b, T *x, T *r, hipStream_t st) {
  dim3 grid(grid_cells(maxcell, lg), nparts);
#define SSAMG_SR(F, N) k_smooth_resid<T, TB, F, N><<<grid, kBlock, 0, st>>>(desc, lg, b, x, r)
  if (fine) {
    if (maxent <= 7) SSAMG_SR(1, 7);
    else if (maxent <= 15) SSAMG_SR(1, 15);
    else SSAMG_SR(1, 27);
  } else {
    if (maxent <= 7) SSAMG_SR(0, 7);
    else if (maxent <= 15) SSAMG_SR(0, 15);
    else SSAMG_SR(0, 27);
  }
#undef SSAMG_SR
}

template <typename T>
void launch_tail(const TailLevel<T> *tl, int nl, int lg, hipStream_t st) {
  k_tail<T><<<1, kTailThreads, 0, st>>>(tl, nl, lg);
}

template void launch_stencil<double, double, double>(int, int, int, const PartDesc<double> *, int, int,
                                                     int, const double *, const double *, double *,
                                                     hipStream_t);
template void launch_stencil<float, float, float>(int, int, int, const PartDesc<float> *, int, int, int,
                                                  const float *, const float *, float *, hipStream_t);
template void launch_stencil<float, double, float>(int, int, int, const PartDesc<float> *, int, int, int,
                                                   const float *, const double *, float *, hipStream_t);
template void launch_stencil<float, double, double>(int, int, int, const PartDesc<float> *, int, int, int,
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
template void launch_smooth_resid<double, double>(int, int, const PartDesc<double> *, int, int, int,
                                                  const double *, double *, double *, hipStream_t);
template void launch_smooth_resid<float, float>(int, int, const PartDesc<float> *, int, int, int,
                                                const float *, float *, float *, hipStream_t);
template void launch_smooth_resid<float, double>(int, int, const PartDesc<float> *, int, int, int,
                                                 const double *, float *, float *, hipStream_t);
template void launch_tail<double>(const TailLevel<double> *, int, int, hipStream_t);
template void launch_tail<float>(const TailLevel<float> *, int, int, hipStream_t);

}  // namespace ssamg
