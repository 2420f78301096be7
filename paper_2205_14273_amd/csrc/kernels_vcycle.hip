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
#include <hip/hip_ext.h>

#include <cstddef>
#include <type_traits>

#include "device_util.h"
#include "ssamg_impl.h"

namespace ssamg {

namespace {

using dev::cell_ijk;
using dev::chunk_index;
using dev::chunk_index_tiled;
using dev::G;
using dev::gload;
using dev::nb_mask;
using dev::nb_ok;


// smoother factor of cell c: omega_p / a_ii (Jacobi) or factor / sum|a_ij| (L1)
template <typename T>
__device__ __forceinline__ T smooth_factor(const PartDesc<T> &d, long long c) {
  return d.rs ? G(d.rs)[c] : d.omega / G(d.coef)[(long long)d.center * d.ncell + c];
}

// sum_s a_s(c) x(c + s) over the part's stencil; all loads are issued before
// the first multiply (entries s >= nent are masked off).
// MIR: coefficients read through the mirror tables (PartDesc::mir).
// LAT (launches on small levels, bound by latency): every load unconditional
// (an absent entry reads entry 0, an absent neighbour the cell itself; the
// value is zeroed afterwards), so that no load and no read of the descriptor's
// offset tables sits behind a branch, where each would wait for the one
// before.  Large levels keep the guarded loads: the unconditional form needs
// about 30 more registers, which costs occupancy and bandwidth there.
template <typename T, int NENT, bool MIR = false, bool LAT = false>
__device__ __forceinline__ T stencil_acc(const PartDesc<T> &d, int c, int lg, const T *xp) {
  int i, j, k;
  cell_ijk(c, d.n[0], d.n[1], i, j, k);
  const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const auto cf = G(d.coef) + c;
  const auto cfb = G(d.coef);
  int co = c;   // LAT: offset of entry s
  T a[NENT], xv[NENT];
#pragma unroll
  for (int s = 0; s < NENT; ++s) {
    const bool act = s < d.nent;
    if constexpr (MIR) {
      const bool ok = act && nb_ok(mx, my, mz, d.code[s]);
      a[s] = act ? cf[(long long)d.mir[s] * d.ncell + (ok ? d.mlin[s] : 0)] : T(0);
      xv[s] = ok ? xp[(long long)d.lin[s] << lg] : T(0);
    } else if constexpr (LAT) {
      // 32-bit coefficient offsets stepped in a vector register, one packed
      // scalar per entry, and absent values zeroed by a 0/1 factor rather than
      // a select (27 lane masks would not fit the scalar registers): all loads
      // stay in flight together.  Exact for finite values.
      const int w = d.lc[s];
      const bool ok = nb_ok(mx, my, mz, w & 63) & act;   // no short circuit: no branch
      const T av = cfb[(unsigned)(act ? co : c)];
      const T xq = xp[(long long)dev::opaque(ok ? (w >> 6) : 0) << lg];
      a[s] = av * (act ? T(1) : T(0));
      xv[s] = xq * (T)dev::opaque((int)ok);
      co = dev::opaque(co + (int)d.ncell);
    } else {
      a[s] = act ? cf[(long long)s * d.ncell] : T(0);
      xv[s] = (act && nb_ok(mx, my, mz, d.code[s])) ? xp[(long long)d.lin[s] << lg] : T(0);
    }
  }
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < NENT; ++s) acc = fma(a[s], xv[s], acc);
  return acc;
}

// sum_s a_s(c) w(c + s) b(c + s): the stencil part of A x at cell c for the
// iterate x = w b of a first sweep from zero (bp points at b of cell c)
template <typename T, typename TB, int NENT, bool LAT = false>
__device__ __forceinline__ T stencil_wb(const PartDesc<T> &d, int c, int lg, const TB *bp) {
  int i, j, k;
  cell_ijk(c, d.n[0], d.n[1], i, j, k);
  const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const auto cf = G(d.coef) + c;
  const auto cfb = G(d.coef);
  int co = c;   // LAT: offset of entry s
  const auto wp = G(d.rs) + c;
  T a[NENT], bv[NENT], wv[NENT];
#pragma unroll
  for (int s = 0; s < NENT; ++s) {   // LAT: unconditional loads, as in stencil_acc
    const bool act = s < d.nent;
    if constexpr (LAT) {   // as in stencil_acc
      const int w = d.lc[s];
      const bool ok = nb_ok(mx, my, mz, w & 63) & act;
      const T av = cfb[(unsigned)(act ? co : c)];
      const int ls = dev::opaque(ok ? (w >> 6) : 0);
      const T bq = (T)bp[(long long)ls << lg];
      const T wq = wp[ls];
      a[s] = av * (act ? T(1) : T(0));
      bv[s] = bq;
      wv[s] = wq * (T)dev::opaque((int)ok);
      co = dev::opaque(co + (int)d.ncell);
    } else {
      const bool ok = act && nb_ok(mx, my, mz, d.code[s]);
      a[s] = act ? cf[(long long)s * d.ncell] : T(0);
      bv[s] = ok ? (T)bp[(long long)d.lin[s] << lg] : T(0);
      wv[s] = ok ? wp[d.lin[s]] : T(0);
    }
  }
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < NENT; ++s) acc = fma(a[s], wv[s] * bv[s], acc);
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

// coupling products staged in LDS per pass: large levels (short rows, and full
// occupancy matters for bandwidth) and small levels (rows up to ~100 entries
// across mismatched part interfaces; few blocks, so fewer passes matter)
constexpr int kUChunkBig = 1024;
constexpr int kUChunkSmall = 4096;
constexpr long long kBigLevel = 1 << 18;   // elements (cells x rhs) from which a level counts as large

// acc + prod[q0] + ... + prod[q1 - 1] (slot kr of each entry), added in entry
// order; the LDS reads are issued eight at a time so that long rows do not
// wait on one read per entry
template <typename T>
__device__ __forceinline__ T row_sum(const T *__restrict__ prod, int q0, int q1, int lg, int kr, T acc) {
  for (int q = q0; q < q1; q += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = q + u < q1 ? prod[((q + u) << lg) | kr] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q + u < q1) acc += v[u];
  }
  return acc;
}

// The U part of A x for every (cell, rhs) slot of one block: sum over the
// entries of the slot's row of val * xs(col, rhs).  The rows of a block and
// their entries are contiguous (rows sorted by cell), so all threads form the
// products of a strided share of the entries (coalesced loads, every gather in
// flight at once), stage them in LDS, and one thread per (row, rhs) adds its
// row's products in entry order (deterministic).  Long rows, which coarse
// levels build across mismatched part interfaces, thus cost no serial chain of
// loads.  Must be called by every thread of the block.
template <int UCH, typename T, typename XS, typename XW = std::nullptr_t>
__device__ __forceinline__ T block_coupling(const PartDesc<T> &d, int chunk, int lg, XS xs,
                                            T *__restrict__ prod, T *__restrict__ rsum,
                                            XW xw = nullptr) {
  // xw (optional): a second factor of the column's value, xw(col, k) * xs(col, k),
  // gathered separately so that no multiply waits between the gathers
  constexpr bool WB = !std::is_same<XW, std::nullptr_t>::value;
  const auto ub = G(d.ublk[lg]) + 2 * chunk;
  const int u0 = ub[0], e0 = ub[1], u1 = ub[2], e1 = ub[3];
  if (u0 == u1) return T(0);                          // block-uniform
  const int tid = threadIdx.x;
  const int mask = (1 << lg) - 1;
  const int cell0 = (int)d.off + chunk * (kBlock >> lg);
  const int nrt = (u1 - u0) << lg;                    // (row, rhs) slots of the block
  int rq0 = 0, rq1 = 0, rslot = 0;
  if (tid < nrt) {
    const int r = u0 + (tid >> lg);
    rq0 = G(d.uptr)[r];
    rq1 = G(d.uptr)[r + 1];
    rslot = ((G(d.urow)[r] - cell0) << lg) | (tid & mask);
  }
  rsum[tid] = T(0);
  T racc = T(0);
  const int per = UCH >> lg;                      // entries per pass
  for (int ec = e0; ec < e1; ec += per) {
    const int np = min(per, e1 - ec) << lg;
    int cc[UCH / kBlock];
    T vv[UCH / kBlock], xx[UCH / kBlock], ww[UCH / kBlock];
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      // unconditional loads (a slot past the chunk reads its first entry and is
      // masked below), so that every entry load of the chunk is in flight at once
      const int qe = ec + (q < np ? (q >> lg) : 0);
      cc[t] = gload(d.ucol + qe);
      vv[t] = gload(d.uval + qe);
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      // gathers behind a block-uniform test only (a slot past the chunk
      // gathers its first entry's column and is masked below)
      xx[t] = ww[t] = T(0);
      if (t * kBlock < np) {
        const int k = (tid + t * kBlock) & mask;
        xx[t] = xs(cc[t], k);
        if constexpr (WB) ww[t] = xw(cc[t], k);
      }
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      if (q < np) prod[q] = vv[t] * (WB ? ww[t] * xx[t] : xx[t]);
    }
    __syncthreads();
    if (tid < nrt) {
      const int qa = max(rq0, ec), qb = min(rq1, ec + (np >> lg));
      racc = row_sum(prod, qa - ec, qb - ec, lg, tid & mask, racc);
    }
    __syncthreads();
  }
  if (tid < nrt) rsum[rslot] = racc;
  __syncthreads();
  return rsum[tid];
}

// The block's coupling range, its rows' entry ranges and output slots, and the
// first kUPre entry loads of every thread, issued before the stencil in the
// small-level sweeps so that their chain of loads runs beside the stencil's
// (block_coupling waits on each link after the stencil has finished).
constexpr int kUPre = 4;
template <typename T>
struct UPre {
  int u0, e0, u1, e1, rq0, rq1, rslot;
  int cc[kUPre];
  T vv[kUPre];
};

template <typename T>
__device__ __forceinline__ void upre_load(const PartDesc<T> &d, int chunk, int lg, UPre<T> &u) {
  const auto ub = G(d.ublk[lg]) + 2 * chunk;
  u.u0 = ub[0];
  u.e0 = ub[1];
  u.u1 = ub[2];
  u.e1 = ub[3];
  u.rq0 = u.rq1 = u.rslot = 0;
  if (u.u0 == u.u1) return;   // block-uniform
  const int tid = threadIdx.x, mask = (1 << lg) - 1;
  const int cell0 = (int)d.off + chunk * (kBlock >> lg);
  // clamped, unconditional loads (slots and entries past the block's are masked later)
  const int r = u.u0 + min(tid >> lg, u.u1 - u.u0 - 1);
  u.rq0 = G(d.uptr)[r];
  u.rq1 = G(d.uptr)[r + 1];
  u.rslot = ((G(d.urow)[r] - cell0) << lg) | (tid & mask);
#pragma unroll
  for (int t = 0; t < kUPre; ++t) {
    const int qe = u.e0 + min((tid + t * kBlock) >> lg, u.e1 - u.e0 - 1);
    u.cc[t] = gload(d.ucol + qe);
    u.vv[t] = gload(d.uval + qe);
  }
}

// block_coupling from the prefetched state (the same sums, in the same order)
template <int UCH, typename T, typename XS, typename XW = std::nullptr_t>
__device__ __forceinline__ T upre_apply(const PartDesc<T> &d, int lg, const UPre<T> &u, XS xs,
                                        T *__restrict__ prod, T *__restrict__ rsum, XW xw = nullptr) {
  constexpr bool WB = !std::is_same<XW, std::nullptr_t>::value;
  static_assert(UCH / kBlock >= kUPre, "prefetch within the first pass");
  if (u.u0 == u.u1) return T(0);                      // block-uniform
  const int tid = threadIdx.x;
  const int mask = (1 << lg) - 1;
  const int nrt = (u.u1 - u.u0) << lg;
  rsum[tid] = T(0);
  T racc = T(0);
  const int per = UCH >> lg;
  for (int ec = u.e0; ec < u.e1; ec += per) {
    const int np = min(per, u.e1 - ec) << lg;
    int cc[UCH / kBlock];
    T vv[UCH / kBlock], xx[UCH / kBlock], ww[UCH / kBlock];
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      if (t < kUPre && ec == u.e0) {   // block-uniform: the prefetched entries
        cc[t] = u.cc[t];
        vv[t] = u.vv[t];
      } else {
        const int qe = ec + (q < np ? (q >> lg) : 0);
        cc[t] = gload(d.ucol + qe);
        vv[t] = gload(d.uval + qe);
      }
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      xx[t] = ww[t] = T(0);
      if (t * kBlock < np) {
        const int k = (tid + t * kBlock) & mask;
        xx[t] = xs(cc[t], k);
        if constexpr (WB) ww[t] = xw(cc[t], k);
      }
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      if (q < np) prod[q] = vv[t] * (WB ? ww[t] * xx[t] : xx[t]);
    }
    __syncthreads();
    if (tid < nrt) {
      const int qa = max(u.rq0, ec), qb = min(u.rq1, ec + (np >> lg));
      racc = row_sum(prod, qa - ec, qb - ec, lg, tid & mask, racc);
    }
    __syncthreads();
  }
  if (tid < nrt) rsum[u.rslot] = racc;
  __syncthreads();
  return rsum[tid];
}

// b_c = P^T r for coarse cell cc: r(2I) + wp(2I-1) r(2I-1) + wm(2I+1) r(2I+1)
template <typename T>
__device__ __forceinline__ void restrict_one(const PartDesc<T> &d, int cc, int kr, int lg,
                                             const T *__restrict__ r, T *__restrict__ bc,
                                             const T *__restrict__ wn = nullptr, T *__restrict__ xn = nullptr) {
  const long long oc = ((d.coff + cc) << lg) + kr;
  if (d.dstar < 0) {
    const T v = r[((d.off + cc) << lg) + kr];
    bc[oc] = v;
    if (xn) xn[oc] = wn[d.coff + cc] * v;
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
    v = fma(G(d.wp)[fl], rp[-((long long)stride << lg)], v);
  }
  if (fi[ds] + 1 <= d.n[ds] - 1) {
    g[ds] = ci[ds];
    const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
    v = fma(G(d.wm)[fl], rp[(long long)stride << lg], v);
  }
  bc[oc] = v;
  // the next level's first sweep from zero, x = w b (k_smooth_zero's arithmetic)
  if (xn) xn[oc] = wn[d.coff + cc] * v;
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
  T v = G(d.wm)[fl] * xc[((d.coff + cm) << lg) + kr];
  if (id + 1 <= d.n[ds] - 1) {
    const int cstride = ds == 0 ? 1 : (ds == 1 ? d.cn[0] : d.cn[0] * d.cn[1]);
    v = fma(G(d.wp)[fl], xc[((d.coff + cm + cstride) << lg) + kr], v);
  }
  x[o] += v;
}

// Sum of v over the block's cells for each right-hand side (fixed tree over
// the 256 threads, strides multiples of 1 << lg), written to out[0 .. 1 << lg).
// Must be called by every thread of the block; sh: kBlock doubles of LDS.
__device__ __forceinline__ void block_dot(double *sh, double v, int lg, double *out) {
  const int nr = 1 << lg;
  __syncthreads();
  sh[threadIdx.x] = v;
  for (int s = kBlock / 2; s >= nr; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) out[threadIdx.x] = sh[threadIdx.x];
}

// y = S x + U x (APPLY), r = b - A x (RESID) or x' = x + w (b - A x) (JACOBI,
// w the smoother factor) over every cell of every part.  T: coefficients and
// x; TB: b; TO: output.  NENT bounds the entries of the level's stencils.
// BIG marks launches on large levels (the finest level always; there, in a
// mixed-precision cycle, they read the FP64 residual and write the FP64
// correction directly); it sets the LDS chunk of the coupling products.
template <typename T, int MODE, typename TB, typename TO, int BIG, int NENT, bool MIR = false>
__global__ __launch_bounds__(kBlock) void k_stencil(const PartDesc<T> *__restrict__ desc, int lg,
                                                    const T *__restrict__ x,
                                                    const TB *__restrict__ b, TO *__restrict__ y,
                                                    double *__restrict__ dotp, const double *__restrict__ aux) {
  constexpr int UCH = BIG ? kUChunkBig : kUChunkSmall;
  constexpr bool DOT = MODE == MODE_APPLY_DOT || MODE == MODE_JACOBI_DOT;
  __shared__ T prod[UCH];
  __shared__ T rsum[kBlock];
  const PartDesc<T> &d = desc[blockIdx.y];
  const int chunk = chunk_index();
  const long long e = (long long)chunk * kBlock + threadIdx.x;
  const long long nel = d.ncell << lg;
  // DOT modes: this block's partial slot (blocks past the grid's last one up
  // to the rounded slot count are covered by the last block, with zeros); the
  // second set (z.q of MODE_JACOBI_DOT, when aux is given) follows the first
  const long long slots = 4LL * ((gridDim.x + 3) / 4);
  double *dslot = DOT ? dotp + (((long long)blockIdx.y * slots + chunk) << lg) : nullptr;
  const long long dset = ((long long)gridDim.y * slots) << lg;
  const int nset = MODE == MODE_JACOBI_DOT && aux ? 2 : 1;
  if (DOT && chunk == (int)gridDim.x - 1 && (int)threadIdx.x < ((int)(slots - gridDim.x) << lg))
    for (int t = 0; t < nset; ++t) dslot[t * dset + (1 << lg) + threadIdx.x] = 0.0;
  if ((long long)chunk * kBlock >= nel) {            // whole block past the part's end
    if (DOT && (int)threadIdx.x < (1 << lg))
      for (int t = 0; t < nset; ++t) dslot[t * dset + threadIdx.x] = 0.0;
    return;
  }
  const bool valid = e < nel;
  const int c = valid ? (int)(e >> lg) : 0;
  const int kr = (int)(e & ((1 << lg) - 1));
  const long long o = ((d.off + c) << lg) + kr;
  const T *xp = x + o;
  T acc;
  TB bo = TB(0);
  T wo = T(0);
  if constexpr (!BIG && (MODE == MODE_RESID || MODE == MODE_JACOBI)) {
    // small levels: every load the sweep needs is requested before the
    // stencil is summed (the coupling chain, b and the factor included)
    UPre<T> u;
    upre_load(d, chunk, lg, u);
    bo = b[o];
    if (MODE == MODE_JACOBI) wo = smooth_factor(d, c);
    acc = stencil_acc<T, NENT, MIR, true>(d, c, lg, xp);
    if (!valid) acc = T(0);
    acc += upre_apply<UCH>(
        d, lg, u, [&](int col, int k) { return x[((long long)col << lg) + k]; }, prod, rsum);
  } else {
    acc = valid ? stencil_acc<T, NENT, MIR, !BIG>(d, c, lg, xp) : T(0);
    acc += block_coupling<UCH>(
        d, chunk, lg, [&](int col, int k) { return x[((long long)col << lg) + k]; }, prod, rsum);
    if (valid && (MODE == MODE_RESID || MODE == MODE_JACOBI)) {
      bo = b[o];
      if (MODE == MODE_JACOBI) wo = smooth_factor(d, c);
    }
  }
  if constexpr (MODE == MODE_APPLY_DOT) {
    if (valid) y[o] = (TO)acc;
    block_dot((double *)rsum, valid ? (double)xp[0] * (double)acc : 0.0, lg, dslot);
    return;
  }
  if constexpr (MODE == MODE_JACOBI_DOT) {
    // z = x + w (b - A x) with b = r, and the partial sums of r.z and z.q
    __shared__ double dsh[kBlock];
    double v = 0.0, w = 0.0;
    if (valid) {
      const TO z = (TO)(xp[0] + smooth_factor(d, c) * ((T)b[o] - acc));
      y[o] = z;
      v = (double)b[o] * (double)z;
      if (aux) w = (double)z * aux[o];
    }
    block_dot(dsh, v, lg, dslot);
    if (aux) block_dot(dsh, w, lg, dslot + dset);
    return;
  }
  if (!valid) return;
  if (MODE == MODE_APPLY) {
    y[o] = (TO)acc;
  } else if (MODE == MODE_RESID) {
    y[o] = (TO)((T)bo - acc);
  } else {
    y[o] = (TO)(xp[0] + wo * ((T)bo - acc));
  }
}

// The first sweep of eq:relax0 from a zero guess, x = w b, fused with the
// residual r = b - A x: the iterate at a neighbour is formed there from its
// own factor and right-hand side, so x and b are each read once.
template <typename T, typename TB, int BIG, int NENT>
__global__ __launch_bounds__(kBlock) void k_smooth_resid(const PartDesc<T> *__restrict__ desc, int lg,
                                                         const TB *__restrict__ b,
                                                         T *__restrict__ x, T *__restrict__ r) {
  constexpr int UCH = BIG ? kUChunkBig : kUChunkSmall;
  __shared__ T prod[UCH];
  __shared__ T rsum[kBlock];
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
  const auto wp = G(d.rs) + c;
  const auto wl = G(d.rs) - d.off;   // factors of the whole level
  T acc, b0, w0;
  if constexpr (!BIG) {   // small levels: all loads requested before the stencil is summed
    UPre<T> u;
    upre_load(d, chunk, lg, u);
    b0 = (T)bp[0];
    w0 = wp[0];
    acc = stencil_wb<T, TB, NENT, true>(d, c, lg, bp);
    if (!valid) acc = T(0);
    acc += upre_apply<UCH>(
        d, lg, u, [&](int col, int k) { return (T)b[((long long)col << lg) + k]; }, prod, rsum,
        [&](int col, int) { return wl[col]; });
  } else {
    acc = valid ? stencil_wb<T, TB, NENT, false>(d, c, lg, bp) : T(0);
    acc += block_coupling<UCH>(
        d, chunk, lg, [&](int col, int k) { return (T)b[((long long)col << lg) + k]; }, prod, rsum,
        [&](int col, int) { return wl[col]; });
    if (!valid) return;
    b0 = (T)bp[0];
    w0 = wp[0];
  }
  if (!valid) return;
  x[o] = w0 * b0;
  r[o] = b0 - acc;
}

// ---------------------------------------------------------------------------
// Batched solves (4 or more right-hand sides): each thread takes four
// consecutive columns of one cell.  The per-cell work (coordinates, masks,
// coefficient loads, addresses) is then shared by four columns, the vector
// loads and stores are 16 or 32 bytes, and a 256-thread block covers
// 1024 >> lg cells (the coupling-row table of lg - 2).  Every value is formed
// with the same operations in the same order as in the one-column kernels.

__device__ __forceinline__ void load4(const float *p, float v[4]) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}
__device__ __forceinline__ void load4(const double *p, double v[4]) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
__device__ __forceinline__ void store4(float *p, const float v[4]) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store4(double *p, const double v[4]) {
  reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}

// stencil_acc for the four columns at xp (x of the cell's first column).  Every
// load is issued unconditionally (an absent entry reads entry 0, an absent
// neighbour the cell itself) and the value is zeroed afterwards, so all loads
// of the stencil are in flight together.
template <typename T, int NENT, bool MIR = false>
__device__ __forceinline__ void stencil_acc4(const PartDesc<T> &d, int c, int lg, const T *xp, T acc[4]) {
  int i, j, k;
  cell_ijk(c, d.n[0], d.n[1], i, j, k);
  const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const T *cf = d.coef + c;
  T a[NENT], xv[NENT][4];
  bool act[NENT], ok[NENT];
#pragma unroll
  for (int s = 0; s < NENT; ++s) {
    act[s] = s < d.nent;
    ok[s] = act[s] && nb_ok(mx, my, mz, d.code[s]);
    if constexpr (MIR)
      a[s] = gload(cf + (act[s] ? (long long)d.mir[s] * d.ncell + (ok[s] ? d.mlin[s] : 0) : 0LL));
    else
      a[s] = gload(cf + (act[s] ? (long long)s * d.ncell : 0LL));
    load4(xp + (ok[s] ? ((long long)d.lin[s] << lg) : 0LL), xv[s]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc[q] = T(0);
#pragma unroll
    for (int s = 0; s < NENT; ++s)
      acc[q] = fma(act[s] ? a[s] : T(0), ok[s] ? xv[s][q] : T(0), acc[q]);
  }
}

// block_coupling for blocks of 1024 >> lg cells: up to four (row, column)
// slots per thread; out[q] receives the sum of the thread's column 4t + q
template <int UCH, typename T, typename XS>
__device__ __forceinline__ void block_coupling4(const PartDesc<T> &d, int chunk, int lg, XS xs,
                                                T *__restrict__ prod, T *__restrict__ rsum, T out[4]) {
  const int lgc = lg - 2;
  const int *ub = d.ublk[lgc] + 2 * chunk;
  const int u0 = gload(ub), e0 = gload(ub + 1), u1 = gload(ub + 2), e1 = gload(ub + 3);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = T(0);
  if (u0 == u1) return;                               // block-uniform
  const int tid = threadIdx.x;
  const int mask = (1 << lg) - 1;
  const int cell0 = (int)d.off + chunk * (kBlock >> lgc);
  const int nrt = (u1 - u0) << lg;                    // (row, column) slots, <= 4 kBlock
  int rq0[4], rq1[4], rslot[4];
  T racc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = tid + q * kBlock;
    rq0[q] = rq1[q] = rslot[q] = 0;
    racc[q] = T(0);
    if (t < nrt) {
      const int r = u0 + (t >> lg);
      rq0[q] = gload(d.uptr + r);
      rq1[q] = gload(d.uptr + r + 1);
      rslot[q] = ((gload(d.urow + r) - cell0) << lg) | (t & mask);
    }
    rsum[t] = T(0);
  }
  const int per = UCH >> lg;
  for (int ec = e0; ec < e1; ec += per) {
    const int np = min(per, e1 - ec) << lg;
    int cc[UCH / kBlock];
    T vv[UCH / kBlock], xx[UCH / kBlock];
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      // unconditional loads (a slot past the chunk reads its first entry and is
      // masked below), so that every entry load of the chunk is in flight at once
      const int qe = ec + (q < np ? (q >> lg) : 0);
      cc[t] = gload(d.ucol + qe);
      vv[t] = gload(d.uval + qe);
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      xx[t] = q < np ? xs(cc[t], q & mask) : T(0);
    }
#pragma unroll
    for (int t = 0; t < UCH / kBlock; ++t) {
      const int q = tid + t * kBlock;
      if (q < np) prod[q] = vv[t] * xx[t];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = tid + q * kBlock;
      if (t < nrt) {
        const int qa = max(rq0[q], ec), qb = min(rq1[q], ec + (np >> lg));
        racc[q] = row_sum(prod, qa - ec, qb - ec, lg, t & mask, racc[q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (tid + q * kBlock < nrt) rsum[rslot[q]] = racc[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = rsum[(tid << 2) + q];
}

// block_dot for a four-column block: its 1024 elements are the four 256-element
// blocks of the one-column launch, each reduced with block_dot's tree and the
// four sums then added in order, ((s0 + s1) + s2) + s3, as the final pass adds
// the one-column launch's four slots of a group; so both layouts give the same
// group sums.  sh: 4 kBlock doubles; out: the group slot.
__device__ __forceinline__ void block_dot4(double *sh, const double v[4], int lg, double *out) {
  const int nr = 1 << lg;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) sh[4 * threadIdx.x + q] = v[q];
  for (int s = kBlock / 2; s >= nr; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int j = 0; j < 4; ++j) sh[j * kBlock + threadIdx.x] += sh[j * kBlock + threadIdx.x + s];
  }
  __syncthreads();
  if ((int)threadIdx.x < nr)
    out[threadIdx.x] = ((sh[threadIdx.x] + sh[kBlock + threadIdx.x]) + sh[2 * kBlock + threadIdx.x]) +
                       sh[3 * kBlock + threadIdx.x];
}

template <typename T, int MODE, typename TB, typename TO, int BIG, int NENT, bool MIR = false>
__global__ __launch_bounds__(kBlock) void k_stencil4(const PartDesc<T> *__restrict__ desc, int lg,
                                                     const T *__restrict__ x,
                                                     const TB *__restrict__ b, TO *__restrict__ y,
                                                     double *__restrict__ dotp, const double *__restrict__ aux) {
  constexpr int UCH = BIG ? kUChunkBig : kUChunkSmall;
  constexpr bool DOT = MODE == MODE_APPLY_DOT || MODE == MODE_JACOBI_DOT;
  __shared__ T prod[UCH];
  __shared__ T rsum[4 * kBlock];
  const PartDesc<T> &d = desc[blockIdx.y];
  const int chunk = chunk_index_tiled(d.tbp[lg], d.tsb[lg]);
  const int lgc = lg - 2;
  const long long e = (long long)chunk * kBlock + threadIdx.x;
  const long long nel = d.ncell << lgc;
  // DOT modes: the group slot of the four one-column slots this block covers
  // (second set after gridDim.y * gridDim.x groups)
  double *dslot = DOT ? dotp + (((long long)blockIdx.y * gridDim.x + chunk) << lg) : nullptr;
  const long long dset = ((long long)gridDim.y * gridDim.x) << lg;
  const int nset = MODE == MODE_JACOBI_DOT && aux ? 2 : 1;
  if ((long long)chunk * kBlock >= nel) {            // whole block past the part's end
    if (DOT && (int)threadIdx.x < (1 << lg))
      for (int t = 0; t < nset; ++t) dslot[t * dset + threadIdx.x] = 0.0;
    return;
  }
  const bool valid = e < nel;
  const int c = valid ? (int)(e >> lgc) : 0;
  const long long o = ((d.off + c) << lg) + 4 * (e & ((1 << lgc) - 1));
  const T *xp = x + o;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  if (valid) stencil_acc4<T, NENT, MIR>(d, c, lg, xp, acc);
  T cu[4];
  block_coupling4<UCH>(
      d, chunk, lg, [&](int col, int k) { return x[((long long)col << lg) + k]; }, prod, rsum, cu);
  if constexpr (MODE == MODE_APPLY_DOT) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      T pv[4], out[4];
      load4(xp, pv);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        out[q] = acc[q] + cu[q];
        v[q] = (double)pv[q] * (double)out[q];
      }
      store4((T *)(y + o), out);
    }
    block_dot4((double *)rsum, v, lg, dslot);
    return;
  }
  if constexpr (MODE == MODE_JACOBI_DOT) {
    // z = x + w (b - A x) with b = r, and the partial sums of r.z and z.q
    __shared__ double dsh[4 * kBlock];
    double v[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      TB bv[4];
      T xv[4];
      TO out[4];
      load4(b + o, bv);
      load4(xp, xv);
      const T wf = smooth_factor(d, c);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T a = acc[q] + cu[q];
        out[q] = (TO)(xv[q] + wf * ((T)bv[q] - a));
        v[q] = (double)bv[q] * (double)out[q];
      }
      store4(y + o, out);
      if (aux) {
        double qv[4];
        load4(aux + o, qv);
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (double)out[q] * qv[q];
      }
    }
    block_dot4(dsh, v, lg, dslot);
    if (aux) block_dot4(dsh, w, lg, dslot + dset);
    return;
  }
  if (!valid) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] += cu[q];
  TO out[4];
  if (MODE == MODE_APPLY) {
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = (TO)acc[q];
  } else {
    TB bv[4];
    load4(b + o, bv);
    if (MODE == MODE_RESID) {
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = (TO)((T)bv[q] - acc[q]);
    } else {
      T xv[4];
      load4(xp, xv);
      const T w = smooth_factor(d, c);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = (TO)(xv[q] + w * ((T)bv[q] - acc[q]));
    }
  }
  store4(y + o, out);
}

// x = w b for four columns per thread
template <typename T, typename TB>
__global__ __launch_bounds__(kBlock) void k_smooth_zero4(const PartDesc<T> *__restrict__ desc, int lg,
                                                         const TB *__restrict__ b, T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const int lgc = lg - 2;
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lgc)) return;
  const int c = (int)(e >> lgc);
  const long long o = ((d.off + c) << lg) + 4 * (e & ((1 << lgc) - 1));
  TB bv[4];
  load4(b + o, bv);
  const T w = smooth_factor(d, c);
  T xv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) xv[q] = w * (T)bv[q];
  store4(x + o, xv);
}

// restrict_one for four columns per thread
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict4(const PartDesc<T> *__restrict__ desc, int lg,
                                                      const T *__restrict__ r, T *__restrict__ bc) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const int lgc = lg - 2;
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.cncell << lgc)) return;
  const int cc = (int)(e >> lgc);
  const int k4 = 4 * (int)(e & ((1 << lgc) - 1));
  T v[4];
  if (d.dstar < 0) {
    load4(r + ((d.off + cc) << lg) + k4, v);
    store4(bc + ((d.coff + cc) << lg) + k4, v);
    return;
  }
  int ci[3];
  cell_ijk(cc, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  const int ds = d.dstar;
  int fi[3] = {ci[0], ci[1], ci[2]};
  fi[ds] = 2 * ci[ds];
  const int f0 = fi[0] + d.n[0] * (fi[1] + d.n[1] * fi[2]);
  const int stride = ds == 0 ? 1 : (ds == 1 ? d.n[0] : d.n[0] * d.n[1]);
  const T *rp = r + ((d.off + f0) << lg) + k4;
  load4(rp, v);
  int g[3] = {ci[0], ci[1], ci[2]};
  if (fi[ds] - 1 >= 0) {
    g[ds] = ci[ds] - 1;
    const T w = G(d.wp)[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])];
    T t[4];
    load4(rp - ((long long)stride << lg), t);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = fma(w, t[q], v[q]);
  }
  if (fi[ds] + 1 <= d.n[ds] - 1) {
    g[ds] = ci[ds];
    const T w = G(d.wm)[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])];
    T t[4];
    load4(rp + ((long long)stride << lg), t);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = fma(w, t[q], v[q]);
  }
  store4(bc + ((d.coff + cc) << lg) + k4, v);
}

// interp_one for four columns per thread
template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp_add4(const PartDesc<T> *__restrict__ desc, int lg,
                                                        const T *__restrict__ xc, T *__restrict__ x) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const int lgc = lg - 2;
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.ncell << lgc)) return;
  const int c = (int)(e >> lgc);
  const int k4 = 4 * (int)(e & ((1 << lgc) - 1));
  T *xp = x + ((d.off + c) << lg) + k4;
  T xv[4], v[4];
  load4(xp, xv);
  if (d.dstar < 0) {
    load4(xc + ((d.coff + c) << lg) + k4, v);
  } else {
    int f[3];
    cell_ijk(c, d.n[0], d.n[1], f[0], f[1], f[2]);
    const int ds = d.dstar;
    const int id = f[ds];
    int g[3] = {f[0], f[1], f[2]};
    if ((id & 1) == 0) {
      g[ds] = id >> 1;
      load4(xc + ((d.coff + g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2])) << lg) + k4, v);
    } else {
      g[ds] = (id - 1) >> 1;
      const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
      const int cm = g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2]);
      T t[4];
      load4(xc + ((d.coff + cm) << lg) + k4, t);
      const T wm = G(d.wm)[fl];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = wm * t[q];
      if (id + 1 <= d.n[ds] - 1) {
        const int cstride = ds == 0 ? 1 : (ds == 1 ? d.cn[0] : d.cn[0] * d.cn[1]);
        load4(xc + ((d.coff + cm + cstride) << lg) + k4, t);
        const T wp = G(d.wp)[fl];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = fma(wp, t[q], v[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) xv[q] += v[q];
  store4(xp, xv);
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

// wn, xn: also the next level's first sweep from zero, xn = wn b_c (wn: that
// level's smoother factors)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const PartDesc<T> *__restrict__ desc, int lg,
                                                     const T *__restrict__ r, T *__restrict__ bc,
                                                     const T *__restrict__ wn, T *__restrict__ xn) {
  const PartDesc<T> &d = desc[blockIdx.y];
  const long long e = (long long)chunk_index() * kBlock + threadIdx.x;
  if (e >= (d.cncell << lg)) return;
  restrict_one(d, (int)(e >> lg), (int)(e & ((1 << lg) - 1)), lg, r, bc, wn, xn);
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

// ------------------------------------------------------------ coarse end

// dst[w] = src(w) for w < n (32-bit words), up to eight loads per thread in
// flight (clamped indices, so that no load sits behind a branch)
template <int TT, typename F>
__device__ __forceinline__ void stage_words(int *__restrict__ dst, int n, F src) {
  for (int w0 = 0; w0 < n; w0 += 8 * TT) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src(min(w0 + u * TT + (int)threadIdx.x, n - 1));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int w = w0 + u * TT + (int)threadIdx.x;
      if (w < n) dst[w] = v[u];
    }
  }
}

// The U part of A x for every (row, rhs) slot of a level, x in LDS: all
// threads form the products of a strided share of up to prodcap entries per
// pass (loads of entries and of the thread's row ranges in flight together),
// stage them in LDS, and each slot adds its row's products in entry order,
// from zero, as block_coupling does.  fin(element, sum) then receives each
// slot's sum.  Rows x rhs <= kTailMax.  Ends with a workgroup barrier.
template <typename T, int TT, typename FIN>
__device__ void tail_u(const TailLevel<T> &v, int lg, const T *__restrict__ x, T *__restrict__ prod,
                       int prodcap, FIN fin) {
  if (v.nrow == 0) return;   // uniform
  constexpr int RPT = kTailMax / TT, EPT = kTailUPer;
  const int tid = threadIdx.x, mask = (1 << lg) - 1;
  const int nslot = v.nrow << lg, nnz = v.nnz;
  int qa[RPT], qb[RPT], slot[RPT];
  T racc[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int t = min(tid + j * TT, nslot - 1);
    const int r = t >> lg;
    qa[j] = gload(v.uptr + r);
    qb[j] = gload(v.uptr + r + 1);
    slot[j] = (gload(v.urow + r) << lg) | (t & mask);
    racc[j] = T(0);
  }
  const int per = prodcap >> lg;
  for (int ec = 0; ec < nnz; ec += per) {
    const int np = min(per, nnz - ec) << lg;
    int cc[EPT];
    T vv[EPT], xx[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
      const int q = tid + t * TT;
      const int qe = ec + (q < np ? (q >> lg) : 0);
      cc[t] = gload(v.ucol + qe);
      vv[t] = gload(v.uval + qe);
    }
#pragma unroll
    for (int t = 0; t < EPT; ++t) xx[t] = x[(cc[t] << lg) | ((tid + t * TT) & mask)];
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
      const int q = tid + t * TT;
      if (q < np) prod[q] = vv[t] * xx[t];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int a = max(qa[j], ec), b = min(qb[j], ec + (np >> lg));
      if (tid + j * TT < nslot && a < b) racc[j] = row_sum(prod, a - ec, b - ec, lg, (tid + j * TT) & mask, racc[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j)
    if (tid + j * TT < nslot) fin(slot[j], racc[j]);
  __syncthreads();
}

// sum_s ca[s][c] x(nb[s][c]) over the pack's stencil of element e (the order
// and operations of stencil_acc: absent entries add 0)
template <typename T>
__device__ __forceinline__ T tail_stencil(const TailLevel<T> &v, int e, int lg, const T *__restrict__ x) {
  const int c = e >> lg, k = e & ((1 << lg) - 1);
  const int n = (int)v.ncell, nw = v.nw;
  const auto nb = G(v.nb) + c;
  const auto ca = G(v.ca) + c;
  int id[kMaxEnt];
  T a[kMaxEnt], xv[kMaxEnt];
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) {   // entries past nw read entry 0 and add 0
    const int ss = s < nw ? s : 0;
    id[s] = nb[ss * n];
    a[s] = ca[ss * n];
  }
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) xv[s] = x[(id[s] << lg) | k];
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) acc = fma(s < nw ? a[s] : T(0), s < nw ? xv[s] : T(0), acc);
  return acc;
}

// The coarse end of one V(1,1) cycle, levels tl[0] .. tl[pl.nl - 1] (the last
// one the coarsest), in a single workgroup whose vectors live in LDS: from
// tl[0].vb (global) into tl[0].vt (global).  The same operations in the same
// order as the grid kernels, over all elements of a level at once, one phase
// at a time with a workgroup barrier between phases; the operands come from
// the levels' packs.  Every level above the coarsest holds at most kTailMax
// elements.  TT threads: 1024 in FP32, 512 in FP64.
// mcol (one workgroup per column, lg = 0): the right-hand side is the unit
// vector e_j (j = blockIdx.x) instead of tl[0].vb, and the result goes to
// column j of mcol (FP64) instead of tl[0].vt.
template <typename T, int TT>
__global__ __launch_bounds__(TT) void k_tail(const TailLevel<T> *__restrict__ tl, TailPlan pl, int lg,
                                             double *__restrict__ mcol) {
  extern __shared__ __align__(16) char sm[];
  const int tid = threadIdx.x, mask = (1 << lg) - 1;
  const int nl = pl.nl;
  const TailLevel<T> *L = reinterpret_cast<const TailLevel<T> *>(sm);
  int *voff = reinterpret_cast<int *>(sm + pl.off_tab);   // [nl]: b of level i at vec + voff[i]
  T *vec = reinterpret_cast<T *>(sm + pl.off_vec);
  T *tv = reinterpret_cast<T *>(sm + pl.off_tv), *acc = reinterpret_cast<T *>(sm + pl.off_acc);
  T *prod = reinterpret_cast<T *>(sm + pl.off_prod);
  stage_words<TT>(reinterpret_cast<int *>(sm), nl * (int)(sizeof(TailLevel<T>) / 4),
                  [&](int w) { return gload(reinterpret_cast<const int *>(tl) + w); });
  __syncthreads();
  if (tid < nl) {
    int o = 0;
    for (int i = 0; i < tid; ++i) o += 2 * (int)(L[i].ncell << lg);
    voff[tid] = o;
  }
  // b of the first level, and its first iterate x = w b (x follows b)
  const int n0 = (int)L[0].ncell;
  {
    const TailLevel<T> &v = L[0];
    const int nel = (int)(v.ncell << lg);
    const bool coarsest = nl == 1;
    for (int e = tid; e < nel; e += TT) {
      const T b = mcol ? (e == (int)blockIdx.x ? T(1) : T(0)) : gload(v.vb + e);
      vec[e] = b;
      if (!coarsest) vec[nel + e] = gload(v.rs + (e >> lg)) * b;
    }
  }
  // the result of the first level: tl[0].vt, or column blockIdx.x of mcol
  auto store0 = [&](int e, T val) {
    if (mcol)
      mcol[(long long)blockIdx.x * n0 + e] = (double)val;
    else
      dev::Gw(L[0].vt)[e] = val;
  };
  __syncthreads();
  // down: t = b - A x (x = w b), b_c = P^T t, x_c = w_c b_c
  for (int i = 0; i + 1 < nl; ++i) {
    const TailLevel<T> &v = L[i];
    const int nel = (int)(v.ncell << lg);
    const T *b = vec + voff[i];
    const T *x = b + nel;
    for (int e = tid; e < nel; e += TT) {
      const T a = tail_stencil(v, e, lg, x);
      if (gload(v.rowof + (e >> lg)) < 0)
        tv[e] = b[e] - a;
      else
        acc[e] = a;
    }
    __syncthreads();
    tail_u<T, TT>(v, lg, x, prod, pl.prodcap, [&](int e, T u) { tv[e] = b[e] - (acc[e] + u); });
    const TailLevel<T> &w = L[i + 1];
    const int ncel = (int)(w.ncell << lg), nc = (int)w.ncell;
    T *bc = vec + voff[i + 1];
    const bool xnext = i + 2 < nl;   // the coarsest level needs no x
    for (int e = tid; e < ncel; e += TT) {
      const int cc = e >> lg, k = e & mask;
      const auto ri = G(v.ri) + cc;
      const auto rw = G(v.rw) + cc;
      const int j0 = ri[0], j1 = ri[nc], j2 = ri[2 * nc];
      const T u1 = rw[0], u2 = rw[nc];
      T r = tv[(j0 << lg) | k];
      r = fma(u1, tv[(j1 << lg) | k], r);
      r = fma(u2, tv[(j2 << lg) | k], r);
      bc[e] = r;
      if (xnext) bc[ncel + e] = gload(w.rs + cc) * r;
    }
    __syncthreads();
  }
  // coarsest: one FP64 sweep from zero, or the direct solve (or the collapsed
  // cycle's matrix, by columns), into tv
  {
    const TailLevel<T> &v = L[nl - 1];
    const int nel = (int)(v.ncell << lg);
    const T *b = vec + voff[nl - 1];
    if (v.ndirect > 0) {
      const int nd = v.ndirect;
      const long long rs_ = v.colmajor ? 1 : nd, cs_ = v.colmajor ? nd : 1;   // strides of a row, a column
      for (int e = tid; e < nel; e += TT) {
        const int row = e >> lg, kr = e & mask;
        const auto ar = G(v.ainv) + (long long)row * rs_;
        double a = 0.0;
        for (int j = 0; j < nd; ++j) a = fma(ar[j * cs_], (double)b[(j << lg) + kr], a);
        if (nl == 1)
          store0(e, (T)a);
        else
          tv[e] = (T)a;
      }
    } else {
      for (int e = tid; e < nel; e += TT) {
        const T val = (T)(gload(v.rs64 + (e >> lg)) * (double)b[e]);
        if (nl == 1)
          store0(e, val);
        else
          tv[e] = val;
      }
    }
    __syncthreads();
  }
  // up: x += P x_c, then x + w (b - A x) into tv (level 0: into tl[0].vt)
  for (int i = nl - 2; i >= 0; --i) {
    const TailLevel<T> &v = L[i];
    const int nel = (int)(v.ncell << lg), n = (int)v.ncell;
    const T *b = vec + voff[i];
    T *x = vec + voff[i] + nel;
    for (int e = tid; e < nel; e += TT) {
      const int c = e >> lg, k = e & mask;
      const auto pi = G(v.pi) + c;
      const auto pw = G(v.pw) + c;
      const int i1 = pi[0], i2 = pi[n];
      const T w1 = pw[0], w2 = pw[n];
      T u = w1 * tv[(i1 << lg) | k];
      u = fma(w2, tv[(i2 << lg) | k], u);
      x[e] += u;
    }
    __syncthreads();
    auto put = [&](int e, T val) {
      if (i == 0)
        store0(e, val);
      else
        tv[e] = val;
    };
    for (int e = tid; e < nel; e += TT) {
      const T a = tail_stencil(v, e, lg, x);
      const int c = e >> lg;
      if (gload(v.rowof + c) < 0)
        put(e, x[e] + gload(v.rs + c) * (b[e] - a));
      else
        acc[e] = a;
    }
    __syncthreads();
    tail_u<T, TT>(v, lg, x, prod, pl.prodcap,
                  [&](int e, T u) { put(e, x[e] + gload(v.rs + (e >> lg)) * (b[e] - (acc[e] + u))); });
  }
}

// Pack of the level records tl[blockIdx.y] (levels 1 .. of at most kTailMax
// cells): one thread per cell of the level, and per cell of the next level
// for the restriction, from the part descriptors as the grid kernels read them.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tail_pack(TailLevel<T> *__restrict__ tl) {
  TailLevel<T> &v = tl[blockIdx.y];
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const int n = (int)v.ncell, nc = (int)v.nnext;
  auto part = [&](long long cell, bool coarse) {
    int lo = 0, hi = v.np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((coarse ? v.desc[mid].coff : v.desc[mid].off) <= cell)
        lo = mid;
      else
        hi = mid - 1;
    }
    return lo;
  };
  if (c < n) {
    const PartDesc<T> &d = v.desc[part(c, false)];
    const int cl = c - (int)d.off;
    int i, j, k;
    cell_ijk(cl, d.n[0], d.n[1], i, j, k);
    const unsigned mx = nb_mask(i, d.n[0]), my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
    // all table and coefficient loads first (clamped to entry 0), then the stores
    int lcv[kMaxEnt];
    T cv[kMaxEnt];
#pragma unroll
    for (int s = 0; s < kMaxEnt; ++s) {
      const int ss = s < d.nent ? s : 0;
      lcv[s] = d.lc[ss];
      cv[s] = d.coef[(long long)ss * d.ncell + cl];
    }
#pragma unroll
    for (int s = 0; s < kMaxEnt; ++s) {
      if (s >= v.nw) break;
      const bool ok = s < d.nent && nb_ok(mx, my, mz, lcv[s] & 63);
      v.nb[(long long)s * n + c] = ok ? c + (lcv[s] >> 6) : c;
      v.ca[(long long)s * n + c] = ok ? cv[s] : T(0);
    }
    // interpolation from the next level (interp_one's cases)
    int i1 = 0, i2 = 0;
    T w1 = T(0), w2 = T(0);
    if (nc > 0) {
      if (d.dstar < 0) {
        i1 = i2 = (int)d.coff + cl;
        w1 = T(1);
      } else {
        int f[3] = {i, j, k};
        const int ds = d.dstar, id = f[ds];
        int g[3] = {i, j, k};
        if ((id & 1) == 0) {
          g[ds] = id >> 1;
          i1 = i2 = (int)d.coff + g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2]);
          w1 = T(1);
        } else {
          g[ds] = (id - 1) >> 1;
          const int fl = g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2]);
          const int cm = g[0] + d.cn[0] * (g[1] + d.cn[1] * g[2]);
          i1 = i2 = (int)d.coff + cm;
          w1 = d.wm[fl];
          if (id + 1 <= d.n[ds] - 1) {
            const int cstride = ds == 0 ? 1 : (ds == 1 ? d.cn[0] : d.cn[0] * d.cn[1]);
            i2 = i1 + cstride;
            w2 = d.wp[fl];
          }
        }
      }
    }
    v.pi[c] = i1;
    v.pi[n + c] = i2;
    v.pw[c] = w1;
    v.pw[n + c] = w2;
    int lo = 0, hi = v.nrow;   // row of U holding c (urow ascending)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (v.urow[mid] < c)
        lo = mid + 1;
      else
        hi = mid;
    }
    v.rowof[c] = lo < v.nrow && v.urow[lo] == c ? lo : -1;
  }
  if (c < nc) {   // restriction into next-level cell c (restrict_one's cases)
    const PartDesc<T> &d = v.desc[part(c, true)];
    const int cc = c - (int)d.coff;
    int j0, j1, j2;
    T u1 = T(0), u2 = T(0);
    if (d.dstar < 0) {
      j0 = j1 = j2 = (int)d.off + cc;
    } else {
      int ci[3];
      cell_ijk(cc, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
      const int ds = d.dstar;
      int fi[3] = {ci[0], ci[1], ci[2]};
      fi[ds] = 2 * ci[ds];
      const int f0 = fi[0] + d.n[0] * (fi[1] + d.n[1] * fi[2]);
      const int stride = ds == 0 ? 1 : (ds == 1 ? d.n[0] : d.n[0] * d.n[1]);
      j0 = j1 = j2 = (int)d.off + f0;
      int g[3] = {ci[0], ci[1], ci[2]};
      if (fi[ds] - 1 >= 0) {
        g[ds] = ci[ds] - 1;
        u1 = d.wp[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])];
        j1 = j0 - stride;
      }
      if (fi[ds] + 1 <= d.n[ds] - 1) {
        g[ds] = ci[ds];
        u2 = d.wm[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])];
        j2 = j0 + stride;
      }
    }
    v.ri[c] = j0;
    v.ri[nc + c] = j1;
    v.ri[2 * nc + c] = j2;
    v.rw[c] = u1;
    v.rw[nc + c] = u2;
  }
}

// One coarsest level of any size with its vectors in global memory (the
// hierarchy's only level, or a coarsest level too large for the coarse-end
// kernel): vt = (FP64 sweep from zero or A^{-1}) vb.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarsest(const TailLevel<T> *__restrict__ tl, int lg) {
  const TailLevel<T> &v = *tl;
  const long long nel = v.ncell << lg;
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nel) return;
  const int mask = (1 << lg) - 1;
  if (v.ndirect > 0) {   // the direct solve's inverse by rows, or the collapsed cycle's matrix by columns
    const int row = (int)(e >> lg), kr = (int)(e & mask);
    const long long rs_ = v.colmajor ? 1 : v.ndirect, cs_ = v.colmajor ? v.ndirect : 1;
    const double *ar = v.ainv + (long long)row * rs_;
    double a = 0.0;
    for (int j = 0; j < v.ndirect; ++j) a = fma(ar[j * cs_], (double)v.vb[((long long)j << lg) + kr], a);
    v.vt[e] = (T)a;
  } else {
    v.vt[e] = (T)(v.rs64[e >> lg] * (double)v.vb[e]);
  }
}

// First pass of the fused product dot over the groups of four one-column slots
// (per = 4: the one-column product's slots, added as ((s0 + s1) + s2) + s3;
// per = 1: the four-column product's group sums).  Block g takes a fixed
// range of groups; within it, lane u of right-hand side k takes every
// (kBlock >> lg)-th group in order, then a fixed tree; out[g][k] with row
// stride kMaxRhs (the layout k_dot_final reads).
__global__ __launch_bounds__(kBlock) void k_dot_groups(const double *__restrict__ dotp, long long ngroups,
                                                       int lg, int per, double *__restrict__ out) {
  __shared__ double sh[kBlock];
  // blockIdx.y: the set (the second one follows the first in both buffers)
  dotp += ((long long)blockIdx.y * ngroups * per) << lg;
  out += (size_t)blockIdx.y * kRedBlocks * kMaxRhs;
  const int nr = 1 << lg;
  const int k = threadIdx.x & (nr - 1), u = threadIdx.x >> lg, nu = kBlock >> lg;
  const long long gpb = (ngroups + gridDim.x - 1) / gridDim.x;
  const long long g0 = (long long)blockIdx.x * gpb;
  const long long g1 = g0 + gpb < ngroups ? g0 + gpb : ngroups;
  double acc = 0.0;
  for (long long g = g0 + u; g < g1; g += nu) {
    if (per == 4) {
      const double *q = dotp + ((4 * g) << lg) + k;
      acc += ((q[0] + q[nr]) + q[2 * nr]) + q[3 * nr];
    } else {
      acc += dotp[(g << lg) + k];
    }
  }
  sh[threadIdx.x] = acc;
  for (int s = kBlock / 2; s >= nr; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) out[blockIdx.x * kMaxRhs + threadIdx.x] = sh[threadIdx.x];
}

// ---------------------------------------------------------------- FP64 product, two cells per thread

// The U part of A x for CPT consecutive cells per thread (one right-hand
// side): the block covers the 256-cell chunks CPT b .. CPT b + CPT - 1, whose
// rows and entries are contiguous; products staged in LDS as in
// block_coupling, each row summed in entry order by one thread (the same sums,
// bit for bit, as there).  out[k] is cell CPT tid + k of the block.  Must be
// called by every thread of the block.
template <int CPT, typename T>
__device__ __forceinline__ void block_coupling_multi(const PartDesc<T> &d, int bk, const T *x,
                                                     T *__restrict__ prod, T *__restrict__ rsum, T (&out)[CPT]) {
#pragma unroll
  for (int k = 0; k < CPT; ++k) out[k] = T(0);
  const long long nch = (d.ncell + kBlock - 1) / kBlock;   // the table holds nch + 1 entries
  const long long ca = min((long long)CPT * bk, nch), cb = min((long long)CPT * bk + CPT, nch);
  const auto ub = G(d.ublk[0]);
  const int u0 = ub[2 * ca], e0 = ub[2 * ca + 1], u1 = ub[2 * cb], e1 = ub[2 * cb + 1];
  if (u0 == u1) return;                                    // block-uniform
  const int tid = threadIdx.x;
  const int cell0 = (int)d.off + bk * CPT * kBlock;
  const int nrt = u1 - u0;                                 // rows of the block, at most CPT * 256
  int rq0[CPT], rq1[CPT], rslot[CPT];
  T racc[CPT];
#pragma unroll
  for (int h = 0; h < CPT; ++h) {
    const int r = tid + h * kBlock;
    rq0[h] = rq1[h] = rslot[h] = 0;
    racc[h] = T(0);
    if (r < nrt) {
      rq0[h] = G(d.uptr)[u0 + r];
      rq1[h] = G(d.uptr)[u0 + r + 1];
      rslot[h] = G(d.urow)[u0 + r] - cell0;
    }
    rsum[tid + h * kBlock] = T(0);
  }
  constexpr int per = kUChunkBig;
  for (int ec = e0; ec < e1; ec += per) {
    const int np = min(per, e1 - ec);
    int cc[per / kBlock];
    T vv[per / kBlock], xx[per / kBlock];
#pragma unroll
    for (int t = 0; t < per / kBlock; ++t) {
      const int q = tid + t * kBlock;
      const int qe = ec + (q < np ? q : 0);
      cc[t] = gload(d.ucol + qe);
      vv[t] = gload(d.uval + qe);
    }
#pragma unroll
    for (int t = 0; t < per / kBlock; ++t) xx[t] = t * kBlock < np ? x[cc[t]] : T(0);
#pragma unroll
    for (int t = 0; t < per / kBlock; ++t) {
      const int q = tid + t * kBlock;
      if (q < np) prod[q] = vv[t] * xx[t];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < CPT; ++h)
      if (tid + h * kBlock < nrt) {
        const int qa = max(rq0[h], ec), qb = min(rq1[h], ec + np);
        racc[h] = row_sum(prod, qa - ec, qb - ec, 0, 0, racc[h]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < CPT; ++h)
    if (tid + h * kBlock < nrt) rsum[rslot[h]] = racc[h];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < CPT; ++k) out[k] = rsum[CPT * tid + k];
}

// q = A p and the per-256-cell partial sums of p.q (Section 2 product; the
// PCG product of Section 4) on the finest level when every part has the full
// 27-point stencil and an even number of cells along x: two cells (c, c + 1)
// of a row per thread, so every coefficient and vector value comes in a
// 16-byte pair - half the load instructions of the one-cell kernel, which
// bound that kernel (its address and data traffic between L1 and registers,
// not HBM).  With MIR the entries of negative offset are read as the
// neighbour's mirrored entry (a_s(c) = a_{-s}(c+s)); their pairs start at an
// odd cell and are assembled from two aligned pairs.  Vector values come as
// the three aligned pairs (c-2, c-1), (c, c+1), (c+2, c+3) of each of the
// nine rows.  A neighbour outside the box reads an in-bounds address and is
// zeroed.  The stencil sums run in (dz, dy, dx) order; the coupling sums and
// the partial slots are those of the one-cell kernel.
// 16-byte load at a uniform base plus a 32-bit byte offset (one offset
// register per load, the base in scalar registers)
typedef double dpair __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dpair ld2(const double *base, unsigned byteoff) {
  return *(dev::gptr<dpair>)((dev::gptr<char>)G(base) + byteoff);
}

__device__ __forceinline__ double ld1(const double *base, unsigned byteoff) {
  return *(dev::gptr<double>)((dev::gptr<char>)G(base) + byteoff);
}

// a double from another lane of the wave by a whole-wave DPP shift (CTRL
// 0x138: from lane - 1; 0x130: from lane + 1; 0 where there is none); every
// lane of the wave must execute it
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <bool MIR>
__global__ __launch_bounds__(kBlock) void k_product2(const PartDesc<double> *__restrict__ desc, int nb1,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     double *__restrict__ dotp) {
  __shared__ double prod[kUChunkBig];
  __shared__ double sh[2 * kBlock];
  const PartDesc<double> &d = desc[blockIdx.y];
  const int b2 = chunk_index();
  const int tid = threadIdx.x;
  const long long c = (long long)b2 * (2 * kBlock) + 2 * tid;
  const bool valid = c < d.ncell;
  const int cc = valid ? (int)c : 0;
  int i, j, k;
  cell_ijk(cc, d.n[0], d.n[1], i, j, k);
  const unsigned my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const bool xl = i > 0;                   // cell c has its -x neighbour
  const bool xr = i + 2 < d.n[0];          // cell c + 1 has its +x neighbour
  const int nx = d.n[0], nxy = d.n[0] * d.n[1];
  const double *xb = x + d.off;
  const unsigned c8 = 8u * (unsigned)cc;
  double acc0 = 0.0, acc1 = 0.0, xc0 = 0.0, xc1 = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const bool row = ((my >> (dy + 1)) & (mz >> (dz + 1)) & 1u) != 0;
      const unsigned r8 = c8 + 8u * (unsigned)(row ? dy * nx + dz * nxy : 0);   // byte offset of (c + row)
      const bool okm = row && xl, okp = row && xr;
      const dpair xm = ld2(xb, okm ? r8 - 16u : r8);
      const dpair xz = ld2(xb, r8);
      const dpair xp = ld2(xb, okp ? r8 + 16u : r8);
      const double xv0[3] = {okm ? xm.y : 0.0, row ? xz.x : 0.0, row ? xz.y : 0.0};
      const double xv1[3] = {row ? xz.x : 0.0, row ? xz.y : 0.0, okp ? xp.x : 0.0};
      if (dz == 0 && dy == 0) {
        xc0 = xz.x;
        xc1 = xz.y;
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const bool neg = dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)));
        double a0, a1;
        if (MIR && neg) {
          // a_s(c) = a_{-s}(c + s): entry -s at the neighbour c + s (row r8 + dx)
          const double *arr = d.coef + (long long)d.cube[26 - o] * d.ncell;
          if (dx == 0) {
            const dpair v = ld2(arr, r8);
            a0 = v.x;
            a1 = v.y;
          } else {
            const bool ok0 = row && (dx > 0 || xl), ok1 = row && (dx < 0 || xr);
            const dpair u = ld2(arr, ok0 ? r8 + 8u * (unsigned)(dx - 1) : c8);
            const dpair w = ld2(arr, ok1 ? r8 + 8u * (unsigned)(dx + 1) : c8);
            a0 = u.y;
            a1 = w.x;
          }
        } else {
          const dpair v = ld2(d.coef + (long long)d.cube[o] * d.ncell, c8);
          a0 = v.x;
          a1 = v.y;
        }
        acc0 = fma(a0, xv0[dx + 1], acc0);
        acc1 = fma(a1, xv1[dx + 1], acc1);
      }
    }
  }
  double u[2];
  block_coupling_multi<2>(d, b2, xb - d.off, prod, sh, u);
  acc0 += u[0];
  acc1 += u[1];
  if (valid) *(double2 *)(y + d.off + cc) = make_double2(acc0, acc1);
  // p.q per 256-cell chunk 2 b2 and 2 b2 + 1 (the one-cell kernel's tree)
  __syncthreads();
  sh[2 * tid] = valid ? xc0 * acc0 : 0.0;
  sh[2 * tid + 1] = valid ? xc1 * acc1 : 0.0;
  const int half = tid >> 7, t = tid & 127;   // threads 0..127 reduce chunk 2 b2, 128..255 the next
  for (int s = kBlock / 2; s >= 1; s >>= 1) {
    __syncthreads();
    if (t < s) sh[half * kBlock + t] += sh[half * kBlock + t + s];
  }
  __syncthreads();
  const long long slots = 4LL * ((nb1 + 3) / 4);
  double *dslot = dotp + (long long)blockIdx.y * slots;
  if (tid < 2) {
    const long long ch = 2LL * b2 + tid;
    if (ch < nb1) dslot[ch] = sh[tid * kBlock];
  }
  // the block holding the one-cell grid's last chunk clears the rounding slots
  if ((nb1 - 1) / 2 == b2 && tid < slots - nb1) dslot[nb1 + tid] = 0.0;
}

// k_product2 with the x values at c - 1 and c + 2 of each row taken from the
// lanes before and after (they hold them as their own pairs; a lane whose
// neighbour in the row lies in another wave loads it): one pair load per row
// instead of three.  Every load is issued first (the rows' own pairs, then
// the coefficients), the few loads of the waves' edge lanes after them in one
// branch, then the shifts and the sums in the same order as k_product2 (the
// same bits).
template <bool MIR>
__global__ __launch_bounds__(kBlock) void k_product2s(const PartDesc<double> *__restrict__ desc, int nb1,
                                                      const double *__restrict__ x, double *__restrict__ y,
                                                      double *__restrict__ dotp) {
  __shared__ double prod[kUChunkBig];
  __shared__ double sh[2 * kBlock];
  const PartDesc<double> &d = desc[blockIdx.y];
  const int b2 = chunk_index();
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const long long c = (long long)b2 * (2 * kBlock) + 2 * tid;
  const bool valid = c < d.ncell;
  const int cc = valid ? (int)c : 0;
  int i, j, k;
  cell_ijk(cc, d.n[0], d.n[1], i, j, k);
  const unsigned my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const bool xl = i > 0;                   // cell c has its -x neighbour
  const bool xr = i + 2 < d.n[0];          // cell c + 1 has its +x neighbour
  const int nx = d.n[0], nxy = d.n[0] * d.n[1];
  const double *xb = x + d.off;
  const unsigned c8 = 8u * (unsigned)cc;
  bool row[9];
  unsigned r8[9];
  dpair xz[9];
  double a0[27], a1[27];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int ri = (dy + 1) + 3 * (dz + 1);
      row[ri] = ((my >> (dy + 1)) & (mz >> (dz + 1)) & 1u) != 0;
      r8[ri] = c8 + 8u * (unsigned)(row[ri] ? dy * nx + dz * nxy : 0);
      xz[ri] = ld2(xb, r8[ri]);
    }
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int ri = (dy + 1) + 3 * (dz + 1);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const bool neg = dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)));
        if (MIR && neg) {
          const double *arr = d.coef + (long long)d.cube[26 - o] * d.ncell;
          if (dx == 0) {
            const dpair v = ld2(arr, r8[ri]);
            a0[o] = v.x;
            a1[o] = v.y;
          } else {
            const bool ok0 = row[ri] && (dx > 0 || xl), ok1 = row[ri] && (dx < 0 || xr);
            const dpair u = ld2(arr, ok0 ? r8[ri] + 8u * (unsigned)(dx - 1) : c8);
            const dpair w = ld2(arr, ok1 ? r8[ri] + 8u * (unsigned)(dx + 1) : c8);
            a0[o] = u.y;
            a1[o] = w.x;
          }
        } else {
          const dpair v = ld2(d.coef + (long long)d.cube[o] * d.ncell, c8);
          a0[o] = v.x;
          a1[o] = v.y;
        }
      }
    }
  // x at c - 1 and c + 2 of every row: from the lanes before and after
  double xlo[9], xhi[9];
#pragma unroll
  for (int ri = 0; ri < 9; ++ri) {
    xlo[ri] = wave_shift<0x138>(xz[ri].y);
    xhi[ri] = wave_shift<0x130>(xz[ri].x);
  }
  if (lane == 0 && xl) {
#pragma unroll
    for (int ri = 0; ri < 9; ++ri)
      if (row[ri]) xlo[ri] = ld1(xb, r8[ri] - 8u);
  }
  if (lane == 63 && xr) {
#pragma unroll
    for (int ri = 0; ri < 9; ++ri)
      if (row[ri]) xhi[ri] = ld1(xb, r8[ri] + 16u);
  }
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int ri = 0; ri < 9; ++ri) {
    const bool okm = row[ri] && xl, okp = row[ri] && xr;
    const double xv0[3] = {okm ? xlo[ri] : 0.0, row[ri] ? xz[ri].x : 0.0, row[ri] ? xz[ri].y : 0.0};
    const double xv1[3] = {row[ri] ? xz[ri].x : 0.0, row[ri] ? xz[ri].y : 0.0, okp ? xhi[ri] : 0.0};
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int o = (dx + 1) + 3 * ri;
      acc0 = fma(a0[o], xv0[dx + 1], acc0);
      acc1 = fma(a1[o], xv1[dx + 1], acc1);
    }
  }
  const double xc0 = xz[4].x, xc1 = xz[4].y;
  double u[2];
  block_coupling_multi<2>(d, b2, xb - d.off, prod, sh, u);
  acc0 += u[0];
  acc1 += u[1];
  if (valid) *(double2 *)(y + d.off + cc) = make_double2(acc0, acc1);
  // p.q per 256-cell chunk 2 b2 and 2 b2 + 1 (the one-cell kernel's tree)
  __syncthreads();
  sh[2 * tid] = valid ? xc0 * acc0 : 0.0;
  sh[2 * tid + 1] = valid ? xc1 * acc1 : 0.0;
  const int half = tid >> 7, t = tid & 127;
  for (int s = kBlock / 2; s >= 1; s >>= 1) {
    __syncthreads();
    if (t < s) sh[half * kBlock + t] += sh[half * kBlock + t + s];
  }
  __syncthreads();
  const long long slots = 4LL * ((nb1 + 3) / 4);
  double *dslot = dotp + (long long)blockIdx.y * slots;
  if (tid < 2) {
    const long long ch = 2LL * b2 + tid;
    if (ch < nb1) dslot[ch] = sh[tid * kBlock];
  }
  if ((nb1 - 1) / 2 == b2 && tid < slots - nb1) dslot[nb1 + tid] = 0.0;
}

// CPT consecutive values of type T at a uniform base plus a 32-bit byte offset
template <typename T, int CPT>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(CPT)));
};
template <typename T, int CPT>
__device__ __forceinline__ typename VecOf<T, CPT>::type ldv(const T *base, unsigned byteoff) {
  return *(dev::gptr<typename VecOf<T, CPT>::type>)((dev::gptr<char>)G(base) + byteoff);
}

// The finest level's residual t = b - A x (MODE_RESID) and post-smoothing
// sweep z = x + w (b - A x) (MODE_JACOBI) of the V-cycle (Section 3.4,
// eq:relax0; one right-hand side, b in FP64) on a level whose parts all have
// the full 27-point stencil and a multiple of CPT cells along x: CPT cells of
// a row per thread (16-byte vectors: 2 FP64 or 4 FP32 values), every entry
// read (no mirror), vector values as the three aligned vectors before, at and
// after the thread's cells in each of the nine rows; stencil sums in
// (dz, dy, dx) order, couplings as in the one-cell kernel.
template <typename T, int MODE, typename TO, int CPT>
__global__ __launch_bounds__(kBlock) void k_sweepN(const PartDesc<T> *__restrict__ desc, const T *__restrict__ x,
                                                   const double *__restrict__ b, TO *__restrict__ y) {
  __shared__ T prod[kUChunkBig];
  __shared__ T sh[CPT * kBlock];
  const PartDesc<T> &d = desc[blockIdx.y];
  const int bk = chunk_index();
  const int tid = threadIdx.x;
  const long long c = (long long)bk * (CPT * kBlock) + CPT * tid;
  const bool valid = c < d.ncell;
  const int cc = valid ? (int)c : 0;
  int i, j, k;
  cell_ijk(cc, d.n[0], d.n[1], i, j, k);
  const unsigned my = nb_mask(j, d.n[1]), mz = nb_mask(k, d.n[2]);
  const bool xl = i > 0, xr = i + CPT < d.n[0];   // first cell's -x, last cell's +x neighbour
  const int nx = d.n[0], nxy = d.n[0] * d.n[1];
  const T *xb = x + d.off;
  constexpr unsigned ts = sizeof(T);
  const unsigned ct = ts * (unsigned)cc;
  T acc[CPT], xc[CPT], ac[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = xc[q] = ac[q] = T(0);
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const bool row = ((my >> (dy + 1)) & (mz >> (dz + 1)) & 1u) != 0;
      const unsigned rt = ct + ts * (unsigned)(row ? dy * nx + dz * nxy : 0);
      const bool okm = row && xl, okp = row && xr;
      const auto xm = ldv<T, CPT>(xb, okm ? rt - CPT * ts : rt);
      const auto xz = ldv<T, CPT>(xb, rt);
      const auto xp = ldv<T, CPT>(xb, okp ? rt + CPT * ts : rt);
      T xv[CPT + 2];   // values at cells c - 1 .. c + CPT of the row
      xv[0] = okm ? xm[CPT - 1] : T(0);
#pragma unroll
      for (int q = 0; q < CPT; ++q) xv[q + 1] = row ? xz[q] : T(0);
      xv[CPT + 1] = okp ? xp[0] : T(0);
      if (dz == 0 && dy == 0)
#pragma unroll
        for (int q = 0; q < CPT; ++q) xc[q] = xz[q];
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const auto v = ldv<T, CPT>(d.coef + (long long)d.cube[o] * d.ncell, ct);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          if (o == 13) ac[q] = v[q];
          acc[q] = fma(v[q], xv[q + 1 + dx], acc[q]);
        }
      }
    }
  }
  T u[CPT];
  block_coupling_multi<CPT>(d, bk, xb - d.off, prod, sh, u);
  if (!valid) return;
  const long long o = d.off + cc;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const T r = (T)b[o + q] - (acc[q] + u[q]);
    if constexpr (MODE == MODE_RESID) {
      y[o + q] = (TO)r;
    } else {
      const T w = d.rs ? G(d.rs)[cc + q] : d.omega / ac[q];
      y[o + q] = (TO)(xc[q] + w * r);
    }
  }
}

// kernel<<<grid, kBlock>>>(args...) on st, timed by ev when ev.start is set
template <typename K, typename... A>
inline void dispatch(K kernel, dim3 grid, hipStream_t st, const LaunchEvents &ev, A... args) {
  if (ev.start)
    hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, ev.start, ev.stop, 0, args...);
  else
    kernel<<<grid, kBlock, 0, st>>>(args...);
}

inline unsigned grid_cells(long long n, int lg) {
  long long nb = ((n << lg) + kBlock - 1) / kBlock;
  return (unsigned)(nb > 0 ? nb : 1);
}

template <typename T, typename TB, typename TO, int BIG, int NENT>
void stencil_mode(int mode, dim3 grid, const PartDesc<T> *desc, int lg, const T *x, const TB *b, TO *y,
                  hipStream_t st, const LaunchEvents &ev, bool c4, double *dotp, const double *aux,
                  bool mir) {
  constexpr bool fp64_out = sizeof(TO) == 8 && sizeof(TB) == 8;
  // the FP64 product of a symmetric stencil: mirrored reads, for one column at
  // any stencil size and for batches on stencils of more than 7 points
  if constexpr (sizeof(T) == 8 && fp64_out) {
    if (mir && (NENT > 7 || lg == 0) && (mode == MODE_APPLY || mode == MODE_APPLY_DOT)) {
      if (c4) {
        dim3 g4((unsigned)(((long long)grid.x + 3) / 4), grid.y);
        if (mode == MODE_APPLY)
          dispatch(k_stencil4<T, MODE_APPLY, TB, TO, BIG, NENT, true>, g4, st, ev, desc, lg, x, b, y, dotp, aux);
        else
          dispatch(k_stencil4<T, MODE_APPLY_DOT, TB, TO, BIG, NENT, true>, g4, st, ev, desc, lg, x, b, y, dotp,
                   aux);
      } else {
        if (mode == MODE_APPLY)
          dispatch(k_stencil<T, MODE_APPLY, TB, TO, BIG, NENT, true>, grid, st, ev, desc, lg, x, b, y, dotp, aux);
        else
          dispatch(k_stencil<T, MODE_APPLY_DOT, TB, TO, BIG, NENT, true>, grid, st, ev, desc, lg, x, b, y, dotp,
                   aux);
      }
      return;
    }
  }
  if (c4) {
    dim3 g4((grid.x + 3) / 4 > 0 ? (unsigned)(((long long)grid.x + 3) / 4) : 1u, grid.y);
#define SSAMG_S4(M) dispatch(k_stencil4<T, M, TB, TO, BIG, NENT>, g4, st, ev, desc, lg, x, b, y, dotp, aux)
    if (mode == MODE_APPLY) SSAMG_S4(MODE_APPLY);
    else if (mode == MODE_RESID) SSAMG_S4(MODE_RESID);
    else if (mode == MODE_JACOBI) SSAMG_S4(MODE_JACOBI);
    else if constexpr (fp64_out && sizeof(T) == 8) { if (mode == MODE_APPLY_DOT) SSAMG_S4(MODE_APPLY_DOT); }
    if constexpr (fp64_out && BIG) { if (mode == MODE_JACOBI_DOT) SSAMG_S4(MODE_JACOBI_DOT); }
#undef SSAMG_S4
    return;
  }
#define SSAMG_S1(M) dispatch(k_stencil<T, M, TB, TO, BIG, NENT>, grid, st, ev, desc, lg, x, b, y, dotp, aux)
  if (mode == MODE_APPLY) SSAMG_S1(MODE_APPLY);
  else if (mode == MODE_RESID) SSAMG_S1(MODE_RESID);
  else if (mode == MODE_JACOBI) SSAMG_S1(MODE_JACOBI);
  else if constexpr (fp64_out && sizeof(T) == 8) { if (mode == MODE_APPLY_DOT) SSAMG_S1(MODE_APPLY_DOT); }
  if constexpr (fp64_out && BIG) { if (mode == MODE_JACOBI_DOT) SSAMG_S1(MODE_JACOBI_DOT); }
#undef SSAMG_S1
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T, typename TO>
void launch_sweep2(int mode, const PartDesc<T> *desc, int nparts, int maxcell, const T *x, const double *b, TO *y,
                   hipStream_t st, LaunchEvents ev) {
  constexpr int cpt = 16 / sizeof(T);
  dim3 grid((unsigned)((grid_cells(maxcell, 0) + cpt - 1) / cpt), nparts);
  if (mode == MODE_RESID)
    dispatch(k_sweepN<T, MODE_RESID, TO, cpt>, grid, st, ev, desc, x, b, y);
  else if (mode == MODE_JACOBI)
    dispatch(k_sweepN<T, MODE_JACOBI, TO, cpt>, grid, st, ev, desc, x, b, y);
  else
    throw Error(SSAMG_ERR_STATE, "internal: multi-cell sweep mode");
}
template void launch_sweep2<float, float>(int, const PartDesc<float> *, int, int, const float *, const double *,
                                          float *, hipStream_t, LaunchEvents);
template void launch_sweep2<float, double>(int, const PartDesc<float> *, int, int, const float *, const double *,
                                           double *, hipStream_t, LaunchEvents);
template void launch_sweep2<double, double>(int, const PartDesc<double> *, int, int, const double *,
                                            const double *, double *, hipStream_t, LaunchEvents);

void launch_product2(const PartDesc<double> *desc, int nparts, int maxcell, bool mir, bool share,
                     const double *x, double *y, double *dotp, hipStream_t st, LaunchEvents ev) {
  const int nb1 = (int)grid_cells(maxcell, 0);
  dim3 grid((unsigned)((nb1 + 1) / 2), nparts);
  if (mir && share)
    dispatch(k_product2s<true>, grid, st, ev, desc, nb1, x, y, dotp);
  else if (mir)
    dispatch(k_product2<true>, grid, st, ev, desc, nb1, x, y, dotp);
  else if (share)
    dispatch(k_product2s<false>, grid, st, ev, desc, nb1, x, y, dotp);
  else
    dispatch(k_product2<false>, grid, st, ev, desc, nb1, x, y, dotp);
}

template <typename T, typename TB, typename TO>
void launch_stencil(int mode, int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell,
                    int lg, const T *x, const TB *b, TO *y, hipStream_t st, LaunchEvents ev, int cols4,
                    double *dotp, const double *aux, bool mir) {
  if (mode == MODE_APPLY_DOT && !(sizeof(T) == 8 && sizeof(TO) == 8 && dotp))
    throw Error(SSAMG_ERR_STATE, "internal: the fused product dot needs FP64 and a partial buffer");
  if (mode == MODE_JACOBI_DOT && !(sizeof(TB) == 8 && sizeof(TO) == 8 && fine && dotp))
    throw Error(SSAMG_ERR_STATE, "internal: the fused sweep dots need the finest level and a partial buffer");
  dim3 grid(grid_cells(maxcell, lg), nparts);
  const bool c4 = cols4 != 0 && stencil_cols4_ok<T>(lg, maxent);
  if (fine || (((long long)maxcell * nparts) << lg) >= kBigLevel) {
    if (maxent <= 7)
      stencil_mode<T, TB, TO, 1, 7>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
    else if (maxent <= 15)
      stencil_mode<T, TB, TO, 1, 15>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
    else
      stencil_mode<T, TB, TO, 1, 27>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
  } else {
    if (maxent <= 7)
      stencil_mode<T, TB, TO, 0, 7>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
    else if (maxent <= 15)
      stencil_mode<T, TB, TO, 0, 15>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
    else
      stencil_mode<T, TB, TO, 0, 27>(mode, grid, desc, lg, x, b, y, st, ev, c4, dotp, aux, mir);
  }
}

template <typename T, typename TB>
void launch_smooth_zero(int fine, const PartDesc<T> *desc, int nparts, int maxcell, int lg, const TB *b,
                        T *x, hipStream_t st) {
  if (lg >= 2)
    k_smooth_zero4<T, TB><<<dim3(grid_cells(maxcell, lg - 2), nparts), kBlock, 0, st>>>(desc, lg, b, x);
  else if (fine)
    k_smooth_zero<T, TB, 1><<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
  else
    k_smooth_zero<T, TB, 0><<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
}

template <typename T>
void launch_restrict(const PartDesc<T> *desc, int nparts, int maxcoarse, int lg, const T *r, T *bc,
                     hipStream_t st, LaunchEvents ev, const T *wn, T *xn) {
  if (lg >= 2) {
    if (xn) throw Error(SSAMG_ERR_STATE, "internal: the four-column restriction forms no first sweep");
    dispatch(k_restrict4<T>, dim3(grid_cells(maxcoarse, lg - 2), nparts), st, ev, desc, lg, r, bc);
  } else {
    dispatch(k_restrict<T>, dim3(grid_cells(maxcoarse, lg), nparts), st, ev, desc, lg, r, bc, wn, xn);
  }
}

template <typename T>
void launch_interp_add(const PartDesc<T> *desc, int nparts, int maxcell, int lg, const T *xc, T *x,
                       hipStream_t st, LaunchEvents ev) {
  if (lg >= 2)
    dispatch(k_interp_add4<T>, dim3(grid_cells(maxcell, lg - 2), nparts), st, ev, desc, lg, xc, x);
  else
    dispatch(k_interp_add<T>, dim3(grid_cells(maxcell, lg), nparts), st, ev, desc, lg, xc, x);
}

void launch_coarse_mixed(const PartDesc<double> *desc, int nparts, int maxcell, int lg, const float *b,
                         float *x, hipStream_t st) {
  k_coarse_mixed<<<dim3(grid_cells(maxcell, lg), nparts), kBlock, 0, st>>>(desc, lg, b, x);
}

template <typename T, typename TB>
void launch_smooth_resid(int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell, int lg,
                         const TB *b, T *x, T *r, hipStream_t st, LaunchEvents ev) {
  dim3 grid(grid_cells(maxcell, lg), nparts);
#define SSAMG_SR(F, N) dispatch(k_smooth_resid<T, TB, F, N>, grid, st, ev, desc, lg, b, x, r)
  if (fine || (((long long)maxcell * nparts) << lg) >= kBigLevel) {
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

void launch_dot_groups(const double *dotp, int64_t ngroups, int lg, int per, int nset, double *partial,
                       hipStream_t st) {
  k_dot_groups<<<dim3(kDotGroupBlocks, nset), kBlock, 0, st>>>(dotp, ngroups, lg, per, partial);
}

template <typename T>
void launch_tail(const TailLevel<T> *tl, const TailPlan &pl, int lg, hipStream_t st, double *mcol, int n) {
  constexpr int tt = sizeof(T) == 8 ? kTailThreads / 2 : kTailThreads;
  k_tail<T, tt><<<mcol ? n : 1, tt, pl.bytes, st>>>(tl, pl, lg, mcol);
}

template <typename T>
void launch_coarsest(const TailLevel<T> *tl, int64_t nel, int lg, hipStream_t st) {
  k_coarsest<T><<<grid_cells(nel, 0), kBlock, 0, st>>>(tl, lg);
}

template <typename T>
void launch_tail_pack(TailLevel<T> *tl, int nlev, int64_t maxcell, hipStream_t st) {
  if (nlev > 0) k_tail_pack<T><<<dim3(grid_cells(maxcell, 0), nlev), kBlock, 0, st>>>(tl);
}

template void launch_stencil<double, double, double>(int, int, int, const PartDesc<double> *, int, int,
                                                     int, const double *, const double *, double *,
                                                     hipStream_t, LaunchEvents, int, double *, const double *, bool);
template void launch_stencil<float, float, float>(int, int, int, const PartDesc<float> *, int, int, int,
                                                  const float *, const float *, float *, hipStream_t, LaunchEvents, int, double *, const double *, bool);
template void launch_stencil<float, double, float>(int, int, int, const PartDesc<float> *, int, int, int,
                                                   const float *, const double *, float *, hipStream_t, LaunchEvents, int, double *, const double *, bool);
template void launch_stencil<float, double, double>(int, int, int, const PartDesc<float> *, int, int, int,
                                                    const float *, const double *, double *, hipStream_t, LaunchEvents, int, double *, const double *, bool);
template void launch_smooth_zero<double, double>(int, const PartDesc<double> *, int, int, int,
                                                 const double *, double *, hipStream_t);
template void launch_smooth_zero<float, float>(int, const PartDesc<float> *, int, int, int, const float *,
                                               float *, hipStream_t);
template void launch_smooth_zero<float, double>(int, const PartDesc<float> *, int, int, int,
                                                const double *, float *, hipStream_t);
template void launch_restrict<double>(const PartDesc<double> *, int, int, int, const double *, double *,
                                      hipStream_t, LaunchEvents, const double *, double *);
template void launch_restrict<float>(const PartDesc<float> *, int, int, int, const float *, float *,
                                     hipStream_t, LaunchEvents, const float *, float *);
template void launch_interp_add<double>(const PartDesc<double> *, int, int, int, const double *, double *,
                                        hipStream_t, LaunchEvents);
template void launch_interp_add<float>(const PartDesc<float> *, int, int, int, const float *, float *,
                                       hipStream_t, LaunchEvents);
template void launch_smooth_resid<double, double>(int, int, const PartDesc<double> *, int, int, int,
                                                  const double *, double *, double *, hipStream_t, LaunchEvents);
template void launch_smooth_resid<float, float>(int, int, const PartDesc<float> *, int, int, int,
                                                const float *, float *, float *, hipStream_t, LaunchEvents);
template void launch_smooth_resid<float, double>(int, int, const PartDesc<float> *, int, int, int,
                                                 const double *, float *, float *, hipStream_t, LaunchEvents);
template void launch_tail<double>(const TailLevel<double> *, const TailPlan &, int, hipStream_t, double *, int);
template void launch_tail<float>(const TailLevel<float> *, const TailPlan &, int, hipStream_t, double *, int);
template void launch_coarsest<double>(const TailLevel<double> *, int64_t, int, hipStream_t);
template void launch_coarsest<float>(const TailLevel<float> *, int64_t, int, hipStream_t);
template void launch_tail_pack<double>(TailLevel<double> *, int, int64_t, hipStream_t);
template void launch_tail_pack<float>(TailLevel<float> *, int, int64_t, hipStream_t);

}  // namespace ssamg
