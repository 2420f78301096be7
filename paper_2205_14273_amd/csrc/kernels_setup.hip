// Setup kernels (gfx950): Dirichlet elimination, the grid-spacing metric
// reduction (Section 3.1), operator-collapse interpolation weights (Section
// 3.2, eq:prolEx), the structured Galerkin product P^T S P as a stencil triple
// product (Section 3.3), the numeric part of P^T U P, and the relaxation
// scale of the coupling rows.
#include "device_util.h"
#include "ssamg_impl.h"

namespace ssamg {

namespace {

__device__ __forceinline__ void cell_ijk(int c, int nx, int ny, int &i, int &j, int &k) {
  i = c % nx;
  int t = c / nx;
  j = t % ny;
  k = t / ny;
}

__device__ __forceinline__ int off_comp(int code, int d) { return ((code >> (2 * d)) & 3) - 1; }

// Zero every coefficient whose neighbour lies outside the box; flag a
// nonpositive or non-finite diagonal or a non-finite coefficient, and
// (separately) an in-box pair that breaks a_s(c) = a_{-s}(c+s).  Both members
// of an in-box pair keep their values, so the test reads them unchanged.
__global__ __launch_bounds__(kBlock) void k_normalise(BoxStencil bs, int *__restrict__ flag) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= bs.ncell) return;
  int i, j, k;
  cell_ijk((int)c, bs.n[0], bs.n[1], i, j, k);
  const int p[3] = {i, j, k};
  int bad = 0, asym = 0;
  for (int s = 0; s < bs.nent; ++s) {
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      const int q = p[d] + off_comp(bs.code[s], d);
      in = in && q >= 0 && q < bs.n[d];
    }
    double *a = bs.coef + (long long)s * bs.ncell + c;
    const double v = in ? *a : 0.0;
    if (!in) *a = 0.0;
    if (!isfinite(v)) bad = 1;
    if (s == bs.center && !(v > 0.0)) bad = 1;
    if (in && s != bs.center) {
      if (bs.mir[s] < 0) {
        asym = 1;
      } else {
        const double m = bs.coef[(long long)bs.mir[s] * bs.ncell + c + bs.lin[s]];
        if (!(fabs(v - m) <= 1e-12 * fmax(fabs(v), fabs(m)))) asym = 1;
      }
    }
  }
  if (bad) flag[0] = 1;
  if (asym) flag[1] = 1;
}

// c_d of Section 3.1 for each part: sum over cells of minus the off-diagonal
// coefficients with a nonzero d component, sign-adjusted by the center.
__global__ __launch_bounds__(kBlock) void k_wsum_partial(const PartDesc<double> *__restrict__ desc,
                                                         double *__restrict__ partial) {
  __shared__ double sh[3][kBlock];
  const PartDesc<double> &d = desc[blockIdx.y];
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < d.ncell;
       c += (long long)gridDim.x * kBlock) {
    const double ac = dev::G(d.coef)[(long long)d.center * d.ncell + c];
    const double sg = ac < 0.0 ? 1.0 : -1.0;
    for (int s = 0; s < d.nent; ++s) {
      if (s == d.center) continue;
      const double v = sg * dev::G(d.coef)[(long long)s * d.ncell + c];
      for (int q = 0; q < 3; ++q)
        if (off_comp(d.code[s], q) != 0) acc[q] += v;
    }
  }
  for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = acc[q];
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
  }
  __syncthreads();
  if (threadIdx.x < 3)
    partial[((long long)blockIdx.y * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_wsum_final(const double *__restrict__ partial, int nblk,
                                                       double *__restrict__ out) {
  __shared__ double sh[3][kBlock];
  const int p = blockIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kBlock)
    for (int q = 0; q < 3; ++q) acc[q] += partial[((long long)p * nblk + b) * 3 + q];
  for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = acc[q];
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
  }
  __syncthreads();
  if (threadIdx.x < 3) out[p * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

// Two-point collapse along d* for every F cell (odd index along d*):
//   den = sum of the coefficients with zero d* component,
//   wm = -(sum of those at -1)/den, wp = -(sum of those at +1)/den;
// a coarse neighbour outside the box is absent (weight 0); if it lies across a
// part face the opposite weight becomes 1 (Section 3.2), or, in the lumped
// reading, takes the dropped weight of the row's couplings on top.  Where den is not
// positive (the collapse is undefined; it happens on Galerkin operators of
// strongly heterogeneous problems) the two off-plane sums are normalised by
// their total so constants are interpolated, or 1/2 each if that total is not
// negative.
__global__ __launch_bounds__(kBlock) void k_interp_weights(const PartDesc<double> *__restrict__ desc,
                                                           const PartDesc<float> *__restrict__ desc32,
                                                           int *__restrict__ flag) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long fidx = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (d.dstar < 0 || fidx >= d.nf) return;
  const int ds = d.dstar;
  int g[3];
  cell_ijk((int)fidx, d.fn[0], d.fn[1], g[0], g[1], g[2]);
  int f[3] = {g[0], g[1], g[2]};
  f[ds] = 2 * g[ds] + 1;
  const long long c = f[0] + (long long)d.n[0] * (f[1] + (long long)d.n[1] * f[2]);
  // all coefficient loads first (entries past nent read entry 0 and are
  // skipped), then the sums in entry order
  double cv[kMaxEnt];
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) cv[s] = dev::G(d.coef)[(long long)(s < d.nent ? s : 0) * d.ncell + c];
  double den = 0.0, sm = 0.0, sp = 0.0;
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) {
    if (s >= d.nent) break;
    const double v = cv[s];
    const int o = off_comp(d.code[s], ds);
    if (o == 0)
      den += v;
    else if (o < 0)
      sm += v;
    else
      sp += v;
  }
  double wm, wp;
  if (den > 0.0) {
    wm = -sm / den;
    wp = -sp / den;
  } else if (sm + sp < 0.0) {
    // non-positive collapse denominator: normalise the two off-plane sums
    wm = sm / (sm + sp);
    wp = sp / (sm + sp);
  } else {
    wm = 0.5;
    wp = 0.5;
  }
  const bool hi_out = f[ds] + 1 > d.n[ds] - 1;   // lower corner 0: f-1 >= 0 always
  if (hi_out) {
    wp = 0.0;
    if ((d.faces >> (2 * ds + 1)) & 1) {
      if (d.pblump && den > 0.0) {
        // lumped reading: the dropped weight is the collapse of the row's
        // couplings, -(sum_j u_fj)/den, added to the opposite one.  The row
        // of cell c lies among the stored rows of its 256-cell block.
        const auto ub = dev::G(d.ublk[0]) + 2 * (c / kBlock);
        const int r0 = ub[0], r1 = ub[2];
        const int cell = (int)(d.off + c);
        double us = 0.0;
        for (int r = r0; r < r1; ++r) {
          if (dev::G(d.urow)[r] != cell) continue;
          for (int q = dev::G(d.uptr)[r]; q < dev::G(d.uptr)[r + 1]; ++q) us += dev::G(d.uval)[q];
          break;
        }
        wm = -(sm + us) / den;
      } else {
        wm = 1.0;
      }
    }
  }
  if (!isfinite(wm) || !isfinite(wp)) flag[0] = 1;
  dev::Gw(const_cast<double *>(d.wm))[fidx] = wm;
  dev::Gw(const_cast<double *>(d.wp))[fidx] = wp;
  if (desc32) {
    const PartDesc<float> &d32 = desc32[blockIdx.y];
    dev::Gw(const_cast<float *>(d32.wm))[fidx] = (float)wm;
    dev::Gw(const_cast<float *>(d32.wp))[fidx] = (float)wp;
  }
}

// Structured Galerkin product for one coarse cell I of a part coarsened along
// d*: fine rows f = 2I + r (r = -1, 0, 1) carry the restriction weights
// rho_{-1} = wp(2I-1), rho_0 = 1, rho_{+1} = wm(2I+1); each fine coefficient
// a_s(f) reaches fine cell g = f + s, which is coarse (weight 1) when
// q = r + s_d* is even and an F cell (weights wm(g), wp(g) toward its two
// coarse neighbours) when q is odd.  The host table lists, for each coarse
// entry, the (r, s, which-weight-of-g) triples that land on it.
//
// Two thread layouts form the same sums in the same order, so the same values.
// Small coarse levels: one thread per (coarse cell, coarse entry), so that
// even a few thousand coarse cells give enough threads; a block covers one
// entry of a tile of kBlock coarse cells, its threads read the same table rows
// and neighbouring fine coefficients, and each thread gathers its entry's
// contributions kRapEntryBatch at a time.  The blocks of one tile are
// consecutive in the XCD-aware block order, so they read the tile's fine
// coefficients through one XCD's L2.
constexpr int kRapEntryBatch = 4;

__global__ __launch_bounds__(kBlock) void k_rap_entry(const PartDesc<double> *__restrict__ desc,
                                                      const RapDesc *__restrict__ rd, int nent_max) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const RapDesc &t = rd[blockIdx.y];
  const int lb = dev::chunk_index();
  const int e = lb % nent_max;
  const long long cidx = (long long)(lb / nent_max) * kBlock + threadIdx.x;
  if (e >= t.nent || cidx >= d.cncell) return;
  if (d.dstar < 0) {
    // identity transfer: same operator, entries permuted into the sorted pattern
    const double v = dev::G(d.coef)[(long long)dev::G(t.code)[e] * d.ncell + cidx];
    dev::Gw(t.out)[(long long)e * d.cncell + cidx] = v;
    if (t.out32) dev::Gw(t.out32)[(long long)e * d.cncell + cidx] = (float)v;
    return;
  }
  const int ds = d.dstar;
  int ci[3];
  cell_ijk((int)cidx, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  const int nd = d.n[ds];
  const int fb = 2 * ci[ds];
  double rho[3];
  bool row_ok[3];
  {
    int g[3] = {ci[0], ci[1], ci[2]};
    row_ok[0] = fb - 1 >= 0;
    row_ok[1] = true;
    row_ok[2] = fb + 1 <= nd - 1;
    g[ds] = ci[ds] - 1;
    rho[0] = row_ok[0] ? dev::G(d.wp)[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])] : 0.0;
    rho[1] = 1.0;
    g[ds] = ci[ds];
    rho[2] = row_ok[2] ? dev::G(d.wm)[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])] : 0.0;
  }
  // Per-thread bases; every contribution then adds block-uniform offsets: the
  // fine row f = 2I + r is f0 + r*stride(d*), the neighbour g = f + s is in the
  // box when each coordinate is, and an odd g's F-box cell is h0 plus the
  // offsets of s (with (r + s_d* - 1)/2 along d*).
  int fc[3] = {ci[0], ci[1], ci[2]};
  fc[ds] = fb;
  const long long f0 = fc[0] + (long long)d.n[0] * (fc[1] + (long long)d.n[1] * fc[2]);
  const long long h0 = ci[0] + (long long)d.fn[0] * (ci[1] + (long long)d.fn[1] * ci[2]);
  const long long str[3] = {1, d.n[0], (long long)d.n[0] * d.n[1]};
  const long long fstr[3] = {1, d.fn[0], (long long)d.fn[0] * d.fn[1]};
  double acc = 0.0;
  const int q0 = dev::G(t.start)[e], q1 = dev::G(t.start)[e + 1];
  for (int qb = q0; qb < q1; qb += kRapEntryBatch) {
    double av[kRapEntryBatch], wv[kRapEntryBatch], rv[kRapEntryBatch];
#pragma unroll
    for (int u = 0; u < kRapEntryBatch; ++u) {
      const int q = qb + u;
      av[u] = 0.0;
      wv[u] = 1.0;
      rv[u] = 0.0;
      if (q >= q1) continue;
      const int w = dev::G(t.code)[q];
      const int r = (w & 3) - 1;
      const int sidx = (w >> 2) & 31;
      const int gsel = (w >> 7) & 3;
      const int cs = d.code[sidx];
      const int o[3] = {off_comp(cs, 0), off_comp(cs, 1), off_comp(cs, 2)};
      bool in = row_ok[r + 1] && (unsigned)(fb + r + o[ds]) < (unsigned)nd;
      long long dfine = r * str[ds], dh = ((r + o[ds] - 1) >> 1) * fstr[ds];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a == ds) continue;
        in = in && (unsigned)(ci[a] + o[a]) < (unsigned)d.n[a];
        dh += o[a] * fstr[a];
      }
      if (!in) continue;
      av[u] = dev::G(d.coef)[(long long)sidx * d.ncell + f0 + dfine];
      rv[u] = rho[r + 1];
      if (gsel != 0) wv[u] = gsel == 1 ? dev::G(d.wm)[h0 + dh] : dev::G(d.wp)[h0 + dh];
    }
#pragma unroll
    for (int u = 0; u < kRapEntryBatch; ++u) acc = fma(rv[u] * av[u], wv[u], acc);
  }
  dev::Gw(t.out)[(long long)e * d.cncell + cidx] = acc;
  if (t.out32) dev::Gw(t.out32)[(long long)e * d.cncell + cidx] = (float)acc;
}

// Large coarse levels: one thread per coarse cell and all coarse entries.  The
// per-cell work (coarse coordinates, restriction weights, fine and F-box bases)
// is done once, and the whole table (at most kRapMaxTab rows) is staged in LDS first with its
// block-uniform parts worked out (coefficient offset, F-box offset, row r,
// weight selector, neighbour offsets), so no thread waits on a table load
// before its gathers.  Each thread walks the table kRapBatch rows at a time
// with every load of a batch in flight before the sums, which keep the table
// order within each entry; an entry's sum is stored when the walk passes its
// last row.
constexpr int kRapBatch = 8;

__global__ __launch_bounds__(kBlock) void k_rap(const PartDesc<double> *__restrict__ desc,
                                                const RapDesc *__restrict__ rd) {
  __shared__ long long s_cof[kRapMaxTab], s_dh[kRapMaxTab];
  __shared__ int s_w[kRapMaxTab];
  __shared__ int s_start[kMaxEnt + 1];
  const PartDesc<double> &d = desc[blockIdx.y];
  const RapDesc &t = rd[blockIdx.y];
  const long long tile = (long long)dev::chunk_index() * kBlock;
  if (tile >= d.cncell) return;                      // block-uniform
  const long long cidx = tile + threadIdx.x;
  const bool valid = cidx < d.cncell;
  const auto coef = dev::G(d.coef);
  const auto out = dev::Gw(t.out);
  const auto out32 = dev::Gw(t.out32);
  const int nent = t.nent;
  if (d.dstar < 0) {
    // identity transfer: same operator, entries permuted into the sorted pattern
    if (!valid) return;
    for (int e = 0; e < nent; ++e) {
      const double v = coef[(long long)dev::G(t.code)[e] * d.ncell + cidx];
      out[(long long)e * d.cncell + cidx] = v;
      if (t.out32) out32[(long long)e * d.cncell + cidx] = (float)v;
    }
    return;
  }
  const int ds = d.dstar;
  const long long str[3] = {1, d.n[0], (long long)d.n[0] * d.n[1]};
  const long long fstr[3] = {1, d.fn[0], (long long)d.fn[0] * d.fn[1]};
  const int ntab = dev::G(t.start)[nent];
  for (int q = threadIdx.x; q < ntab; q += kBlock) {
    const int w = dev::G(t.code)[q];
    const int r = (w & 3) - 1;
    const int sidx = (w >> 2) & 31;
    const int gsel = (w >> 7) & 3;
    const int cs = d.code[sidx];
    long long dh = ((r + off_comp(cs, ds) - 1) >> 1) * fstr[ds];
    for (int a = 0; a < 3; ++a)
      if (a != ds) dh += off_comp(cs, a) * fstr[a];
    s_cof[q] = (long long)sidx * d.ncell + r * str[ds];
    s_dh[q] = dh;
    s_w[q] = (r + 1) | (gsel << 2) | ((cs & 63) << 4);
  }
  if ((int)threadIdx.x <= nent) s_start[threadIdx.x] = dev::G(t.start)[threadIdx.x];
  __syncthreads();
  if (!valid) return;
  int ci[3];
  cell_ijk((int)cidx, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  const int nd = d.n[ds];
  const int fb = 2 * ci[ds];
  const auto wm = dev::G(d.wm), wp = dev::G(d.wp);
  double rho[3];
  bool row_ok[3];
  {
    int g[3] = {ci[0], ci[1], ci[2]};
    row_ok[0] = fb - 1 >= 0;
    row_ok[1] = true;
    row_ok[2] = fb + 1 <= nd - 1;
    g[ds] = ci[ds] - 1;
    rho[0] = row_ok[0] ? wp[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])] : 0.0;
    rho[1] = 1.0;
    g[ds] = ci[ds];
    rho[2] = row_ok[2] ? wm[g[0] + d.fn[0] * (g[1] + d.fn[1] * g[2])] : 0.0;
  }
  // Per-thread bases; every row then adds block-uniform offsets: the fine row
  // f = 2I + r is f0 + r*stride(d*), the neighbour g = f + s is in the box when
  // each coordinate is, and an odd g's F-box cell is h0 plus the offsets of s
  // (with (r + s_d* - 1)/2 along d*).
  int fc[3] = {ci[0], ci[1], ci[2]};
  fc[ds] = fb;
  const long long f0 = fc[0] + (long long)d.n[0] * (fc[1] + (long long)d.n[1] * fc[2]);
  const long long h0 = ci[0] + (long long)d.fn[0] * (ci[1] + (long long)d.fn[1] * ci[2]);
  double acc = 0.0;
  int e = 0;
  int next = s_start[1];
  for (int qb = 0; qb < ntab; qb += kRapBatch) {
    double av[kRapBatch], wv[kRapBatch], rv[kRapBatch];
#pragma unroll
    for (int u = 0; u < kRapBatch; ++u) {
      const int q = qb + u;
      av[u] = 0.0;
      wv[u] = 1.0;
      rv[u] = 0.0;
      if (q >= ntab) continue;                       // block-uniform
      const int w = s_w[q];
      const int r = (w & 3) - 1, gsel = (w >> 2) & 3, cs = w >> 4;
      bool in = row_ok[r + 1] && (unsigned)(fb + r + off_comp(cs, ds)) < (unsigned)nd;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a != ds) in = in && (unsigned)(ci[a] + off_comp(cs, a)) < (unsigned)d.n[a];
      if (!in) continue;
      av[u] = coef[s_cof[q] + f0];
      rv[u] = rho[r + 1];
      if (gsel != 0) wv[u] = gsel == 1 ? wm[h0 + s_dh[q]] : wp[h0 + s_dh[q]];
    }
#pragma unroll
    for (int u = 0; u < kRapBatch; ++u) {
      const int q = qb + u;
      if (q >= ntab) break;                          // block-uniform
      while (q == next) {                            // entry e complete (block-uniform)
        out[(long long)e * d.cncell + cidx] = acc;
        if (t.out32) out32[(long long)e * d.cncell + cidx] = (float)acc;
        acc = 0.0;
        ++e;
        next = s_start[e + 1];
      }
      acc = fma(rv[u] * av[u], wv[u], acc);
    }
  }
  for (; e < nent; ++e) {                            // the last entry, and any empty ones after it
    out[(long long)e * d.cncell + cidx] = acc;
    if (t.out32) out32[(long long)e * d.cncell + cidx] = (float)acc;
    acc = 0.0;
  }
}

// Direct coarsest solve (Section 3.5 option): the coarsest operator A = S + U
// assembled densely in LDS and inverted in place by Gauss-Jordan elimination
// without pivoting (A is symmetric positive definite, so every pivot is
// positive; a pivot that is not sets flag 2).  One workgroup, n <= kDirectMax.
__global__ __launch_bounds__(kBlock) void k_direct_setup(const PartDesc<double> *__restrict__ desc, int np,
                                                         int n, int nrow, const int *__restrict__ urow,
                                                         const int *__restrict__ uptr,
                                                         const int *__restrict__ ucol,
                                                         const double *__restrict__ uval,
                                                         double *__restrict__ ainv, int *__restrict__ flag) {
  __shared__ double a[kDirectMax * kDirectMax];
  __shared__ double fcol[kDirectMax];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int i = tid; i < n * n; i += kBlock) a[i] = 0.0;
  __syncthreads();
  if (tid < n) {   // stencil part of row tid
    int p = 0;
    while (p + 1 < np && desc[p + 1].off <= tid) ++p;
    const PartDesc<double> &d = desc[p];
    const int cl = tid - (int)d.off;
    int c[3];
    cell_ijk(cl, d.n[0], d.n[1], c[0], c[1], c[2]);
    for (int s = 0; s < d.nent; ++s) {
      int g[3];
      bool in = true;
      for (int k = 0; k < 3; ++k) {
        g[k] = c[k] + off_comp(d.code[s], k);
        in = in && g[k] >= 0 && g[k] < d.n[k];
      }
      if (in)
        a[tid * n + (int)d.off + g[0] + d.n[0] * (g[1] + d.n[1] * g[2])] += d.coef[(long long)s * d.ncell + cl];
    }
  }
  __syncthreads();
  for (int r = tid; r < nrow; r += kBlock)   // couplings: one thread per stored row
    for (int q = uptr[r]; q < uptr[r + 1]; ++q) a[urow[r] * n + ucol[q]] += uval[q];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      piv = a[k * n + k];
      if (!(piv > 0.0) || !isfinite(piv)) flag[0] = 2;
    }
    if (tid < n) fcol[tid] = a[tid * n + k];
    __syncthreads();
    const double pv = piv;
    if (tid < n) a[k * n + tid] = (tid == k ? 1.0 : a[k * n + tid]) / pv;
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += kBlock) {
      const int i = idx / n, j = idx - i * n;
      if (i != k) a[idx] = (j == k ? 0.0 : a[idx]) - fcol[i] * a[k * n + j];
    }
    __syncthreads();
  }
  for (int i = tid; i < n * n; i += kBlock) ainv[i] = a[i];
}

// U_c = P^T U P on the host-built structure: each coarse entry sums, in a
// fixed order, w(a) * U[k] * w(b) over its contributions (w(-1) = 1).
__global__ __launch_bounds__(kBlock) void k_uc_numeric(long long nnz, const int *__restrict__ start,
                                                       const int *__restrict__ kk,
                                                       const int *__restrict__ ia,
                                                       const int *__restrict__ ib,
                                                       const double *__restrict__ uprev,
                                                       const double *__restrict__ w,
                                                       double *__restrict__ uval,
                                                       float *__restrict__ uval32) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  double acc = 0.0;
  const int q0 = start[e], q1 = start[e + 1];
  // four contributions at a time, every load issued before the sums (clamped
  // indices, masked afterwards), added in contribution order
  for (int q = q0; q < q1; q += 4) {
    int a[4], b[4], k[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int qq = min(q + t, q1 - 1);
      a[t] = ia[qq];
      b[t] = ib[qq];
      k[t] = kk[qq];
    }
    double wa[4], wb[4], u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double va = w[max(a[t], 0)], vb = w[max(b[t], 0)];
      wa[t] = a[t] < 0 ? 1.0 : va;
      wb[t] = b[t] < 0 ? 1.0 : vb;
      u[t] = uprev[k[t]];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (q + t < q1) acc = fma(wa[t] * u[t], wb[t], acc);
  }
  uval[e] = acc;
  if (uval32) uval32[e] = (float)acc;
}

// Weighted L1-Jacobi (Section 3.4): M_ii = sum_j |a_ij| over the whole row
// of A = S + U; the smoother factor of cell i is factor / M_ii.
// desc32 (finest level of a mixed-precision cycle, else null): the pass also
// writes the FP32 copy of the coefficients it reads.
__global__ __launch_bounds__(kBlock) void k_l1_cells(const PartDesc<double> *__restrict__ desc,
                                                     const PartDesc<float> *__restrict__ desc32,
                                                     double *__restrict__ l1) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.ncell) return;
  const auto cf = dev::G(d.coef);
  const auto c32 = desc32 ? dev::Gw(const_cast<float *>(desc32[blockIdx.y].coef)) : nullptr;
  double cv[kMaxEnt];   // all loads first, as in k_interp_weights
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) cv[s] = cf[(long long)(s < d.nent ? s : 0) * d.ncell + c];
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) {
    if (s >= d.nent) break;
    acc += fabs(cv[s]);
    if (desc32) c32[(long long)s * d.ncell + c] = (float)cv[s];
  }
  l1[d.off + c] = acc;
}

__global__ __launch_bounds__(kBlock) void k_l1_urows(int nrow, const int *__restrict__ urow,
                                                     const int *__restrict__ uptr,
                                                     const double *__restrict__ uval,
                                                     double *__restrict__ l1) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrow) return;
  double acc = 0.0;
  for (int q = uptr[r]; q < uptr[r + 1]; ++q) acc += fabs(uval[q]);
  l1[urow[r]] += acc;
}

__global__ __launch_bounds__(kBlock) void k_l1_finish(long long n, double factor,
                                                      double *__restrict__ rs,
                                                      float *__restrict__ rs32,
                                                      int *__restrict__ flag) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double m = rs[i];
  const double v = factor / m;
  if (!(m > 0.0) || !isfinite(v)) flag[0] = 1;
  rs[i] = v;
  if (rs32) rs32[i] = (float)v;
}

// Weighted Jacobi (eq:relax0, eq:relax1): the factor of cell i is omega_p / a_ii.
__global__ __launch_bounds__(kBlock) void k_jacobi_scale(const PartDesc<double> *__restrict__ desc,
                                                         double *__restrict__ rs,
                                                         float *__restrict__ rs32,
                                                         int *__restrict__ flag) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.ncell) return;
  const double a = dev::G(d.coef)[(long long)d.center * d.ncell + c];
  const double v = d.omega / a;
  if (!(a > 0.0) || !isfinite(v)) flag[0] = 1;
  rs[d.off + c] = v;
  if (rs32) rs32[d.off + c] = (float)v;
}

inline unsigned nblk(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

void launch_normalise(const BoxStencil &bs, int *flag, hipStream_t st) {
  if (bs.ncell > 0) k_normalise<<<nblk(bs.ncell), kBlock, 0, st>>>(bs, flag);
}

void launch_wsum(const PartDesc<double> *desc, int nparts, int maxcell, double *partial, double *out,
                 hipStream_t st) {
  long long nb = (maxcell + kBlock - 1) / kBlock;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  k_wsum_partial<<<dim3((unsigned)nb, nparts), kBlock, 0, st>>>(desc, partial);
  k_wsum_final<<<nparts, kBlock, 0, st>>>(partial, (int)nb, out);
}

void launch_interp_weights(const PartDesc<double> *desc, const PartDesc<float> *desc32, int nparts,
                           int maxf, int *flag, hipStream_t st) {
  k_interp_weights<<<dim3(nblk(maxf), nparts), kBlock, 0, st>>>(desc, desc32, flag);
}

void launch_smoother_scale(bool l1, const PartDesc<double> *desc, int nparts, int maxcell, int64_t n,
                           int nrow, const int *urow, const int *uptr, const double *uval,
                           double factor, double *rs, float *rs32, int *flag, hipStream_t st,
                           const PartDesc<float> *cast32) {
  if (l1) {
    k_l1_cells<<<dim3(nblk(maxcell), nparts), kBlock, 0, st>>>(desc, cast32, rs);
    if (nrow > 0) k_l1_urows<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, uval, rs);
    k_l1_finish<<<nblk(n), kBlock, 0, st>>>(n, factor, rs, rs32, flag);
  } else {
    k_jacobi_scale<<<dim3(nblk(maxcell), nparts), kBlock, 0, st>>>(desc, rs, rs32, flag);
  }
}

void launch_rap(const PartDesc<double> *desc, const RapDesc *rd, int nparts, int maxcoarse,
                int maxent_c, int64_t cell_min, hipStream_t st) {
  if ((int64_t)maxcoarse * nparts >= cell_min) {
    k_rap<<<dim3(nblk(maxcoarse), nparts), kBlock, 0, st>>>(desc, rd);
  } else {
    // tiles x entries, rounded up to a multiple of 8 so that the XCD-aware order applies
    const unsigned nb = (nblk(maxcoarse) * (unsigned)maxent_c + 7u) & ~7u;
    k_rap_entry<<<dim3(nb, nparts), kBlock, 0, st>>>(desc, rd, maxent_c);
  }
}

void launch_direct_setup(const PartDesc<double> *desc, int np, int n, int nrow, const int *urow,
                         const int *uptr, const int *ucol, const double *uval, double *ainv, int *flag,
                         hipStream_t st) {
  k_direct_setup<<<1, kBlock, 0, st>>>(desc, np, n, nrow, urow, uptr, ucol, uval, ainv, flag);
}

void launch_uc_numeric(int64_t nnz, const int *start, const int *k, const int *a, const int *b,
                       const double *uprev, const double *w, double *uval, float *uval32,
                       hipStream_t st) {
  if (nnz > 0) k_uc_numeric<<<nblk(nnz), kBlock, 0, st>>>(nnz, start, k, a, b, uprev, w, uval, uval32);
}

}  // namespace ssamg
