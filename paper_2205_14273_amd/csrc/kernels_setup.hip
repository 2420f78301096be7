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
// weights from the collapse sums (den: zero d* component, sm / sp: -1 / +1)
__device__ __forceinline__ void collapse_weights(double den, double sm, double sp, double &wm, double &wp) {
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
}

__global__ __launch_bounds__(kBlock) void k_interp_weights(const PartDesc<double> *__restrict__ desc,
                                                           const PartDesc<float> *__restrict__ desc32,
                                                           int *__restrict__ flag) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long fidx = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (d.dstar < 0 || d.wfused || fidx >= d.nf) return;
  const int ds = d.dstar;
  int g[3];
  cell_ijk((int)fidx, d.fn[0], d.fn[1], g[0], g[1], g[2]);
  int f[3] = {g[0], g[1], g[2]};
  f[ds] = 2 * g[ds] + 1;
  const long long c = f[0] + (long long)d.n[0] * (f[1] + (long long)d.n[1] * f[2]);
  double den = 0.0, sm = 0.0, sp = 0.0;
  if (d.csum) {
    // formed by the assembly in the same order
    const auto cs = dev::G(d.csum);
    den = cs[fidx];
    sm = cs[d.nf + fidx];
    sp = cs[2 * d.nf + fidx];
  } else {
    // all coefficient loads first (in summation order; slots past nent read
    // the first entry and are skipped), then the sums
    double cv[kMaxEnt];
#pragma unroll
    for (int s = 0; s < kMaxEnt; ++s)
      cv[s] = dev::G(d.coef)[(long long)d.wsum[s < d.nent ? s : 0] * d.ncell + c];
#pragma unroll
    for (int s = 0; s < kMaxEnt; ++s) {
      if (s >= d.nent) break;
      const double v = cv[s];
      const int o = off_comp(d.code[d.wsum[s]], ds);
      if (o == 0)
        den += v;
      else if (o < 0)
        sm += v;
      else
        sp += v;
    }
  }
  double wm, wp;
  collapse_weights(den, sm, sp, wm, wp);
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

// Structured Galerkin product P^T S P (Section 3.3, eq:galerkin), factorised
// along d*.  Coarse cell I of a part coarsened along d* has the fine rows
// f_r = 2I + r (r = -1, 0, 1) with restriction weights rho_{-1} = wp(2I-1),
// rho_0 = 1, rho_{+1} = wm(2I+1).  Write a stencil offset as (t, s) with t its
// two components across d* and s its d* component.  The coefficient a_(t,s)(f_r)
// reaches the fine cell at d* offset q = r + s from 2I, so for each t the sums
//   B_t(q) = sum_r rho_r a_(t, q-r)(f_r),   q = -2 .. 2,   (r ascending)
// collect everything that lands there.  An even q is a coarse cell (weight 1)
// at coarse offset q/2; an odd q is an F cell whose weights wm, wp carry it to
// the coarse offsets (q-1)/2 and (q+1)/2.  Hence the coarse entry
//   c_(t,Q)(I) = B_t(2Q) + B_t(2Q-1) wp(F_{2Q-1}) + B_t(2Q+1) wm(F_{2Q+1}),
// with every term whose fine or F cell lies outside the box left out.  Each of
// the 3 x 27 fine coefficients is read once per coarse cell and each F weight
// once per perpendicular offset.
//
// Two thread layouts evaluate the same expressions with the same operations:
// one thread per coarse cell for large levels (all entries; it also reads every
// coefficient of rows 2I and 2I+1, so it forms their L1 row sums and the FP32
// copy of the finest level on the way), one thread per (coarse cell, entry)
// for small ones.  The results agree bit for bit.

__host__ __device__ constexpr int cube_stride(int a) { return a == 0 ? 1 : a == 1 ? 3 : 9; }

__device__ __forceinline__ int cube_comp(int o, int a) {
  return (a == 0 ? o % 3 : a == 1 ? (o / 3) % 3 : o / 9) - 1;
}

// B_t(q) from the three rows' coefficients a[r+1][s+1] (pres[s+1]: the fine
// stencil has the offset (t, s))
__device__ __forceinline__ double rap_b(int q, const double (&a)[3][3], const bool (&pres)[3],
                                        const double (&rho)[3]) {
  double b = 0.0;
#pragma unroll
  for (int r = -1; r <= 1; ++r) {
    const int sd = q - r;
    if (sd < -1 || sd > 1 || !pres[sd + 1]) continue;
    b = fma(rho[r + 1], a[r + 1][sd + 1], b);
  }
  return b;
}

// c_(t,Q) from B_t(2Q) (ve: its cell is in the box) and the F cells below
// (vl, weight wl) and above (vh, weight wh)
__device__ __forceinline__ double rap_combine(bool ve, double be, bool vl, double bl, double wl, bool vh,
                                              double bh, double wh) {
  double acc = ve ? be : 0.0;
  acc = fma(vl ? bl : 0.0, wl, acc);
  acc = fma(vh ? bh : 0.0, wh, acc);
  return acc;
}

// per coarse cell: coordinates, the fine rows (clamped into the box; a row
// outside has rho = 0), restriction weights and the F-box cell of index
// (I across d*, I along d*)
struct RapGeo {
  int ci[3];
  int fb, nd;
  bool row_ok[3];
  double rho[3];
  long long fr[3];
  long long h0;
};

template <int DS>
__device__ __forceinline__ void rap_geo(const PartDesc<double> &d, long long cidx, RapGeo &g) {
  cell_ijk((int)cidx, d.cn[0], d.cn[1], g.ci[0], g.ci[1], g.ci[2]);
  g.nd = d.n[DS];
  g.fb = 2 * g.ci[DS];
  g.row_ok[0] = g.fb >= 1;
  g.row_ok[1] = true;
  g.row_ok[2] = g.fb + 1 <= g.nd - 1;
  const long long strd = DS == 0 ? 1 : DS == 1 ? (long long)d.n[0] : (long long)d.n[0] * d.n[1];
  const long long fstrd = DS == 0 ? 1 : DS == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
  int fc[3] = {g.ci[0], g.ci[1], g.ci[2]};
  fc[DS] = g.fb;
  const long long f0 = fc[0] + (long long)d.n[0] * (fc[1] + (long long)d.n[1] * fc[2]);
  g.fr[0] = g.row_ok[0] ? f0 - strd : f0;
  g.fr[1] = f0;
  g.fr[2] = g.row_ok[2] ? f0 + strd : f0;
  g.h0 = g.ci[0] + (long long)d.fn[0] * (g.ci[1] + (long long)d.fn[1] * g.ci[2]);
  g.rho[0] = g.row_ok[0] ? dev::G(d.wp)[g.h0 - fstrd] : 0.0;
  g.rho[1] = 1.0;
  g.rho[2] = g.row_ok[2] ? dev::G(d.wm)[g.h0] : 0.0;
}

template <int DS>
__device__ __forceinline__ long long fstride(const PartDesc<double> &d) {
  return DS == 0 ? 1 : DS == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
}

// the three rows' coefficients of perpendicular offset (ta, tb)
template <int DS>
__device__ __forceinline__ void rap_rows(const PartDesc<double> &d, const RapDesc &t, const RapGeo &g,
                                         int ob, double (&a)[3][3], bool (&pres)[3], int (&ent)[3]) {
  const auto coef = dev::G(d.coef);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    ent[s] = t.fmap[ob + s * cube_stride(DS)];
    pres[s] = ent[s] >= 0;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 3; ++s)
      a[r][s] = pres[s] ? coef[(long long)ent[s] * d.ncell + g.fr[r]] : 0.0;
}

// one coarse cell, every entry
template <int DS>
__device__ __forceinline__ void rap_cell(const PartDesc<double> &d, const RapDesc &t, long long cidx) {
  constexpr int AX = (DS + 1) % 3, BX = (DS + 2) % 3;
  RapGeo g;
  rap_geo<DS>(d, cidx, g);
  const auto wm = dev::G(d.wm), wp = dev::G(d.wp);
  const auto out = dev::Gw(t.out);
  const auto out32 = dev::Gw(t.out32);
  const auto f32 = dev::Gw(t.fine32);
  const long long fa = AX == 0 ? 1 : AX == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
  const long long fbx = BX == 0 ? 1 : BX == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
  const long long fd = fstride<DS>(d);
  const bool okm = g.row_ok[0], okp = g.row_ok[2];
  const bool ok2m = g.fb - 2 >= 0, ok2p = g.fb + 2 <= g.nd - 1;
  double l1c = 0.0, l1f = 0.0;
  double wden = 0.0, wsm = 0.0, wsp = 0.0;
#pragma unroll
  for (int tb = -1; tb <= 1; ++tb) {
#pragma unroll
    for (int ta = -1; ta <= 1; ++ta) {
      const int ob = (ta + 1) * cube_stride(AX) + (tb + 1) * cube_stride(BX);
      double a[3][3];
      bool pres[3];
      int ent[3];
      rap_rows<DS>(d, t, g, ob, a, pres, ent);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (!pres[s]) continue;
        l1c += fabs(a[1][s]);
        l1f += fabs(a[2][s]);
        if (t.fine32) {
          f32[(long long)ent[s] * d.ncell + g.fr[1]] = (float)a[1][s];
          if (okp) f32[(long long)ent[s] * d.ncell + g.fr[2]] = (float)a[2][s];
        }
      }
      const bool perp = (unsigned)(g.ci[AX] + ta) < (unsigned)d.n[AX] &&
                        (unsigned)(g.ci[BX] + tb) < (unsigned)d.n[BX];
      const long long tl = ta * fa + tb * fbx;
      const bool vm = perp && okm, vp = perp && okp;
      const long long gm = vm ? g.h0 - fd + tl : 0, gp = vp ? g.h0 + tl : 0;
      const double wmm = wm[gm], wpm = wp[gm], wmp = wm[gp], wpp = wp[gp];
      const double bm1 = rap_b(-1, a, pres, g.rho), bp1 = rap_b(1, a, pres, g.rho);
      double v[3];
      v[0] = rap_combine(perp && ok2m, rap_b(-2, a, pres, g.rho), false, 0.0, 0.0, vm, bm1, wmm);
      v[1] = rap_combine(perp, rap_b(0, a, pres, g.rho), vm, bm1, wpm, vp, bp1, wmp);
      v[2] = rap_combine(perp && ok2p, rap_b(2, a, pres, g.rho), vp, bp1, wpp, false, 0.0, 0.0);
#pragma unroll
      for (int Q = 0; Q < 3; ++Q) {
        const int e = t.cmap[ob + Q * cube_stride(DS)];
        if (e < 0) continue;
        out[(long long)e * d.cncell + cidx] = v[Q];
        if (t.out32) out32[(long long)e * d.cncell + cidx] = (float)v[Q];
        // the coarse row's collapse sums along its own direction, in the
        // order of formation (the order of the descriptor's wsum)
        const int comp = t.wdir == DS ? Q - 1 : t.wdir == AX ? ta : tb;
        if (comp == 0)
          wden += v[Q];
        else if (comp < 0)
          wsm += v[Q];
        else
          wsp += v[Q];
      }
    }
  }
  if (t.l1) {
    const auto l1 = dev::Gw(t.l1);
    l1[g.fr[1]] = l1c;
    if (okp) l1[g.fr[2]] = l1f;
  }
  // the coarse cell's own interpolation weights if it is an F cell of its level
  // (selects, not a runtime index into the coordinate registers)
  const int wd = t.wdir;
  const int cw = wd == 0 ? g.ci[0] : wd == 1 ? g.ci[1] : g.ci[2];
  if (wd >= 0 && (cw & 1)) {
    const int f0 = wd == 0 ? (cw - 1) >> 1 : g.ci[0];
    const int f1 = wd == 1 ? (cw - 1) >> 1 : g.ci[1];
    const int f2 = wd == 2 ? (cw - 1) >> 1 : g.ci[2];
    const long long fidx = f0 + (long long)t.wfn[0] * (f1 + (long long)t.wfn[1] * f2);
    double wmv, wpv;
    collapse_weights(wden, wsm, wsp, wmv, wpv);
    if (cw + 1 > d.cn[wd] - 1) {
      wpv = 0.0;
      if ((t.wfaces >> (2 * wd + 1)) & 1) wmv = 1.0;
    }
    if (!isfinite(wmv) || !isfinite(wpv)) t.wflag[0] = 1;
    dev::Gw(t.wm)[fidx] = wmv;
    dev::Gw(t.wp)[fidx] = wpv;
    if (t.wm32) {
      dev::Gw(t.wm32)[fidx] = (float)wmv;
      dev::Gw(t.wp32)[fidx] = (float)wpv;
    }
  }
}

// one coarse cell, one entry (cube offset o)
template <int DS>
__device__ __forceinline__ double rap_entry_value(const PartDesc<double> &d, const RapDesc &t, long long cidx,
                                                  int o) {
  constexpr int AX = (DS + 1) % 3, BX = (DS + 2) % 3;
  RapGeo g;
  rap_geo<DS>(d, cidx, g);
  const int ta = cube_comp(o, AX), tb = cube_comp(o, BX), Q = cube_comp(o, DS);
  const int ob = (ta + 1) * cube_stride(AX) + (tb + 1) * cube_stride(BX);
  double a[3][3];
  bool pres[3];
  int ent[3];
  rap_rows<DS>(d, t, g, ob, a, pres, ent);
  const long long fa = AX == 0 ? 1 : AX == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
  const long long fbx = BX == 0 ? 1 : BX == 1 ? (long long)d.fn[0] : (long long)d.fn[0] * d.fn[1];
  const bool perp = (unsigned)(g.ci[AX] + ta) < (unsigned)d.n[AX] &&
                    (unsigned)(g.ci[BX] + tb) < (unsigned)d.n[BX];
  const long long tl = ta * fa + tb * fbx;
  const bool vm = perp && g.row_ok[0], vp = perp && g.row_ok[2];
  const long long gm = vm ? g.h0 - fstride<DS>(d) + tl : 0, gp = vp ? g.h0 + tl : 0;
  const auto wm = dev::G(d.wm), wp = dev::G(d.wp);
  if (Q < 0)
    return rap_combine(perp && g.fb - 2 >= 0, rap_b(-2, a, pres, g.rho), false, 0.0, 0.0, vm,
                       rap_b(-1, a, pres, g.rho), wm[gm]);
  if (Q == 0)
    return rap_combine(perp, rap_b(0, a, pres, g.rho), vm, rap_b(-1, a, pres, g.rho), wp[gm], vp,
                       rap_b(1, a, pres, g.rho), wm[gp]);
  return rap_combine(perp && g.fb + 2 <= g.nd - 1, rap_b(2, a, pres, g.rho), vp, rap_b(1, a, pres, g.rho),
                     wp[gp], false, 0.0, 0.0);
}

// Non-Galerkin coarse stencil of a star part (SSAMG_COARSE_OP_NONGALERKIN;
// Section 5 plans it for isotropic problems).  From the Galerkin entries G,
// each entry of offset (t, Q) with t != 0 across d* and Q != 0 along d* is
// replaced by its rectangle's four sides (I, I+t), (I, I+Q), (I+t, J),
// (I+Q, J) at half its value, and the diagonals of I+t and I+Q lose half of
// it (row sums kept).  Gathered per coarse entry of cell I, over the four
// unit offsets t across d* and Q = -1, 1:
//   C_(t,0)(I) = G_(t,0)(I) + 1/2 sum_Q [G_(t,Q)(I) + G_(t,Q)(I - Q)]
//   C_(0,Q)(I) = G_(0,Q)(I) + 1/2 sum_t [G_(t,Q)(I) + G_(t,Q)(I - t)]
//   C_0(I)     = G_0(I)     - 1/2 sum_t sum_Q [G_(t,Q)(I - t) + G_(t,Q)(I - Q)]
// with the terms of cells outside the coarse box left out.
// Galerkin entry of offset (ua, ub across d*, q along d*) at coarse cell
// ci - (sa, sb, sd); 0 if that cell is outside the coarse box
template <int DS>
__device__ __forceinline__ double ng_g(const PartDesc<double> &d, const RapDesc &t, const int (&ci)[3], int ua,
                                       int ub, int q, int sa, int sb, int sd) {
  constexpr int AX = (DS + 1) % 3, BX = (DS + 2) % 3;
  int c[3] = {ci[0], ci[1], ci[2]};
  c[AX] -= sa;
  c[BX] -= sb;
  c[DS] -= sd;
  if ((unsigned)c[0] >= (unsigned)d.cn[0] || (unsigned)c[1] >= (unsigned)d.cn[1] ||
      (unsigned)c[2] >= (unsigned)d.cn[2])
    return 0.0;
  const long long cc = c[0] + (long long)d.cn[0] * (c[1] + (long long)d.cn[1] * c[2]);
  return rap_entry_value<DS>(d, t, cc,
                             (ua + 1) * cube_stride(AX) + (ub + 1) * cube_stride(BX) + (q + 1) * cube_stride(DS));
}

// the four unit offsets across d* (components along AX, BX), in summation order
__constant__ const int kNgT[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};

template <int DS>
__device__ __forceinline__ double rap_ng_value(const PartDesc<double> &d, const RapDesc &t, long long cidx,
                                               int o) {
  constexpr int AX = (DS + 1) % 3, BX = (DS + 2) % 3;
  int ci[3];
  cell_ijk((int)cidx, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  const int ta = cube_comp(o, AX), tb = cube_comp(o, BX), Q = cube_comp(o, DS);
  double sum = 0.0;
  if (ta == 0 && tb == 0 && Q == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = -1; q <= 1; q += 2) {
        sum += ng_g<DS>(d, t, ci, kNgT[k][0], kNgT[k][1], q, kNgT[k][0], kNgT[k][1], 0);
        sum += ng_g<DS>(d, t, ci, kNgT[k][0], kNgT[k][1], q, 0, 0, q);
      }
    return ng_g<DS>(d, t, ci, 0, 0, 0, 0, 0, 0) - 0.5 * sum;
  }
  if (ta == 0 && tb == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sum += ng_g<DS>(d, t, ci, kNgT[k][0], kNgT[k][1], Q, 0, 0, 0);
      sum += ng_g<DS>(d, t, ci, kNgT[k][0], kNgT[k][1], Q, kNgT[k][0], kNgT[k][1], 0);
    }
    return ng_g<DS>(d, t, ci, 0, 0, Q, 0, 0, 0) + 0.5 * sum;
  }
#pragma unroll
  for (int q = -1; q <= 1; q += 2) {
    sum += ng_g<DS>(d, t, ci, ta, tb, q, 0, 0, 0);
    sum += ng_g<DS>(d, t, ci, ta, tb, q, 0, 0, q);
  }
  return ng_g<DS>(d, t, ci, ta, tb, 0, 0, 0, 0) + 0.5 * sum;
}

// one coarse cell of a non-Galerkin part, every entry: each of the 31
// Galerkin values once, combined in rap_ng_value's order (so the same bits);
// then the L1 row sums and FP32 copy of rows 2I and 2I+1 in entry order
template <int DS>
__device__ __forceinline__ void rap_cell_ng(const PartDesc<double> &d, const RapDesc &t, long long cidx) {
  constexpr int AX = (DS + 1) % 3, BX = (DS + 2) % 3;
  int ci[3];
  cell_ijk((int)cidx, d.cn[0], d.cn[1], ci[0], ci[1], ci[2]);
  double own[4][2], sht[4][2], shq[4][2], gt0[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ua = kNgT[k][0], ub = kNgT[k][1];
    gt0[k] = ng_g<DS>(d, t, ci, ua, ub, 0, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int q = 2 * j - 1;
      own[k][j] = ng_g<DS>(d, t, ci, ua, ub, q, 0, 0, 0);
      sht[k][j] = ng_g<DS>(d, t, ci, ua, ub, q, ua, ub, 0);
      shq[k][j] = ng_g<DS>(d, t, ci, ua, ub, q, 0, 0, q);
    }
  }
  const double g0 = ng_g<DS>(d, t, ci, 0, 0, 0, 0, 0, 0);
  // the coarse pattern is the star: every entry is one of the seven below
  auto put = [&](int o, double v) {
    const int e = t.cmap[o];
    if (e < 0) return;
    dev::Gw(t.out)[(long long)e * d.cncell + cidx] = v;
    if (t.out32) dev::Gw(t.out32)[(long long)e * d.cncell + cidx] = (float)v;
  };
  {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        sum += sht[k][j];
        sum += shq[k][j];
      }
    put(13, g0 - 0.5 * sum);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sum += own[k][j];
      sum += sht[k][j];
    }
    put(13 + (2 * j - 1) * cube_stride(DS), ng_g<DS>(d, t, ci, 0, 0, 2 * j - 1, 0, 0, 0) + 0.5 * sum);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      sum += own[k][j];
      sum += shq[k][j];
    }
    put(13 + kNgT[k][0] * cube_stride(AX) + kNgT[k][1] * cube_stride(BX), gt0[k] + 0.5 * sum);
  }
  if (!t.l1 && !t.fine32) return;
  RapGeo g;
  rap_geo<DS>(d, cidx, g);
  const bool okp = g.row_ok[2];
  double l1c = 0.0, l1f = 0.0;
  for (int e = 0; e < d.nent; ++e) {
    const double a0 = dev::G(d.coef)[(long long)e * d.ncell + g.fr[1]];
    const double a1 = dev::G(d.coef)[(long long)e * d.ncell + g.fr[2]];
    l1c += fabs(a0);
    l1f += fabs(a1);
    if (t.fine32) {
      dev::Gw(t.fine32)[(long long)e * d.ncell + g.fr[1]] = (float)a0;
      if (okp) dev::Gw(t.fine32)[(long long)e * d.ncell + g.fr[2]] = (float)a1;
    }
  }
  if (t.l1) {
    dev::Gw(t.l1)[g.fr[1]] = l1c;
    if (okp) dev::Gw(t.l1)[g.fr[2]] = l1f;
  }
}

// Small coarse levels: one thread per (coarse cell, coarse entry); a block
// covers one entry of a tile of kBlock coarse cells, and the blocks of one
// tile are consecutive in the XCD-aware order, so they read the tile's fine
// coefficients through one XCD's L2.
__global__ __launch_bounds__(kBlock) void k_rap_entry(const PartDesc<double> *__restrict__ desc,
                                                      const RapDesc *__restrict__ rd, int nent_max) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const RapDesc &t = rd[blockIdx.y];
  const int lb = dev::chunk_index();
  const int e = lb % nent_max;
  const long long cidx = (long long)(lb / nent_max) * kBlock + threadIdx.x;
  if (e >= t.nent || cidx >= d.cncell) return;
  const int o = t.cofs[e];
  double v;
  switch (d.dstar + (t.ng ? 3 : 0)) {
    case 0: v = rap_entry_value<0>(d, t, cidx, o); break;
    case 1: v = rap_entry_value<1>(d, t, cidx, o); break;
    case 2: v = rap_entry_value<2>(d, t, cidx, o); break;
    case 3: v = rap_ng_value<0>(d, t, cidx, o); break;
    case 4: v = rap_ng_value<1>(d, t, cidx, o); break;
    case 5: v = rap_ng_value<2>(d, t, cidx, o); break;
    default:   // identity transfer: the same operator, entries in the coarse order
      v = dev::G(d.coef)[(long long)t.fmap[o] * d.ncell + cidx];
  }
  dev::Gw(t.out)[(long long)e * d.cncell + cidx] = v;
  if (t.out32) dev::Gw(t.out32)[(long long)e * d.cncell + cidx] = (float)v;
}

// Large coarse levels: one thread per coarse cell.
__global__ __launch_bounds__(kBlock) void k_rap(const PartDesc<double> *__restrict__ desc,
                                                const RapDesc *__restrict__ rd) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const RapDesc &t = rd[blockIdx.y];
  const long long cidx = (long long)dev::chunk_index() * kBlock + threadIdx.x;
  if (cidx >= d.cncell) return;
  if (t.ng) return;                                   // k_rap_ng's parts
  switch (d.dstar) {
    case 0: rap_cell<0>(d, t, cidx); break;
    case 1: rap_cell<1>(d, t, cidx); break;
    case 2: rap_cell<2>(d, t, cidx); break;
    default: {   // identity transfer
      double l1 = 0.0;
      for (int e = 0; e < t.nent; ++e) {
        const int fe = t.fmap[t.cofs[e]];
        const double v = dev::G(d.coef)[(long long)fe * d.ncell + cidx];
        dev::Gw(t.out)[(long long)e * d.cncell + cidx] = v;
        if (t.out32) dev::Gw(t.out32)[(long long)e * d.cncell + cidx] = (float)v;
        if (t.fine32) dev::Gw(t.fine32)[(long long)fe * d.ncell + cidx] = (float)v;
        l1 += fabs(v);
      }
      if (t.l1) dev::Gw(t.l1)[cidx] = l1;
    }
  }
}

// The non-Galerkin parts of a large level (a kernel of its own: its register
// demand would otherwise lower the occupancy of k_rap)
__global__ __launch_bounds__(kBlock) void k_rap_ng(const PartDesc<double> *__restrict__ desc,
                                                   const RapDesc *__restrict__ rd) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const RapDesc &t = rd[blockIdx.y];
  const long long cidx = (long long)dev::chunk_index() * kBlock + threadIdx.x;
  if (!t.ng || cidx >= d.cncell) return;
  switch (d.dstar) {
    case 0: rap_cell_ng<0>(d, t, cidx); break;
    case 1: rap_cell_ng<1>(d, t, cidx); break;
    default: rap_cell_ng<2>(d, t, cidx); break;
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
// The weighted L1-Jacobi factor of a part's cells in one pass, on levels
// whose stencil sums no Galerkin kernel has formed (small levels: one launch
// instead of three): the stencil sum in entry order (with the FP32 copy when
// desc32 is given) plus the sum of |u| over the cell's coupling row in entry
// order (found among the stored rows of its 256-cell block), then factor /
// sum.  On large levels the per-cell searches cost more than the launches
// they save, so there the rows add their sums in a row-parallel pass.
__global__ __launch_bounds__(kBlock) void k_l1_fused(const PartDesc<double> *__restrict__ desc,
                                                     const PartDesc<float> *__restrict__ desc32, double factor,
                                                     double *__restrict__ rs, float *__restrict__ rs32,
                                                     int *__restrict__ flag) {
  const PartDesc<double> &d = desc[blockIdx.y];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.ncell) return;
  const auto cf = dev::G(d.coef);
  const auto c32 = desc32 ? dev::Gw(const_cast<float *>(desc32[blockIdx.y].coef)) : nullptr;
  double cv[kMaxEnt];
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) cv[s] = cf[(long long)(s < d.nent ? s : 0) * d.ncell + c];
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < kMaxEnt; ++s) {
    if (s >= d.nent) break;
    acc += fabs(cv[s]);
    if (desc32) c32[(long long)s * d.ncell + c] = (float)cv[s];
  }
  if (d.urow) {
    // the block's stored rows are ascending: binary search for the cell's
    const auto ub = dev::G(d.ublk[0]) + 2 * (c / kBlock);
    int lo = ub[0], hi = ub[2];
    const int cell = (int)(d.off + c);
    const auto urow = dev::G(d.urow);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (urow[mid] < cell)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < ub[2] && urow[lo] == cell) {
      double us = 0.0;
      for (int q = dev::G(d.uptr)[lo]; q < dev::G(d.uptr)[lo + 1]; ++q) us += fabs(dev::G(d.uval)[q]);
      acc += us;
    }
  }
  const double v = factor / acc;
  if (!(acc > 0.0) || !isfinite(v)) flag[0] = 1;
  rs[d.off + c] = v;
  if (rs32) rs32[d.off + c] = (float)v;
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

void launch_wsum_final(const double *partial, int nparts, int nblk, double *out, hipStream_t st) {
  k_wsum_final<<<nparts, kBlock, 0, st>>>(partial, nblk, out);
}

void launch_interp_weights(const PartDesc<double> *desc, const PartDesc<float> *desc32, int nparts,
                           int maxf, int *flag, hipStream_t st) {
  k_interp_weights<<<dim3(nblk(maxf), nparts), kBlock, 0, st>>>(desc, desc32, flag);
}

void launch_smoother_scale(bool l1, const PartDesc<double> *desc, int nparts, int maxcell, int64_t n,
                           int nrow, const int *urow, const int *uptr, const double *uval,
                           double factor, double *rs, float *rs32, int *flag, hipStream_t st,
                           const PartDesc<float> *cast32, bool stencil_sums_done) {
  if (l1 && !stencil_sums_done) {
    k_l1_fused<<<dim3(nblk(maxcell), nparts), kBlock, 0, st>>>(desc, cast32, factor, rs, rs32, flag);
  } else if (l1) {
    // the per-cell Galerkin kernel has written the stencil sums into rs
    if (nrow > 0) k_l1_urows<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, uval, rs);
    k_l1_finish<<<nblk(n), kBlock, 0, st>>>(n, factor, rs, rs32, flag);
  } else {
    k_jacobi_scale<<<dim3(nblk(maxcell), nparts), kBlock, 0, st>>>(desc, rs, rs32, flag);
  }
}

bool rap_per_cell(int nparts, int maxcoarse, int64_t cell_min) {
  return (int64_t)maxcoarse * nparts >= cell_min;
}

void launch_rap(const PartDesc<double> *desc, const RapDesc *rd, int nparts, int maxcoarse,
                int maxent_c, int64_t cell_min, bool any_ng, hipStream_t st) {
  if (rap_per_cell(nparts, maxcoarse, cell_min)) {
    // 8-aligned grid so that the XCD-aware block order applies
    const dim3 grid((nblk(maxcoarse) + 7u) & ~7u, nparts);
    k_rap<<<grid, kBlock, 0, st>>>(desc, rd);
    if (any_ng) k_rap_ng<<<grid, kBlock, 0, st>>>(desc, rd);
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
