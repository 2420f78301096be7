// Finite-volume diffusion operator of the synthetic workloads and its adjoint
// gradient (gfx950).
//
// For a link from cell i to its neighbour j at stencil offset s:
//   t_ij = g_s * H(a_{p(i),s} kappa_i, a_{p(j),s} kappa_j),  H(x,y) = 2xy/(x+y),
//   g_s = 1 / 2^(nnz(s)-1), a_{p,s} = mean of part p's directional factors over
//   the nonzero components of s.  A neighbour outside every part is a ghost
//   with kappa_j = kappa_i (t = g_s a_{p(i),s} kappa_i, diagonal only).
//   A_ii = sum of t over the links of i, A_ij = -t_ij; same-part entries are the
//   stencil S, cross-part entries the couplings U.
// Gradient of L(x): dL/dkappa_c = -lambda^T (dA/dkappa_c) x with A lambda = dL/dx,
//   i.e. minus the sum over the links of c of dt/dkappa_c times
//   (lambda_c - lambda_j)(x_c - x_j), or lambda_c x_c for a ghost link.  With
//   several right-hand sides (x and lambda [cell][nrhs]) the loss is the sum
//   over the columns, and so is each link's factor.
#include "device_util.h"
#include "ssamg_impl.h"

namespace ssamg {

namespace {

__device__ __forceinline__ int oc(int code, int d) { return ((code >> (2 * d)) & 3) - 1; }

__device__ __forceinline__ double link_factor(const double *aniso, int p, int code) {
  double sum = 0.0;
  int cnt = 0;
  for (int d = 0; d < 3; ++d)
    if (oc(code, d) != 0) {
      sum += aniso[3 * p + d];
      ++cnt;
    }
  return sum / cnt;
}

__device__ __forceinline__ double geom_weight(int code) {
  int cnt = 0;
  for (int d = 0; d < 3; ++d) cnt += oc(code, d) != 0;
  return cnt == 1 ? 1.0 : (cnt == 2 ? 0.5 : 0.25);
}

// geometry table: per part origin[3], dims[3], offset
struct Geo {
  int o[3], n[3], off;
};

__device__ __forceinline__ Geo geo_of(const int *g, int p) {
  Geo r;
  for (int d = 0; d < 3; ++d) {
    r.o[d] = g[7 * p + d];
    r.n[d] = g[7 * p + 3 + d];
  }
  r.off = g[7 * p + 6];
  return r;
}

// part q != p holding global point G, and the cell id there; -1 if none
__device__ int find_part(const int *geom, int nparts, int p, const int G[3], int &cell) {
  for (int q = 0; q < nparts; ++q) {
    if (q == p) continue;
    const Geo h = geo_of(geom, q);
    bool in = true;
    for (int d = 0; d < 3; ++d) in = in && G[d] >= h.o[d] && G[d] < h.o[d] + h.n[d];
    if (in) {
      const int l0 = G[0] - h.o[0], l1 = G[1] - h.o[1], l2 = G[2] - h.o[2];
      cell = h.off + l0 + h.n[0] * (l1 + h.n[1] * l2);
      return q;
    }
  }
  return -1;
}

// one cell of k_fv_stencil: its stencil row, its links' metric terms and,
// along every direction d in which the cell is odd, its collapse sums: den
// (the coefficients with zero d component), sm / sp (those at -1 / +1), the
// off-center entries in entry order and then the center
__device__ __forceinline__ void fv_cell(const FvArgs &fa, const double *__restrict__ kappa,
                                        const double *__restrict__ aniso, double *const *__restrict__ coef,
                                        const Geo &me, int p, long long c, const double *s_as,
                                        const double *s_gw, double (&md)[3], double *__restrict__ csum,
                                        const long long *__restrict__ csoff) {
  const long long ncell = (long long)me.n[0] * me.n[1] * me.n[2];
  const int i = (int)(c % me.n[0]);
  const int j = (int)((c / me.n[0]) % me.n[1]);
  const int k = (int)(c / ((long long)me.n[0] * me.n[1]));
  const int loc[3] = {i, j, k};
  const double kc = kappa[me.off + c];
  const auto cf = dev::Gw(coef[p]);
  const auto kp = dev::G(kappa) + me.off;
  const long long sy = me.n[0], sz = (long long)me.n[0] * me.n[1];
  double diag = 0.0;
  double cd[3] = {0.0, 0.0, 0.0}, cm[3] = {0.0, 0.0, 0.0}, cp[3] = {0.0, 0.0, 0.0};
  for (int s = 1; s < fa.nent; ++s) {
    const int code = fa.code[s];
    const double as = s_as[s];
    const double xi = as * kc;
    const double gw = s_gw[s];
    int nb[3];
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      nb[d] = loc[d] + oc(code, d);
      in = in && (unsigned)nb[d] < (unsigned)me.n[d];
    }
    double t, v = 0.0;
    if (in) {
      const double xj = as * kp[c + oc(code, 0) + sy * oc(code, 1) + sz * oc(code, 2)];
      t = gw * 2.0 * xi * xj / (xi + xj);
      v = -t;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (oc(code, q) != 0) md[q] += t;
    } else {
      const int G[3] = {me.o[0] + nb[0], me.o[1] + nb[1], me.o[2] + nb[2]};
      int cell = 0;
      const int q = find_part(fa.geom, fa.nparts, p, G, cell);
      if (q >= 0) {
        const double xj = link_factor(aniso, q, code) * kappa[cell];
        t = gw * 2.0 * xi * xj / (xi + xj);
      } else {
        t = gw * xi;
      }
    }
    diag += t;
    cf[(long long)s * ncell + c] = v;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int o = oc(code, d);
      if (o == 0)
        cd[d] += v;
      else if (o < 0)
        cm[d] += v;
      else
        cp[d] += v;
    }
  }
  cf[c] = diag;   // entry 0 is the center
  if (!csum) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!(loc[d] & 1)) continue;
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    const long long h = me.n[d] >> 1;
    const long long nf = h * me.n[a] * me.n[b];
    // F-box index: the coordinates with loc[d] -> (loc[d]-1)/2 in the extents with n[d] -> n[d]/2
    const int g[3] = {d == 0 ? (loc[0] - 1) >> 1 : loc[0], d == 1 ? (loc[1] - 1) >> 1 : loc[1],
                      d == 2 ? (loc[2] - 1) >> 1 : loc[2]};
    const long long e0 = d == 0 ? h : me.n[0], e1 = d == 1 ? h : me.n[1];
    const long long fi = g[0] + e0 * (g[1] + e1 * g[2]);
    const auto out = dev::Gw(csum) + csoff[3 * p + d];
    out[fi] = cd[d] + diag;
    out[nf + fi] = cm[d];
    out[2 * nf + fi] = cp[d];
  }
}

// Also the block's partial sums of the direction metric c_d of Section 3.1
// (minus the off-diagonal same-part coefficients with a nonzero d component,
// the center being positive): the conductance of every same-part link, per
// direction its offset has; [part][block][3], reduced as k_wsum_partial's.
__global__ __launch_bounds__(kBlock) void k_fv_stencil(FvArgs fa, const double *__restrict__ kappa,
                                                       const double *__restrict__ aniso,
                                                       double *const *__restrict__ coef,
                                                       double *__restrict__ mpart, double *__restrict__ csum,
                                                       const long long *__restrict__ csoff) {
  // the part's link factors and geometric weights, once per block
  __shared__ double s_as[kMaxEnt], s_gw[kMaxEnt];
  __shared__ double sh[3][kBlock];
  const int p = blockIdx.y;
  if ((int)threadIdx.x < fa.nent) {
    s_as[threadIdx.x] = link_factor(aniso, p, fa.code[threadIdx.x]);
    s_gw[threadIdx.x] = geom_weight(fa.code[threadIdx.x]);
  }
  __syncthreads();
  const Geo me = geo_of(fa.geom, p);
  const long long ncell = (long long)me.n[0] * me.n[1] * me.n[2];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  double md[3] = {0.0, 0.0, 0.0};
  if (c < ncell) fv_cell(fa, kappa, aniso, coef, me, p, c, s_as, s_gw, md, csum, csoff);
  for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = md[q];
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
  }
  __syncthreads();
  if (threadIdx.x < 3) mpart[((long long)p * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_fv_coupling(int nrow, const int *__restrict__ urow,
                                                        const int *__restrict__ uptr,
                                                        const int *__restrict__ ucol,
                                                        const int *__restrict__ ucode,
                                                        const double *__restrict__ kappa,
                                                        const double *__restrict__ aniso,
                                                        double *__restrict__ uval) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrow) return;
  const int i = urow[r];
  for (int q = uptr[r]; q < uptr[r + 1]; ++q) {
    const unsigned w = (unsigned)ucode[q];   // offset (6 bits), row part, column part (13 bits each)
    const int code = (int)(w & 63u), pi = (int)((w >> 6) & 8191u), pj = (int)((w >> 19) & 8191u);
    const double xi = link_factor(aniso, pi, code) * kappa[i];
    const double xj = link_factor(aniso, pj, code) * kappa[ucol[q]];
    uval[q] = -geom_weight(code) * 2.0 * xi * xj / (xi + xj);
  }
}

// sum over the nrhs right-hand sides k of (lam_i,k - lam_j,k)(x_i,k - x_j,k)
// (vectors [cell][nrhs], right-hand side fastest)
__device__ __forceinline__ double pair_sum(const double *__restrict__ lam, const double *__restrict__ x,
                                           long long i, long long j, int nrhs) {
  double s = 0.0;
  for (int k = 0; k < nrhs; ++k)
    s += (lam[i * nrhs + k] - lam[j * nrhs + k]) * (x[i * nrhs + k] - x[j * nrhs + k]);
  return s;
}

__device__ __forceinline__ double self_sum(const double *__restrict__ lam, const double *__restrict__ x,
                                           long long i, int nrhs) {
  double s = 0.0;
  for (int k = 0; k < nrhs; ++k) s += lam[i * nrhs + k] * x[i * nrhs + k];
  return s;
}

__global__ __launch_bounds__(kBlock) void k_fv_grad(FvArgs fa, const double *__restrict__ kappa,
                                                    const double *__restrict__ aniso,
                                                    const double *__restrict__ lam,
                                                    const double *__restrict__ x, int nrhs,
                                                    double *__restrict__ grad) {
  const int p = blockIdx.y;
  const Geo me = geo_of(fa.geom, p);
  const long long ncell = (long long)me.n[0] * me.n[1] * me.n[2];
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  const int loc[3] = {(int)(c % me.n[0]), (int)((c / me.n[0]) % me.n[1]),
                      (int)(c / ((long long)me.n[0] * me.n[1]))};
  const long long gi = me.off + c;
  const double kc = kappa[gi];
  double acc = 0.0;
  for (int s = 1; s < fa.nent; ++s) {
    const int code = fa.code[s];
    const double as = link_factor(aniso, p, code);
    const double xi = as * kc;
    const double gw = geom_weight(code);
    int nb[3];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      nb[d] = loc[d] + oc(code, d);
      in = in && nb[d] >= 0 && nb[d] < me.n[d];
    }
    if (in) {
      const long long gj = me.off + nb[0] + (long long)me.n[0] * (nb[1] + (long long)me.n[1] * nb[2]);
      const double xj = as * kappa[gj];
      const double dt = gw * as * 2.0 * xj * xj / ((xi + xj) * (xi + xj));
      acc += dt * pair_sum(lam, x, gi, gj, nrhs);
    } else {
      const int G[3] = {me.o[0] + nb[0], me.o[1] + nb[1], me.o[2] + nb[2]};
      int cell = 0;
      if (find_part(fa.geom, fa.nparts, p, G, cell) < 0) acc += gw * as * self_sum(lam, x, gi, nrhs);
    }
  }
  grad[gi] = -acc;
}

__global__ __launch_bounds__(kBlock) void k_fv_grad_u(int nrow, const int *__restrict__ urow,
                                                      const int *__restrict__ uptr,
                                                      const int *__restrict__ ucol,
                                                      const int *__restrict__ ucode,
                                                      const double *__restrict__ kappa,
                                                      const double *__restrict__ aniso,
                                                      const double *__restrict__ lam,
                                                      const double *__restrict__ x, int nrhs,
                                                      double *__restrict__ grad) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrow) return;
  const int i = urow[r];
  double acc = 0.0;
  for (int q = uptr[r]; q < uptr[r + 1]; ++q) {
    const unsigned w = (unsigned)ucode[q];   // offset (6 bits), row part, column part (13 bits each)
    const int code = (int)(w & 63u), pi = (int)((w >> 6) & 8191u), pj = (int)((w >> 19) & 8191u);
    const int j = ucol[q];
    const double ai = link_factor(aniso, pi, code);
    const double xi = ai * kappa[i];
    const double xj = link_factor(aniso, pj, code) * kappa[j];
    const double dt = geom_weight(code) * ai * 2.0 * xj * xj / ((xi + xj) * (xi + xj));
    acc += dt * pair_sum(lam, x, i, j, nrhs);
  }
  grad[i] -= acc;
}

inline unsigned nblk(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

void launch_fv_stencil(const FvArgs &fa, int maxcell, const double *kappa, const double *aniso,
                       double *const *coef, double *mpart, double *csum, const long long *csoff,
                       hipStream_t st) {
  k_fv_stencil<<<dim3(fv_blocks(maxcell), fa.nparts), kBlock, 0, st>>>(fa, kappa, aniso, coef, mpart, csum,
                                                                       csoff);
}

void launch_fv_coupling(int nrow, const int *urow, const int *uptr, const int *ucol,
                        const int *ucode, const double *kappa, const double *aniso, double *uval,
                        hipStream_t st) {
  if (nrow > 0)
    k_fv_coupling<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, ucol, ucode, kappa, aniso, uval);
}

void launch_fv_grad(const FvArgs &fa, int maxcell, const double *kappa, const double *aniso,
                    const double *lam, const double *x, int nrhs, double *grad, int nrow, const int *urow,
                    const int *uptr, const int *ucol, const int *ucode, hipStream_t st) {
  k_fv_grad<<<dim3(nblk(maxcell), fa.nparts), kBlock, 0, st>>>(fa, kappa, aniso, lam, x, nrhs, grad);
  if (nrow > 0)
    k_fv_grad_u<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, ucol, ucode, kappa, aniso, lam, x,
                                               nrhs, grad);
}

}  // namespace ssamg
