// Symbolic Galerkin product of the couplings on the device (Section 3.3,
// eq:galerkin, term P^T U P): the structure of U_{l+1} = P_l^T U_l P_l and,
// for each of its entries, the ordered list of contributions
// (U_l entry, weight source of P(f, I), weight source of P(g, J)).
//
// Every U_l entry (f, g) meets at most two nonzeros in row f and two in row
// g of P (two-point interpolation), so it emits up to four records keyed by
// the coarse pair (I, J).  A stable radix sort on the key groups the records
// by coarse entry while keeping the emission order (row-major over U_l), so
// the numeric pass sums each entry in a fixed order.  Runs of equal keys are
// the coarse entries; runs of equal I are the stored rows.
#include <hipcub/hipcub.hpp>

#include "ssamg_impl.h"

namespace ssamg {

namespace {

__device__ int part_of_cell(const SymPart *sp, int np, long long cell) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sp[mid].off <= cell)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// nonzeros of row `cell` of P: coarse ids and weight sources (-1 = 1.0, else
// an index into the level's weight buffer, wm block then wp block per part)
__device__ int prow(const SymPart *sp, int np, long long cell, int col[2], int src[2]) {
  const SymPart &q = sp[part_of_cell(sp, np, cell)];
  const long long loc = cell - q.off;
  if (q.dstar < 0) {
    col[0] = (int)(q.coff + loc);
    src[0] = -1;
    return 1;
  }
  int f[3];
  f[0] = (int)(loc % q.n[0]);
  f[1] = (int)((loc / q.n[0]) % q.n[1]);
  f[2] = (int)(loc / ((long long)q.n[0] * q.n[1]));
  const int ds = q.dstar;
  int c[3] = {f[0], f[1], f[2]};
  if ((f[ds] & 1) == 0) {
    c[ds] = f[ds] >> 1;
    col[0] = (int)(q.coff + c[0] + (long long)q.cn[0] * (c[1] + (long long)q.cn[1] * c[2]));
    src[0] = -1;
    return 1;
  }
  int g[3] = {f[0], f[1], f[2]};
  g[ds] = (f[ds] - 1) >> 1;
  const long long fl = g[0] + (long long)q.fn[0] * (g[1] + (long long)q.fn[1] * g[2]);
  c[ds] = (f[ds] - 1) >> 1;
  col[0] = (int)(q.coff + c[0] + (long long)q.cn[0] * (c[1] + (long long)q.cn[1] * c[2]));
  src[0] = (int)(q.wofs + fl);
  if (f[ds] + 1 <= q.n[ds] - 1) {
    c[ds] = (f[ds] + 1) >> 1;
    col[1] = (int)(q.coff + c[0] + (long long)q.cn[0] * (c[1] + (long long)q.cn[1] * c[2]));
    src[1] = (int)(q.wofs + q.nf + fl);
    return 2;
  }
  return 1;
}

// one thread per entry q of U_l (row cell erow[q]); its records sit at 4q .. 4q+3
__global__ __launch_bounds__(kBlock) void k_emit(const SymPart *__restrict__ sp, int np, long long nnz,
                                                 const int *__restrict__ erow,
                                                 const int *__restrict__ ucol,
                                                 unsigned long long nc, unsigned long long invalid,
                                                 unsigned long long *__restrict__ key,
                                                 unsigned *__restrict__ idx, int *__restrict__ rk,
                                                 int *__restrict__ ra, int *__restrict__ rb,
                                                 int *__restrict__ small) {
  const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (q < 4) small[q] = 0;   // counts of k_flags / k_counts start at zero
  if (q >= nnz) return;
  int cf[2], sf[2], cg[2], sg[2];
  const int nf = prow(sp, np, erow[q], cf, sf);
  const int ng = prow(sp, np, ucol[q], cg, sg);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const long long i = 4LL * q + t;
    const int a = t >> 1, b = t & 1;
    idx[i] = (unsigned)i;
    if (a < nf && b < ng) {
      key[i] = (unsigned long long)cf[a] * nc + (unsigned long long)cg[b];
      rk[i] = (int)q;
      ra[i] = sf[a];
      rb[i] = sg[b];
    } else {
      key[i] = invalid;
      rk[i] = ra[i] = rb[i] = 0;
    }
  }
}

// The records in key order, ties in record order (the order of a stable sort):
// count the valid records of every coarse row, scan the counts into row
// offsets, scatter every valid record into its row's range (any order), then
// place each at its row offset plus its rank among the row's records by
// (key, record index).  Positions past the valid records get the invalid key.
__global__ __launch_bounds__(kBlock) void k_row_count(const unsigned long long *__restrict__ key, long long n,
                                                      unsigned long long nc, unsigned long long invalid,
                                                      int *__restrict__ cnt) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = key[i];
  if (k != invalid) atomicAdd(&cnt[k / nc], 1);
}

// cnt holds the row counts on entry and zeros on exit
__global__ __launch_bounds__(kBlock) void k_row_scatter(const unsigned long long *__restrict__ key,
                                                        const unsigned *__restrict__ idx, long long n,
                                                        unsigned long long nc, unsigned long long invalid,
                                                        const int *__restrict__ roff, int *__restrict__ cnt,
                                                        unsigned long long *__restrict__ tk,
                                                        unsigned *__restrict__ ti) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = key[i];
  if (k == invalid) return;
  const long long r = (long long)(k / nc);
  const int pos = roff[r] + atomicSub(&cnt[r], 1) - 1;
  tk[pos] = k;
  ti[pos] = idx[i];
}

__global__ __launch_bounds__(kBlock) void k_row_rank(const unsigned long long *__restrict__ tk,
                                                     const unsigned *__restrict__ ti, long long n,
                                                     unsigned long long nc, unsigned long long invalid,
                                                     const int *__restrict__ roff,
                                                     unsigned long long *__restrict__ key,
                                                     unsigned *__restrict__ idx) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  if (p >= roff[nc]) {
    key[p] = invalid;
    return;
  }
  const unsigned long long k = tk[p];
  const unsigned s = ti[p];
  const long long r = (long long)(k / nc);
  const int b = roff[r], e = roff[r + 1];
  int rank = 0;
  for (int j = b; j < e; ++j) {
    const unsigned long long kj = tk[j];
    const unsigned sj = ti[j];
    rank += (kj < k || (kj == k && sj < s)) ? 1 : 0;
  }
  key[b + rank] = k;
  idx[b + rank] = s;
}

// after the sort: flags of records that open a coarse entry / a coarse row,
// and the count of valid records (invalid keys sort last)
// packed flags: bit 0 a record that opens a coarse entry, bit 32 one that
// opens a coarse row (one 64-bit scan then counts both)
__global__ __launch_bounds__(kBlock) void k_flags(const unsigned long long *__restrict__ key,
                                                  long long n, unsigned long long nc,
                                                  unsigned long long invalid,
                                                  long long *__restrict__ flags, int *__restrict__ small) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const bool v = key[i] != invalid;
  const long long fnew = v && (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
  const long long frow = v && (i == 0 || key[i] / nc != key[i - 1] / nc) ? 1 : 0;
  flags[i] = fnew | (frow << 32);
  if (v && (i == n - 1 || key[i + 1] == invalid)) small[0] = (int)(i + 1);
}

// entry and row counts from the inclusive scan of the packed flags
__global__ void k_counts(const long long *__restrict__ scan, int *__restrict__ small) {
  const int nvalid = small[0];
  small[1] = nvalid > 0 ? (int)(scan[nvalid - 1] & 0xffffffffLL) : 0;
  small[2] = nvalid > 0 ? (int)(scan[nvalid - 1] >> 32) : 0;
}

// coarse entries (column, row), rows (cell, first entry) and the
// contributions in sorted order
__global__ __launch_bounds__(kBlock) void k_fill(const unsigned long long *__restrict__ key,
                                                 const unsigned *__restrict__ idx,
                                                 const long long *__restrict__ flags,
                                                 const long long *__restrict__ scan, long long nvalid,
                                                 unsigned long long nc, const int *__restrict__ rk,
                                                 const int *__restrict__ ra,
                                                 const int *__restrict__ rb, int *__restrict__ ucol,
                                                 int *__restrict__ erow, int *__restrict__ start,
                                                 int *__restrict__ urow, int *__restrict__ uptr,
                                                 int *__restrict__ ck, int *__restrict__ ca,
                                                 int *__restrict__ cb) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nvalid) return;
  const unsigned s = idx[i];
  ck[i] = rk[s];
  ca[i] = ra[s];
  cb[i] = rb[s];
  const long long f = flags[i], sc = scan[i];
  const int e = (int)(sc & 0xffffffffLL) - 1, rid = (int)(sc >> 32);
  if (f & 1) {
    ucol[e] = (int)(key[i] % nc);
    erow[e] = (int)(key[i] / nc);
    start[e] = (int)i;
  }
  if (f >> 32) {
    urow[rid - 1] = (int)(key[i] / nc);
    uptr[rid - 1] = e;
  }
  if (i == nvalid - 1) {
    start[e + 1] = (int)nvalid;
    uptr[rid] = e + 1;
  }
}

// entry -> row cell of a compressed-row matrix (the emitter's input)
__global__ __launch_bounds__(kBlock) void k_entry_rows(int nrow, const int *__restrict__ urow,
                                                       const int *__restrict__ uptr,
                                                       int *__restrict__ erow) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrow) return;
  for (int q = uptr[r]; q < uptr[r + 1]; ++q) erow[q] = urow[r];
}

// first stored row of every block of a grid-over-cells launch (1 << lg rhs)
// and that row's first entry: out[2b] = row, out[2b + 1] = uptr[row]
__global__ __launch_bounds__(kBlock) void k_ublk(const SymPart *__restrict__ sp, int np, int lg,
                                                 const long long *__restrict__ boff, int nrow,
                                                 const int *__restrict__ urow,
                                                 const int *__restrict__ uptr, int *__restrict__ out) {
  const int p = blockIdx.y;
  const SymPart &q = sp[p];
  const long long cpb = kBlock >> lg;
  const long long nchunk = (q.ncell + cpb - 1) / cpb;
  const long long b = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (b > nchunk) return;
  const long long first = q.off + (b * cpb < q.ncell ? b * cpb : q.ncell);
  int lo = 0, hi = nrow;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (urow[mid] < first)
      lo = mid + 1;
    else
      hi = mid;
  }
  out[2 * (boff[p] + b)] = lo;
  out[2 * (boff[p] + b) + 1] = nrow > 0 ? uptr[lo] : 0;
}

inline unsigned nblk(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

void DevBuf::reserve(size_t bytes) {
  if (bytes <= cap) return;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  const size_t want = bytes + bytes / 4 + 256;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    throw Error(SSAMG_ERR_ALLOC, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  cap = want;
}

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

// U_{l+1} structure and recipe from U_l (entries with row cells erow);
// returns (nnz, nrow) of U_{l+1}.  One host synchronization.
void coarse_coupling_device(SymScratch &w, const SymPart *sp, int np, int64_t nnz, const int *erow,
                            const int *ucol, int64_t nc, CouplingStore &out, int64_t &out_nnz,
                            int &out_nrow, hipStream_t st, const std::function<void()> &before_sync) {
  out_nnz = 0;
  out_nrow = 0;
  if (nnz == 0) return;
  const long long n = 4LL * nnz;
  int end_bit = 1;
  while (end_bit < 64 && ((unsigned long long)1 << end_bit) <= (unsigned long long)nc * nc) ++end_bit;
  const unsigned long long invalid = end_bit >= 64 ? ~0ULL : (((unsigned long long)1 << end_bit) - 1);
  w.key0.reserve(n * 8);
  w.key1.reserve(n * 8);
  w.idx0.reserve(n * 4);
  w.idx1.reserve(n * 4);
  w.rk.reserve(n * 4);
  w.ra.reserve(n * 4);
  w.rb.reserve(n * 4);
  w.flags.reserve(n * 8);
  w.scan.reserve(n * 8);
  w.small.reserve(64);
  if (!w.host_small) {
    void *h = nullptr;
    SSAMG_HIP(hipHostMalloc(&h, 64));
    w.host_small = (int *)h;
  }
  auto *k0 = (unsigned long long *)w.key0.p, *k1 = (unsigned long long *)w.key1.p;
  auto *i0 = (unsigned *)w.idx0.p, *i1 = (unsigned *)w.idx1.p;
  int *rk = (int *)w.rk.p, *ra = (int *)w.ra.p, *rb = (int *)w.rb.p;
  long long *flags = (long long *)w.flags.p, *scan = (long long *)w.scan.p;
  int *small = (int *)w.small.p;
  k_emit<<<nblk(nnz), kBlock, 0, st>>>(sp, np, nnz, erow, ucol, (unsigned long long)nc, invalid, k0, i0,
                                       rk, ra, rb, small);
  // key order, ties in record order.  Up to w.row_sort records: k0/i0 ->
  // row buckets in k1/i1 -> ranked in k0/i0 (five launches); above, a stable
  // radix sort k0/i0 -> k1/i1 (its passes pay off on large levels)
  if (n > w.row_sort) {
    size_t rbytes = 0;
    SSAMG_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, rbytes, k0, k1, i0, i1, (int)n, 0, end_bit, st));
    w.temp.reserve(rbytes);
    SSAMG_HIP(hipcub::DeviceRadixSort::SortPairs(w.temp.p, rbytes, k0, k1, i0, i1, (int)n, 0, end_bit, st));
  } else {
    w.rcnt.reserve((size_t)(nc + 1) * 4);
    w.roff.reserve((size_t)(nc + 1) * 4);
    int *rcnt = (int *)w.rcnt.p, *roff = (int *)w.roff.p;
    SSAMG_HIP(hipMemsetAsync(rcnt, 0, (size_t)(nc + 1) * 4, st));
    k_row_count<<<nblk(n), kBlock, 0, st>>>(k0, n, (unsigned long long)nc, invalid, rcnt);
    size_t tbytes = 0;
    SSAMG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tbytes, rcnt, roff, (int)(nc + 1), st));
    w.temp.reserve(tbytes);
    SSAMG_HIP(hipcub::DeviceScan::ExclusiveSum(w.temp.p, tbytes, rcnt, roff, (int)(nc + 1), st));
    k_row_scatter<<<nblk(n), kBlock, 0, st>>>(k0, i0, n, (unsigned long long)nc, invalid, roff, rcnt, k1, i1);
    k_row_rank<<<nblk(n), kBlock, 0, st>>>(k1, i1, n, (unsigned long long)nc, invalid, roff, k0, i0);
    std::swap(k0, k1);
    std::swap(i0, i1);
  }
  k_flags<<<nblk(n), kBlock, 0, st>>>(k1, n, (unsigned long long)nc, invalid, flags, small);
  size_t tbytes = 0;
  SSAMG_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tbytes, flags, scan, (int)n, st));
  w.temp.reserve(tbytes);
  SSAMG_HIP(hipcub::DeviceScan::InclusiveSum(w.temp.p, tbytes, flags, scan, (int)n, st));
  k_counts<<<1, 1, 0, st>>>(scan, small);
  SSAMG_HIP(hipMemcpyAsync(w.host_small, small, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
  if (before_sync) before_sync();   // host work that overlaps the device's
  SSAMG_HIP(hipStreamSynchronize(st));
  const int nvalid = w.host_small[0], nent = w.host_small[1], nr = w.host_small[2];
  if (nvalid == 0) return;
  out.ucol.reserve((size_t)nent * 4);
  out.erow.reserve((size_t)nent * 4);
  out.start.reserve((size_t)(nent + 1) * 4);
  out.urow.reserve((size_t)nr * 4);
  out.uptr.reserve((size_t)(nr + 1) * 4);
  out.ck.reserve((size_t)nvalid * 4);
  out.ca.reserve((size_t)nvalid * 4);
  out.cb.reserve((size_t)nvalid * 4);
  k_fill<<<nblk(nvalid), kBlock, 0, st>>>(k1, i1, flags, scan, nvalid, (unsigned long long)nc,
                                          rk, ra, rb, (int *)out.ucol.p, (int *)out.erow.p,
                                          (int *)out.start.p, (int *)out.urow.p, (int *)out.uptr.p,
                                          (int *)out.ck.p, (int *)out.ca.p, (int *)out.cb.p);
  SSAMG_HIP(hipGetLastError());
  out_nnz = nent;
  out_nrow = nr;
  out.ncontrib = nvalid;
}

void launch_entry_rows(int nrow, const int *urow, const int *uptr, int *erow, hipStream_t st) {
  if (nrow > 0) k_entry_rows<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, erow);
}

void launch_ublk(const SymPart *sp, int np, int lg, int64_t maxchunk, const long long *boff, int nrow,
                 const int *urow, const int *uptr, int *out, hipStream_t st) {
  k_ublk<<<dim3(nblk(maxchunk + 1), np), kBlock, 0, st>>>(sp, np, lg, boff, nrow, urow, uptr, out);
}

}  // namespace ssamg
