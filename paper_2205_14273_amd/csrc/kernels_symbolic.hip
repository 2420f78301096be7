// Symbolic Galerkin product of the couplings on the device (Section 3.3,
// eq:galerkin, term P^T U P): the structure of U_{l+1} = P_l^T U_l P_l and,
// for each of its entries, the ordered list of contributions
// (U_l entry, weight source of P(f, I), weight source of P(g, J)).
//
// Every U_l entry (f, g) meets at most two nonzeros in row f and two in row
// g of P (two-point interpolation), so it emits up to four records keyed by
// the coarse pair (I, J).  The records are put in key order with ties in
// emission order (row-major over U_l, the order of a stable sort), so the
// numeric pass sums each entry in a fixed order: counted into coarse-row
// buckets (as they are emitted), scattered, and ranked inside each row, which
// also numbers the row's entries.  Runs of equal keys are the coarse entries;
// runs of equal I are the stored rows.  All scans are the block scans below.
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

// The lanes of a wave with the same coarse row r >= 0 form a group: one lane
// of each group calls f(r, group mask, leader lane); wave-uniform loop
template <typename F>
__device__ __forceinline__ void wave_groups(int r, F &&f) {
  unsigned long long pending = __ballot(r >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int val = __shfl(r, leader, 64);
    const unsigned long long same = __ballot(r == val) & pending;
    f(val, same, leader);
    pending &= ~same;
  }
}

// one thread per entry q of U_l (row cell erow[q]); its records sit at
// 4q .. 4q+3 (a record's index is its position).  The valid records are counted into their coarse rows' buckets
// (cnt, zero on entry), a wave's records with the same row with one atomic.
__global__ __launch_bounds__(kBlock) void k_emit(const SymPart *__restrict__ sp, int np, long long nnz,
                                                 const int *__restrict__ erow,
                                                 const int *__restrict__ ucol,
                                                 unsigned long long nc, unsigned long long invalid,
                                                 unsigned long long *__restrict__ key,
                                                 int *__restrict__ rk, int *__restrict__ ra,
                                                 int *__restrict__ rb, int *__restrict__ cnt) {
  const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int cf[2] = {-1, -1}, sf[2], cg[2], sg[2];
  int nf = 0, ng = 0;
  if (q < nnz) {
    nf = prow(sp, np, erow[q], cf, sf);
    ng = prow(sp, np, ucol[q], cg, sg);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const long long i = 4LL * q + t;
      const int a = t >> 1, b = t & 1;
      if (a < nf && b < ng) {
        key[i] = (unsigned long long)cf[a] * nc + (unsigned long long)cg[b];
        rk[i] = (int)q;
        ra[i] = sf[a];
        rb[i] = sg[b];
      } else {
        key[i] = invalid;   // never ranked or read again
      }
    }
  }
  // coarse row cf[a] takes ng valid records of this entry (one or two)
  const unsigned long long two = __ballot(ng == 2);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int r = a < nf && ng > 0 ? cf[a] : -1;
    wave_groups(r, [&](int val, unsigned long long same, int leader) {
      if (lane == leader) atomicAdd(&cnt[val], __popcll(same) + __popcll(same & two));
    });
  }
}

// The records in key order, ties in record order (the order of a stable sort):
// count the valid records of every coarse row (k_emit), scan the counts into row
// offsets, scatter every valid record into its row's range (any order), then
// place each at its row offset plus its rank among the row's records by
// (key, record index).  Positions past the valid records get the invalid key.
// A wave's 64 records fall in few coarse rows (those of a handful of fine
// rows), though not in runs (the two coarse rows of an F row alternate), so
// the wave groups its lanes by row: one lane per distinct row touches that
// row's counter, with the group's size, and each lane gets its rank in its
// group.
__device__ __forceinline__ int rec_row(const unsigned long long *__restrict__ key, long long n,
                                       unsigned long long nc, unsigned long long invalid) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const unsigned long long k = i < n ? key[i] : invalid;
  return k != invalid ? (int)(k / nc) : -1;
}

// cnt holds the row counts on entry and zeros on exit; a group takes
// consecutive slots of its row's range
__global__ __launch_bounds__(kBlock) void k_row_scatter(const unsigned long long *__restrict__ key, long long n,
                                                        unsigned long long nc, unsigned long long invalid,
                                                        const int *__restrict__ roff, int *__restrict__ cnt,
                                                        unsigned long long *__restrict__ tk,
                                                        unsigned *__restrict__ ti) {
  const int r = rec_row(key, n, nc, invalid);
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ULL << lane) - 1;
  int pos = 0;
  wave_groups(r, [&](int val, unsigned long long same, int leader) {
    const int m = __popcll(same);
    int base = 0;
    if (lane == leader) base = roff[val] + atomicSub(&cnt[val], m) - m;
    base = __shfl(base, leader, 64);
    if ((same >> lane) & 1) pos = base + __popcll(same & below);
  });
  if (r < 0) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  tk[pos] = key[i];
  ti[pos] = (unsigned)i;
}

// coarse entries (column, row), rows (cell, first entry) and the
// contributions in sorted order; rscan[r] = first entry | row number << 32
__global__ __launch_bounds__(kBlock) void k_fill(const unsigned long long *__restrict__ key,
                                                 const unsigned *__restrict__ idx,
                                                 const int *__restrict__ ent,
                                                 const int *__restrict__ roff,
                                                 const long long *__restrict__ rscan,
                                                 long long *__restrict__ rinfo, long long nvalid,
                                                 long long nent, long long nrow,
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
  const unsigned long long k = key[i];
  const long long r = (long long)(k / nc);
  const long long rs = rscan[r];
  const int e0 = (int)(rs & 0xffffffffLL), rid = (int)(rs >> 32);
  const int en = ent[i];
  const bool rowstart = roff[r] == i;
  if (rowstart || ent[i - 1] != en) {                     // first record of a coarse entry
    ucol[e0 + en] = (int)(k % nc);
    erow[e0 + en] = (int)r;
    start[e0 + en] = (int)i;
  }
  if (rowstart) {
    urow[rid] = (int)r;
    uptr[rid] = e0;
    rinfo[r] = 0;                                          // zero again for the next call
  }
  if (i == nvalid - 1) {
    start[nent] = (int)nvalid;
    uptr[nrow] = (int)nent;
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
__global__ __launch_bounds__(kBlock) void k_ublk(const SymPart *__restrict__ sp_all, int np,
                                                 const long long *__restrict__ boff_all, UblkJobs jobs) {
  const UblkJob &jb = jobs.j[blockIdx.z];
  const int p = blockIdx.y;
  const SymPart &q = sp_all[jb.spat + p];
  const long long *boff = boff_all + jb.boffat;
  const long long cpb = kBlock >> jb.lg;
  const long long nchunk = (q.ncell + cpb - 1) / cpb;
  const long long b = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (b > nchunk) return;
  const long long first = q.off + (b * cpb < q.ncell ? b * cpb : q.ncell);
  const int nrow = jb.nrow;
  int lo = 0, hi = nrow;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (jb.urow[mid] < first)
      lo = mid + 1;
    else
      hi = mid;
  }
  jb.out[2 * (boff[p] + b)] = lo;
  jb.out[2 * (boff[p] + b) + 1] = nrow > 0 ? jb.uptr[lo] : 0;
}

// Rank of every record inside its row by (key, record index), one wave per
// chunk of 64 sorted positions: the wave takes each row that starts in its
// chunk and every lane counts, for its records, the smaller ones.  Inside a
// row every key has the same coarse row, so (column, record index) packed in
// 64 bits orders it; rows of at most cap records are staged and ordered in
// LDS that way (else read from and ordered in memory).  The same positions as
// a stable sort.  A scan over the ordered row then numbers its distinct
// columns (the coarse entries): ent[i] is record i's entry inside its row, and
// rowinfo[r] = entry count | 1 << 32 for a row with records, whose scan over
// the rows gives every row's first entry and its row number.
constexpr int kRankCap = 512;
__global__ __launch_bounds__(64) void k_row_rank_lds(const unsigned long long *__restrict__ tk,
                                                     const unsigned *__restrict__ ti, long long n,
                                                     unsigned long long nc, unsigned long long invalid,
                                                     const int *__restrict__ roff, int cap,
                                                     unsigned long long *__restrict__ key,
                                                     unsigned *__restrict__ idx, int *__restrict__ ent,
                                                     long long *__restrict__ rowinfo) {
  __shared__ unsigned long long sv[kRankCap];
  __shared__ unsigned long long ss[kRankCap];
  const int lane = threadIdx.x;
  const long long p = (long long)blockIdx.x * 64 + lane;
  const long long total = roff[nc];
  if (p < n && p >= total) key[p] = invalid;
  bool start = false;
  if (p < total) {
    const long long r = (long long)(tk[p] / nc);
    start = roff[r] == p;
  }
  unsigned long long starts = __ballot(start);
  while (starts) {                                         // wave-uniform
    const int l = __ffsll((long long)starts) - 1;
    starts &= starts - 1;
    const long long p0 = (long long)blockIdx.x * 64 + l;
    const long long r = (long long)(tk[p0] / nc);
    const int b = roff[r], e = roff[r + 1], len = e - b;
    const unsigned long long rbase = (unsigned long long)r * nc;
    auto packed = [&](int q) { return ((tk[q] - rbase) << 32) | ti[q]; };
    const bool lds = len <= cap;
    if (lds) {
      for (int q = lane; q < len; q += 64) sv[q] = packed(b + q);
      __syncthreads();
      for (int q = lane; q < len; q += 64) {
        const unsigned long long v = sv[q];
        int rank = 0;
        int j = 0;
        for (; j + 4 <= len; j += 4)
          rank += (sv[j] < v) + (sv[j + 1] < v) + (sv[j + 2] < v) + (sv[j + 3] < v);
        for (; j < len; ++j) rank += sv[j] < v;
        ss[rank] = v;
      }
    } else {
      for (int q = lane; q < len; q += 64) {
        const unsigned long long v = packed(b + q);
        int rank = 0;
        for (int j = b; j < e; ++j) rank += packed(j) < v;
        key[b + rank] = rbase + (v >> 32);
        idx[b + rank] = (unsigned)v;
      }
    }
    __syncthreads();
    // number the distinct columns in order (a wave scan per 64 positions)
    auto col = [&](int q) { return lds ? ss[q] >> 32 : key[b + q] - rbase; };
    int carry = 0;
    for (int q0 = 0; q0 < len; q0 += 64) {                 // wave-uniform
      const int q = q0 + lane;
      int f = 0;
      if (q < len) f = q == 0 || col(q) != col(q - 1);
      int sc = f;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(sc, o, 64);
        if (lane >= o) sc += t;
      }
      if (q < len) {
        if (lds) {
          key[b + q] = rbase + (ss[q] >> 32);
          idx[b + q] = (unsigned)ss[q];
        }
        ent[b + q] = carry + sc - 1;
      }
      carry += __shfl(sc, 63, 64);
    }
    if (lane == 0) rowinfo[r] = (long long)carry | (1LL << 32);
    __syncthreads();
  }
}

// Three-pass scans over blocks of kScanItems elements (kBlock threads of
// kScanPer consecutive items): per-block sums, an exclusive scan of those sums
// in one block, then each block's scan plus its offset.
constexpr int kScanPer = 8;
constexpr int kScanItems = kBlock * kScanPer;

template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T *sh, T &total) {
  // exclusive prefix of v over the block's threads (Hillis-Steele in LDS)
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const T add = tid >= o ? sh[tid - o] : T(0);
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[kBlock - 1];
  const T incl = sh[tid];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T *__restrict__ in, long long n,
                                                        T *__restrict__ bsum) {
  __shared__ T sh[kBlock];
  const long long base = (long long)blockIdx.x * kScanItems + (long long)threadIdx.x * kScanPer;
  T v = T(0);
#pragma unroll
  for (int q = 0; q < kScanPer; ++q)
    if (base + q < n) v += in[base + q];
  T total;
  (void)block_exclusive(v, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// in place: bsum[b] <- sum of bsum[0 .. b-1]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_sums(T *__restrict__ bsum, int nb) {
  __shared__ T sh[kBlock];
  T carry = T(0);
  for (int c0 = 0; c0 < nb; c0 += kBlock) {
    const int i = c0 + (int)threadIdx.x;
    const T v = i < nb ? bsum[i] : T(0);
    T total;
    const T ex = block_exclusive(v, sh, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
}

// bsum null: a single block (offset 0).  sizes non-null: the thread that
// writes out[n-1] of the row scan also stores the sizes for the host:
// sizes[0] = *nvalid, sizes[1] = out[n-1] & 0xffffffff, sizes[2] = out[n-1] >> 32
template <typename T, bool INCLUSIVE>
__global__ __launch_bounds__(kBlock) void k_scan_down(const T *__restrict__ in, long long n,
                                                      const T *__restrict__ bsum, T *__restrict__ out,
                                                      const int *__restrict__ nvalid,
                                                      int *__restrict__ sizes) {
  __shared__ T sh[kBlock];
  const long long base = (long long)blockIdx.x * kScanItems + (long long)threadIdx.x * kScanPer;
  T v[kScanPer];
  T tsum = T(0);
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = base + q < n ? in[base + q] : T(0);
    tsum += v[q];
  }
  T total;
  T run = (bsum ? bsum[blockIdx.x] : T(0)) + block_exclusive(tsum, sh, total);
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (INCLUSIVE) run += v[q];
    if (base + q < n) out[base + q] = run;
    if (sizes && base + q == n - 1) {
      const long long w = (long long)run;
      sizes[0] = *nvalid;
      sizes[1] = (int)(w & 0xffffffffLL);
      sizes[2] = (int)(w >> 32);
    }
    if (!INCLUSIVE) run += v[q];
  }
}

inline unsigned nblk(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b > 0 ? b : 1);
}

// out = scan of in[0 .. n) (exclusive or inclusive); bs: scratch for the
// block sums (one launch when a block covers n); nvalid, sizes: see k_scan_down
template <typename T, bool INCLUSIVE>
void device_scan(const T *in, T *out, long long n, DevBuf &bs, hipStream_t st, const int *nvalid = nullptr,
                 int *sizes = nullptr) {
  if (n <= 0) return;
  const long long nb = (n + kScanItems - 1) / kScanItems;
  T *b = nullptr;
  if (nb > 1) {
    bs.reserve((size_t)(nb + 1) * sizeof(T));
    b = (T *)bs.p;
    k_scan_reduce<T><<<(unsigned)nb, kBlock, 0, st>>>(in, n, b);
    k_scan_sums<T><<<1, kBlock, 0, st>>>(b, (int)nb);
  }
  k_scan_down<T, INCLUSIVE><<<(unsigned)nb, kBlock, 0, st>>>(in, n, b, out, nvalid, sizes);
}

// reserve a buffer that the caller keeps all zero between calls: cleared
// here only when its allocation is new
void zero_reserve(DevBuf &b, size_t bytes, const void *&zp, size_t &zcap, hipStream_t st) {
  b.reserve(bytes);
  if (b.p != zp || b.cap != zcap) {
    zp = nullptr;
    SSAMG_HIP(hipMemsetAsync(b.p, 0, b.cap, st));
    zp = b.p;
    zcap = b.cap;
  }
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
  // every buffer first: nothing below throws before the two zero-kept
  // buffers are zero again, except a device error (which clears the record)
  w.key0.reserve(n * 8);
  w.key1.reserve(n * 8);
  w.idx0.reserve(n * 4);
  w.idx1.reserve(n * 4);
  w.rk.reserve(n * 4);
  w.ra.reserve(n * 4);
  w.rb.reserve(n * 4);
  w.ent.reserve(n * 4);
  w.roff.reserve((size_t)(nc + 1) * 4);
  w.rscan.reserve((size_t)(nc + 1) * 8);
  w.temp.reserve((size_t)((nc + 1 + kScanItems - 1) / kScanItems + 1) * 8);
  zero_reserve(w.rcnt, (size_t)(nc + 1) * 4, w.rcnt_zero, w.rcnt_zcap, st);
  zero_reserve(w.rinfo, (size_t)(nc + 1) * 8, w.rinfo_zero, w.rinfo_zcap, st);
  if (!w.host_small) {
    // coherent pinned memory the scan kernel writes the sizes into
    void *h = nullptr, *dv = nullptr;
    SSAMG_HIP(hipHostMalloc(&h, 64, hipHostMallocCoherent | hipHostMallocMapped));
    w.host_small = (int *)h;
    SSAMG_HIP(hipHostGetDevicePointer(&dv, h, 0));
    w.dev_small = (int *)dv;
  }
  auto *k0 = (unsigned long long *)w.key0.p, *k1 = (unsigned long long *)w.key1.p;
  auto *i0 = (unsigned *)w.idx0.p, *i1 = (unsigned *)w.idx1.p;
  int *rk = (int *)w.rk.p, *ra = (int *)w.ra.p, *rb = (int *)w.rb.p;
  int *ent = (int *)w.ent.p;
  int *rcnt = (int *)w.rcnt.p, *roff = (int *)w.roff.p;
  long long *rinfo = (long long *)w.rinfo.p, *rscan = (long long *)w.rscan.p;
  // a device error leaves the zero-kept buffers unknown
  struct Guard {
    SymScratch &w;
    bool armed = true;
    ~Guard() {
      if (armed) w.rcnt_zero = w.rinfo_zero = nullptr;
    }
  } guard{w};
  // records and row counts (rcnt) -> row offsets -> row buckets in k1/i1
  // (rcnt back to zero) -> ranked inside each row into k0/i0 with entry
  // numbers and row counts (rinfo) -> row scan and the sizes
  k_emit<<<nblk(nnz), kBlock, 0, st>>>(sp, np, nnz, erow, ucol, (unsigned long long)nc, invalid, k0, rk, ra,
                                       rb, rcnt);
  device_scan<int, false>(rcnt, roff, nc + 1, w.temp, st);
  k_row_scatter<<<nblk(n), kBlock, 0, st>>>(k0, n, (unsigned long long)nc, invalid, roff, rcnt, k1, i1);
  k_row_rank_lds<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(k1, i1, n, (unsigned long long)nc, invalid, roff,
                                                            (int)std::min<int64_t>(w.row_sort, kRankCap), k0, i0,
                                                            ent, rinfo);
  std::swap(k0, k1);
  std::swap(i0, i1);
  // the sizes go straight to the host's pinned buffer (read after the sync)
  device_scan<long long, false>(rinfo, rscan, nc + 1, w.temp, st, roff + nc, w.dev_small);
  if (before_sync) before_sync();   // host work that overlaps the device's
  SSAMG_HIP(hipStreamSynchronize(st));
  const int nvalid = w.host_small[0], nent = w.host_small[1], nr = w.host_small[2];
  if (nvalid == 0) {
    guard.armed = false;                  // no row written, rcnt back to zero
    return;
  }
  out.ucol.reserve((size_t)nent * 4);
  out.erow.reserve((size_t)nent * 4);
  out.start.reserve((size_t)(nent + 1) * 4);
  out.urow.reserve((size_t)nr * 4);
  out.uptr.reserve((size_t)(nr + 1) * 4);
  out.ck.reserve((size_t)nvalid * 4);
  out.ca.reserve((size_t)nvalid * 4);
  out.cb.reserve((size_t)nvalid * 4);
  k_fill<<<nblk(nvalid), kBlock, 0, st>>>(k1, i1, ent, roff, rscan, rinfo, nvalid, nent, nr, (unsigned long long)nc,
                                          rk, ra, rb, (int *)out.ucol.p, (int *)out.erow.p,
                                          (int *)out.start.p, (int *)out.urow.p, (int *)out.uptr.p,
                                          (int *)out.ck.p, (int *)out.ca.p, (int *)out.cb.p);
  SSAMG_HIP(hipGetLastError());
  guard.armed = false;
  out_nnz = nent;
  out_nrow = nr;
  out.ncontrib = nvalid;
}

void launch_entry_rows(int nrow, const int *urow, const int *uptr, int *erow, hipStream_t st) {
  if (nrow > 0) k_entry_rows<<<nblk(nrow), kBlock, 0, st>>>(nrow, urow, uptr, erow);
}

void launch_ublk(const SymPart *sp, int np, const long long *boff, const UblkJobs &jobs, int64_t nbx,
                 hipStream_t st) {
  if (jobs.n > 0) k_ublk<<<dim3((unsigned)nbx, np, jobs.n), kBlock, 0, st>>>(sp, np, boff, jobs);
}

}  // namespace ssamg
