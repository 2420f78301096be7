// SSAMG solver: symbolic setup (Section 3.1 metric and Algorithm 1, symbolic
// coarse stencils and Galerkin tables, structure of every coarse coupling
// matrix), numeric setup (device kernels), the V(1,1) cycle and PCG.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <numeric>
#include <type_traits>

#include "capi_common.h"
#include "ssamg_impl.h"

namespace ssamg {

thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

namespace {

constexpr double kTieRtol = 1e-10;
constexpr double kInf = std::numeric_limits<double>::infinity();

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Bump allocator over the workspace; run once with base = nullptr to size it.
struct Carver {
  char *base = nullptr;
  size_t off = 0;
  size_t tab_begin = 0, tab_end = 0;   // host-built tables, uploaded with one copy
  template <typename T>
  T *take(size_t n) {
    off = align_up(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

int64_t vol(const std::array<int, 3> &n) { return (int64_t)n[0] * n[1] * n[2]; }

void carve(Solver &s, Carver &cv);

int argmin_tied(const std::array<double, 3> &w, const std::vector<int> &cand) {
  double wmin = kInf;
  for (int d : cand) wmin = std::min(wmin, w[d]);
  for (int d : cand)
    if (w[d] == wmin || w[d] <= wmin * (1.0 + kTieRtol)) return d;
  return cand.front();
}

// eq:relax1 / eq:alpha-beta: omega_p = 2 / (3 - beta_p / alpha_p)
double relax_weight(const std::array<double, 3> &w, int dstar, int ndim) {
  double alpha = 0.0, beta = 0.0;
  for (int d = 0; d < ndim; ++d) {
    const double inv = std::isfinite(w[d]) ? 1.0 / (w[d] * w[d]) : 0.0;
    alpha += inv;
    if (d != dstar) beta += inv;
  }
  const double ratio = alpha > 0.0 ? beta / alpha : 0.0;
  return 2.0 / (3.0 - ratio);
}

// symbolic coarse stencil: along d*, 0 -> {-1,0,1} and +-1 -> {0,+-1}; sorted (dz,dy,dx)
std::vector<std::array<int, 3>> coarse_pattern(const std::vector<std::array<int, 3>> &fine, int ds) {
  std::vector<std::array<int, 3>> out;
  auto add = [&](std::array<int, 3> t) {
    if (std::find(out.begin(), out.end(), t) == out.end()) out.push_back(t);
  };
  for (auto s : fine) {
    if (ds < 0) {
      add(s);
    } else if (s[ds] == 0) {
      for (int t = -1; t <= 1; ++t) {
        auto u = s;
        u[ds] = t;
        add(u);
      }
    } else {
      auto u = s;
      u[ds] = 0;
      add(u);
      add(s);
    }
  }
  std::sort(out.begin(), out.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
    return std::make_tuple(a[2], a[1], a[0]) < std::make_tuple(b[2], b[1], b[0]);
  });
  return out;
}

int index_of(const std::vector<std::array<int, 3>> &pat, const std::array<int, 3> &t) {
  for (size_t e = 0; e < pat.size(); ++e)
    if (pat[e] == t) return (int)e;
  return -1;
}

// whether a part's coarse stencil is the non-Galerkin one (SSAMG_COARSE_OP_NONGALERKIN
// and a coarsened star stencil)
bool nongalerkin(const Solver &s, const PartLevel &q) {
  if (s.prm.coarse_op != SSAMG_COARSE_OP_NONGALERKIN || q.dstar < 0) return false;
  for (const auto &t : q.pat)
    if ((t[0] != 0) + (t[1] != 0) + (t[2] != 0) > 1) return false;
  return true;
}

// Entry maps of one part's Galerkin product over the 27 offsets (see k_rap):
// fine entry and coarse entry of each offset, and the offset of each coarse
// entry.  Every coarse entry a fine one reaches must be in the coarse pattern.
int cube_index(const std::array<int, 3> &o) { return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1); }

void build_rap_table(PartLevel &f, const std::vector<std::array<int, 3>> &cpat, bool ng) {
  f.rap_fmap.fill(-1);
  f.rap_cmap.fill(-1);
  f.rap_cofs.fill(0);
  for (size_t e = 0; e < f.pat.size(); ++e) f.rap_fmap[cube_index(f.pat[e])] = (int)e;
  for (size_t e = 0; e < cpat.size(); ++e) {
    f.rap_cmap[cube_index(cpat[e])] = (int)e;
    f.rap_cofs[e] = cube_index(cpat[e]);
  }
  f.rap_nent = (int)cpat.size();
  f.rap_ng = ng;
  if (f.dstar < 0) {
    for (const auto &t : cpat)
      if (f.rap_fmap[cube_index(t)] < 0) throw Error(SSAMG_ERR_STATE, "internal: identity transfer changes the pattern");
    return;
  }
  const int ds = f.dstar;
  if (f.nf < 1) throw Error(SSAMG_ERR_STATE, "internal: coarsened part without F cells");
  for (const auto &s : f.pat)
    for (int r = -1; r <= 1; ++r) {
      const int q = r + s[ds];
      for (int td : {(q & 1) == 0 ? q / 2 : (q - 1) / 2, (q & 1) == 0 ? q / 2 : (q + 1) / 2}) {
        auto t = s;
        t[ds] = td;
        const bool rerouted = ng && t[ds] != 0 && (t[0] != 0) + (t[1] != 0) + (t[2] != 0) > 1;
        if (td < -1 || td > 1 || (f.rap_cmap[cube_index(t)] < 0 && !rerouted))
          throw Error(SSAMG_ERR_STATE, "internal: Galerkin target outside coarse pattern");
      }
    }
}

// The FP64 product reads mirrored entries when the caller declares A symmetric
// and every part's given coefficients passed the symmetry test of set_coeffs.
bool mirrored(const Solver &s) {
  if (s.prm.symmetric == 0) return false;
  for (int ok : s.prob->sym_ok)
    if (!ok) return false;
  return true;
}

// Mirror reads of a symmetric stencil (see PartDesc::mir): an offset is
// positive when its last nonzero component (z, then y, then x) is positive.
bool positive_offset(const std::array<int, 3> &o) {
  for (int a = 2; a >= 0; --a)
    if (o[a] != 0) return o[a] > 0;
  return false;
}

// coefficient arrays the kernels stream for a part (all, or the center and the
// positive half when mirrored reads apply)
int streamed_entries(const PartLevel &q, bool symmetric) {
  int neg = 0;
  bool all = true;
  for (const auto &o : q.pat) {
    if (!positive_offset({-o[0], -o[1], -o[2]})) continue;
    ++neg;
    bool found = false;
    for (const auto &t : q.pat) found = found || (t[0] == -o[0] && t[1] == -o[1] && t[2] == -o[2]);
    all = all && found;
  }
  return symmetric && all ? (int)q.pat.size() - neg : (int)q.pat.size();
}

template <typename T>
PartDesc<T> make_desc(const Level &V, const PartLevel &q, size_t p, const T *coef, const T *w,
                      const T *uval, const T *rs, const int strips[kMaxLg + 1], bool symmetric = false) {
  PartDesc<T> d{};
  d.rs = rs ? rs + q.off : nullptr;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = q.n[a];
    d.fn[a] = q.fn[a];
    d.cn[a] = q.cn[a];
  }
  d.nent = (int)q.pat.size();
  d.center = q.center;
  d.dstar = q.dstar;
  d.faces = q.faces;
  d.off = q.off;
  d.ncell = q.ncell;
  d.coff = q.coff;
  d.cncell = q.cncell;
  d.nf = q.nf;
  d.omega = (T)q.omega;
  d.coef = coef;
  d.wm = w ? w + q.wofs : nullptr;
  d.wp = w ? w + q.wofs + q.nf : nullptr;
  d.urow = V.d_urow;
  d.uptr = V.d_uptr;
  d.ucol = V.d_ucol;
  d.uval = uval;
  for (int lg = 0; lg <= kMaxLg; ++lg)
    d.ublk[lg] = V.d_ublk[lg] ? V.d_ublk[lg] + 2 * V.ublk_off[lg][p] : nullptr;
  // block order of the four-column sweeps: whole blocks per z-plane, strips of it
  for (int lg = 2; lg <= kMaxLg; ++lg) {
    const long long cpb = (long long)(kBlock * 4) >> lg, plane = (long long)q.n[0] * q.n[1];
    d.tbp[lg] = (plane % cpb == 0) ? (int)(plane / cpb) : 0;
    d.tsb[lg] = (d.tbp[lg] > 0 && strips[lg] > 1) ? (d.tbp[lg] + strips[lg] - 1) / strips[lg] : 0;
  }
  for (int o = 0; o < 27; ++o) d.cube[o] = -1;
  for (size_t e = 0; e < q.pat.size(); ++e) {
    const auto &o = q.pat[e];
    d.cube[cube_index(o)] = (int)e;
    d.lin[e] = o[0] + q.n[0] * (o[1] + q.n[1] * o[2]);
    d.code[e] = pack_off(o[0], o[1], o[2]);
    d.lc[e] = d.lin[e] * 64 + d.code[e];
    d.mir[e] = (int)e;
    d.mlin[e] = 0;
  }
  if (symmetric) {
    // every negative offset needs its mirror in the pattern, else full reads
    std::vector<int> mir(q.pat.size(), -1);
    bool all = true;
    for (size_t e = 0; e < q.pat.size(); ++e) {
      if (!positive_offset({-q.pat[e][0], -q.pat[e][1], -q.pat[e][2]})) continue;   // e not negative
      for (size_t f = 0; f < q.pat.size(); ++f)
        if (q.pat[f][0] == -q.pat[e][0] && q.pat[f][1] == -q.pat[e][1] && q.pat[f][2] == -q.pat[e][2])
          mir[e] = (int)f;
      all = all && mir[e] >= 0;
    }
    if (all)
      for (size_t e = 0; e < q.pat.size(); ++e)
        if (mir[e] >= 0) {
          d.mir[e] = mir[e];
          d.mlin[e] = d.lin[e];
        }
  }
  return d;
}

template <typename T>
void upload(T *dst, const std::vector<T> &src, hipStream_t st) {
  if (!src.empty())
    SSAMG_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Part descriptors of level l in FP64 and (mixed-precision cycle) FP32, with
// the block order of the stored launch options: the cycle's descriptors take
// the cycle's strips; in a mixed-precision cycle the FP64 ones of level 0 serve
// the FP64 product of PCG and take its strips.
// Part p of level l gets its interpolation weights from the one-thread-per-
// coarse-cell Galerkin product that forms it (not for the lumped part-face
// reading, which needs the level's couplings, formed after that product).
bool weights_fused(const Solver &s, int l, size_t p) {
  const int L = (int)s.lv.size();
  if (l < 1 || l >= L - 1) return false;
  const Level &F = s.lv[l - 1];
  if (!rap_per_cell((int)F.parts.size(), F.maxcoarse, s.rap_cell_min)) return false;
  const PartLevel &pf = F.parts[p], &q = s.lv[l].parts[p];
  return pf.dstar >= 0 && !pf.rap_ng && q.dstar >= 0 && s.prm.pb_interp != SSAMG_PB_LUMP;
}

// Order in which the collapse sums of level l's part p take its entries: the
// order in which the Galerkin product forms a coarse row (perpendicular
// offsets (tb, ta) in the two other axes after the previous direction, then
// that direction's component), entry order where no product forms the level.
void weight_order(const Solver &s, int l, size_t p, int (&ord)[kMaxEnt]) {
  const PartLevel &q = s.lv[l].parts[p];
  const int nent = (int)q.pat.size();
  for (int e = 0; e < kMaxEnt; ++e) ord[e] = e < nent ? e : 0;
  if (l < 1) {
    // finest level: the off-center entries in entry order, then the center
    // (the order in which the finite-volume assembly forms a row)
    int k = 0;
    for (int e = 0; e < nent; ++e)
      if (e != q.center) ord[k++] = e;
    ord[k++] = q.center;
    return;
  }
  const PartLevel &pf = s.lv[l - 1].parts[p];
  if (pf.dstar < 0 || pf.rap_ng) return;
  const int ds = pf.dstar, ax = (ds + 1) % 3, bx = (ds + 2) % 3;
  auto stride = [](int a) { return a == 0 ? 1 : a == 1 ? 3 : 9; };
  int k = 0;
  for (int tb = -1; tb <= 1; ++tb)
    for (int ta = -1; ta <= 1; ++ta)
      for (int qd = -1; qd <= 1; ++qd) {
        const int e = pf.rap_cmap[(ta + 1) * stride(ax) + (tb + 1) * stride(bx) + (qd + 1) * stride(ds)];
        if (e >= 0) ord[k++] = e;
      }
  if (k != nent) throw Error(SSAMG_ERR_STATE, "internal: coarse stencil not covered by its Galerkin table");
}

void build_descs(const Solver &s, int l, std::vector<PartDesc<double>> &h64,
                 std::vector<PartDesc<float>> &h32) {
  const Level &V = s.lv[l];
  const bool mixed = s.prm.cycle_precision == SSAMG_FP32;
  int cyc[kMaxLg + 1], mv[kMaxLg + 1];
  for (int lg = 0; lg <= kMaxLg; ++lg) {
    const TuneRec r = tune_rec(s, l, lg);
    cyc[lg] = r.strips;
    mv[lg] = mixed ? (l == 0 ? r.strips_mv : 1) : r.strips;
  }
  h64.clear();
  h32.clear();
  for (size_t p = 0; p < V.parts.size(); ++p) {
    const PartLevel &q = V.parts[p];
    // mirror tables for the FP64 product (used only by its mirrored kernels)
    const bool sym = mirrored(s);
    h64.push_back(make_desc<double>(V, q, p, q.coef64, V.d_w64, V.d_uval64, V.d_rs64, mv, sym));
    h64.back().pblump = s.prm.pb_interp == SSAMG_PB_LUMP;
    weight_order(s, l, p, h64.back().wsum);
    h64.back().wfused = weights_fused(s, l, p) ? 1 : 0;
    const Problem &pr = *s.prob;
    h64.back().csum = l == 0 && q.dstar >= 0 && pr.fv_stencil && pr.d_csum &&
                              pr.metric_version == pr.coef_version && (int)pr.csum_off.size() == 3 * pr.nparts
                          ? pr.d_csum + pr.csum_off[3 * p + q.dstar]
                          : nullptr;
    if (mixed) h32.push_back(make_desc<float>(V, q, p, q.coef32, V.d_w32, V.d_uval32, V.d_rs32, cyc, false));
  }
}

// Shape of level l as the launch options see it (cycle precision, first level
// or not, and per part the box, stencil size and coarsening direction).
std::string level_sig(const Solver &s, int l) {
  const Level &V = s.lv[l];
  std::string k = (s.prm.cycle_precision == SSAMG_FP32 ? "f32" : "f64");
  k += l == 0 ? ":fine" : ":coarse";
  for (const auto &q : V.parts)
    k += ":" + std::to_string(q.n[0]) + "x" + std::to_string(q.n[1]) + "x" + std::to_string(q.n[2]) + "e" +
         std::to_string(q.pat.size()) + "d" + std::to_string(q.dstar);
  return k;
}

void drop_graph(Solver &s) {
  if (s.graph_exec) (void)hipGraphExecDestroy(s.graph_exec);
  if (s.graph) (void)hipGraphDestroy(s.graph);
  s.graph_exec = nullptr;
  s.graph = nullptr;
  s.graph_nrhs = 0;
}

}  // namespace

std::string tune_key(const Solver &s, int l, int lg) {
  return s.sig.at(l) + "|lg" + std::to_string(lg);
}

TuneRec tune_rec(const Solver &s, int l, int lg, bool *found) {
  if (found) *found = false;
  if (l < 0 || l >= (int)s.sig.size() || s.tune.empty()) return TuneRec{};
  auto it = s.tune.find(tune_key(s, l, lg));
  if (it == s.tune.end()) return TuneRec{};
  if (found) *found = true;
  return it->second;
}

void tune_store(Solver &s, int l, int lg, const TuneRec &r) {
  if (s.state < 1) throw Error(SSAMG_ERR_STATE, "launch options need the symbolic setup");
  if (l < 0 || l >= (int)s.lv.size()) throw Error(SSAMG_ERR_ARG, "level out of range");
  if (lg < 0 || lg > kMaxLg) throw Error(SSAMG_ERR_ARG, "batch width out of range");
  auto tri = [](int v) { return v >= -1 && v <= 1; };
  if (r.strips < 1 || r.strips > 64 || r.strips_mv < 1 || r.strips_mv > 64)
    throw Error(SSAMG_ERR_ARG, "strips must be in 1..64");
  if (!tri(r.cols4) || !tri(r.split) || !tri(r.cols4_mv))
    throw Error(SSAMG_ERR_ARG, "cols4, split and cols4_mv take -1, 0 or 1");
  const Level &V = s.lv[l];
  const bool mixed = s.prm.cycle_precision == SSAMG_FP32;
  const bool ok_cyc = mixed ? stencil_cols4_ok<float>(lg, V.maxent) : stencil_cols4_ok<double>(lg, V.maxent);
  if (r.cols4 == 1 && !ok_cyc)
    throw Error(SSAMG_ERR_ARG, "four columns per thread need a batch of 4 or more (and no FP64 27-point stencil)");
  if (r.cols4_mv == 1 && !stencil_cols4_ok<double>(lg, V.maxent))
    throw Error(SSAMG_ERR_ARG, "four columns per thread for the FP64 product need a batch of 4 or more "
                               "and at most 15-point stencils");
  s.tune[tune_key(s, l, lg)] = r;
  drop_graph(s);
  if (s.state >= 2) {
    std::vector<PartDesc<double>> h64;
    std::vector<PartDesc<float>> h32;
    build_descs(s, l, h64, h32);
    upload(s.lv[l].d_desc64, h64, s.stream);
    if (mixed) upload(s.lv[l].d_desc32, h32, s.stream);
    SSAMG_HIP(hipStreamSynchronize(s.stream));
  }
}

Solver::~Solver() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ws_owned && ws) (void)hipFree(ws);
  if (h_pin) (void)hipHostFree(h_pin);
  if (h_tab) (void)hipHostFree(h_tab);
  for (auto e : pev) (void)hipEventDestroy(e);
  if (ev_scal) (void)hipEventDestroy(ev_scal);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ---------------------------------------------------------------- symbolic

namespace {

// ---- host form of the coupling product, for the small coarse levels

// nonzeros of row `cell` of P (coarse cells and weight sources: -1 = 1.0, else
// an index into the level's weight buffer, wm block then wp block per part);
// the same cases as the device emitter
int host_prow(const SymPart *sp, int np, long long cell, int col[2], int src[2]) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sp[mid].off <= cell)
      lo = mid;
    else
      hi = mid - 1;
  }
  const SymPart &q = sp[lo];
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

// Structure and recipe of U_{l+1} from U_l (entries with row cells erow and
// columns ucol), as the device path forms them: every entry q emits a record
// for each pair of its rows' P nonzeros, a stable sort by coarse pair keeps the
// emission order within a pair, runs of equal pairs are the entries and runs
// of equal rows the stored rows.
struct HostCpl {
  std::vector<int> urow, uptr, ucol, erow, start, ck, ca, cb;
};

void host_coarse_coupling(const SymPart *sp, int np, const std::vector<int> &erow,
                          const std::vector<int> &ucol, int64_t nc, HostCpl &out) {
  out = HostCpl{};
  const size_t nnz = erow.size();
  if (nnz == 0) return;
  // the valid records in emission order (the device's invalid keys sort last
  // and are never read)
  std::vector<uint64_t> key, key2;
  std::vector<uint32_t> idx, idx2;
  std::vector<int> rk, ra, rb;
  key.reserve(4 * nnz);
  idx.reserve(4 * nnz);
  rk.reserve(4 * nnz);
  ra.reserve(4 * nnz);
  rb.reserve(4 * nnz);
  const uint64_t ncu = (uint64_t)nc;
  for (size_t q = 0; q < nnz; ++q) {
    int cf[2], sf[2], cg[2], sg[2];
    const int nf = host_prow(sp, np, erow[q], cf, sf);
    const int ng = host_prow(sp, np, ucol[q], cg, sg);
    for (int t = 0; t < 4; ++t) {
      const int a = t >> 1, b = t & 1;
      if (a < nf && b < ng) {
        const uint64_t k = (uint64_t)cf[a] * ncu + (uint64_t)cg[b];
        idx.push_back((uint32_t)rk.size());
        key.push_back(k);
        rk.push_back((int)q);
        ra.push_back(sf[a]);
        rb.push_back(sg[b]);
      }
    }
  }
  const size_t nvalid = key.size();
  if (nvalid == 0) return;
  // key order, ties in emission order (a stable sort), as the device forms
  // it: count the records of every coarse row, place them row by row in
  // emission order, then order each row by key with a stable insertion sort
  // (rows hold few records)
  {
    std::vector<int> rpos((size_t)nc + 1, 0);
    for (size_t i = 0; i < nvalid; ++i) ++rpos[(size_t)(key[i] / ncu) + 1];
    for (int64_t r = 0; r < nc; ++r) rpos[r + 1] += rpos[r];
    key2.resize(nvalid);
    idx2.resize(nvalid);
    std::vector<int> fillp(rpos.begin(), rpos.end() - 1);
    for (size_t i = 0; i < nvalid; ++i) {
      const size_t at = (size_t)fillp[(size_t)(key[i] / ncu)]++;
      key2[at] = key[i];
      idx2[at] = idx[i];
    }
    for (int64_t r = 0; r < nc; ++r)
      for (int64_t j = rpos[r] + 1; j < rpos[r + 1]; ++j) {
        const uint64_t k = key2[j];
        const uint32_t v = idx2[j];
        int64_t m = j - 1;
        for (; m >= rpos[r] && key2[m] > k; --m) {
          key2[m + 1] = key2[m];
          idx2[m + 1] = idx2[m];
        }
        key2[m + 1] = k;
        idx2[m + 1] = v;
      }
    key.swap(key2);
    idx.swap(idx2);
  }
  out.ck.resize(nvalid);
  out.ca.resize(nvalid);
  out.cb.resize(nvalid);
  for (size_t i = 0; i < nvalid; ++i) {
    const uint32_t r = idx[i];
    out.ck[i] = rk[r];
    out.ca[i] = ra[r];
    out.cb[i] = rb[r];
    const bool fnew = i == 0 || key[i] != key[i - 1];
    const bool frow = i == 0 || key[i] / ncu != key[i - 1] / ncu;
    if (fnew) {
      out.ucol.push_back((int)(key[i] % ncu));
      out.erow.push_back((int)(key[i] / ncu));
      out.start.push_back((int)i);
    }
    if (frow) {
      out.urow.push_back((int)(key[i] / ncu));
      out.uptr.push_back((int)out.ucol.size() - 1);
    }
  }
  out.start.push_back((int)nvalid);
  out.uptr.push_back((int)out.ucol.size());
}

// host k_ublk: first stored row of every block of a grid-over-cells launch
// (1 << lg rhs) and that row's first entry
void host_ublk(const SymPart *sp, int np, int lg, const long long *boff, const std::vector<int> &urow,
               const std::vector<int> &uptr, int *out) {
  const int nrow = (int)urow.size();
  for (int p = 0; p < np; ++p) {
    const SymPart &q = sp[p];
    const long long cpb = kBlock >> lg;
    const long long nchunk = (q.ncell + cpb - 1) / cpb;
    for (long long b = 0; b <= nchunk; ++b) {
      const long long first = q.off + (b * cpb < q.ncell ? b * cpb : q.ncell);
      const int lo = (int)(std::lower_bound(urow.begin(), urow.end(), (int)first) - urow.begin());
      out[2 * (boff[p] + b)] = lo;
      out[2 * (boff[p] + b) + 1] = nrow > 0 ? uptr[lo] : 0;
    }
  }
}

// Structure of every coarse coupling matrix (device: emit, sort, segment;
// host for the small coarse levels) and the per-block row ranges the stencil
// kernels use, for all levels.
void symbolic_couplings(Solver &s, int lgmax) {
  hipStream_t st = s.stream;
  const int L = (int)s.lv.size();
  const int np = (int)s.lv[0].parts.size();
  // the structured Galerkin tables (host) of levels 0 .. L-2, built two levels
  // at a time while the device forms a coupling product, the rest at the end
  int next_tab = 0;
  auto tables = [&](int nlev) {
    for (; nlev > 0 && next_tab < L - 1; --nlev, ++next_tab)
      for (int p = 0; p < np; ++p)
        build_rap_table(s.lv[next_tab].parts[p], s.lv[next_tab + 1].parts[p].pat,
                        nongalerkin(s, s.lv[next_tab].parts[p]));
  };
  while ((int)s.store.size() < L) s.store.emplace_back(new LevelStore());
  // one upload: SymPart tables of all levels and the block offsets of ublk
  std::vector<SymPart> sp;
  std::vector<long long> boff;
  std::vector<size_t> sp_at(L), boff_at(L * (kMaxLg + 1));
  for (int l = 0; l < L; ++l) {
    Level &V = s.lv[l];
    sp_at[l] = sp.size();
    for (auto &q : V.parts) {
      SymPart x{};
      for (int a = 0; a < 3; ++a) {
        x.n[a] = q.n[a];
        x.cn[a] = q.cn[a];
        x.fn[a] = q.fn[a];
      }
      x.dstar = q.dstar;
      x.off = q.off;
      x.ncell = q.ncell;
      x.coff = q.coff;
      x.nf = q.nf;
      x.wofs = q.wofs;
      sp.push_back(x);
    }
    for (int lg = 0; lg <= kMaxLg; ++lg) {
      V.ublk_off[lg].assign(np, 0);
      boff_at[l * (kMaxLg + 1) + lg] = boff.size();
      if (lg > lgmax) continue;
      const int64_t cpb = kBlock >> lg;
      int64_t tot = 0;
      for (int p = 0; p < np; ++p) {
        V.ublk_off[lg][p] = tot;
        boff.push_back(tot);
        tot += (V.parts[p].ncell + cpb - 1) / cpb + 1;
      }
      V.ublk_len[lg] = tot;
    }
  }
  const size_t sp_bytes = align_up(sp.size() * sizeof(SymPart));
  s.symtab.reserve(sp_bytes + boff.size() * sizeof(long long) + 256);
  std::vector<char> stage(sp_bytes + boff.size() * sizeof(long long));
  std::memcpy(stage.data(), sp.data(), sp.size() * sizeof(SymPart));
  if (!boff.empty()) std::memcpy(stage.data() + sp_bytes, boff.data(), boff.size() * sizeof(long long));
  SSAMG_HIP(hipMemcpyAsync(s.symtab.p, stage.data(), stage.size(), hipMemcpyHostToDevice, st));
  const SymPart *d_sp = (const SymPart *)s.symtab.p;
  const long long *d_boff = (const long long *)((char *)s.symtab.p + sp_bytes);
  {
    // entry -> row cell of the input couplings
    Level &V0 = s.lv[0];
    DevBuf &e0 = s.store[0]->cpl.erow;
    e0.reserve((size_t)std::max<int64_t>(V0.nnz, 1) * sizeof(int));
    launch_entry_rows(V0.nrow, V0.d_urow, V0.d_uptr, (int *)e0.p, st);
    V0.d_erow = (int *)e0.p;
  }
  // levels from lh on are formed on the host (their inputs shrink below
  // host_sym records); lh = L: none
  int lh = L;
  std::vector<HostCpl> hc(L);
  {
    std::vector<int> h_erow, h_ucol;
    for (int l = 0; l + 1 < L; ++l) {
      Level &V = s.lv[l], &C = s.lv[l + 1];
      if (lh == L && 4 * V.nnz <= s.host_sym) {
        lh = l + 1;
        h_erow.resize((size_t)V.nnz);
        h_ucol.resize((size_t)V.nnz);
        if (V.nnz > 0) {
          SSAMG_HIP(hipMemcpyAsync(h_erow.data(), V.d_erow, (size_t)V.nnz * sizeof(int), hipMemcpyDeviceToHost, st));
          SSAMG_HIP(hipMemcpyAsync(h_ucol.data(), V.d_ucol, (size_t)V.nnz * sizeof(int), hipMemcpyDeviceToHost, st));
          SSAMG_HIP(hipStreamSynchronize(st));
        }
      }
      if (lh <= l + 1) {
        HostCpl &o = hc[l + 1];
        host_coarse_coupling(sp.data() + sp_at[l], np, h_erow, h_ucol, C.N, o);
        C.nnz = (int64_t)o.ucol.size();
        C.nrow = (int)o.urow.size();
        C.ncontrib = (int64_t)o.ck.size();
        h_erow = o.erow;
        h_ucol = o.ucol;
        continue;
      }
      CouplingStore &cs = s.store[l + 1]->cpl;
      int64_t nnz = 0;
      int nrow = 0;
      coarse_coupling_device(s.scratch, d_sp + sp_at[l], np, V.nnz, V.d_erow, V.d_ucol, C.N, cs, nnz, nrow,
                             st, [&] { tables(2); });
      C.nnz = nnz;
      C.nrow = nrow;
      C.ncontrib = nnz ? cs.ncontrib : 0;
      C.d_urow = nnz ? (int *)cs.urow.p : nullptr;
      C.d_uptr = nnz ? (int *)cs.uptr.p : nullptr;
      C.d_ucol = nnz ? (int *)cs.ucol.p : nullptr;
      C.d_erow = nnz ? (int *)cs.erow.p : nullptr;
      C.d_uc_start = nnz ? (int *)cs.start.p : nullptr;
      C.d_uc_k = nnz ? (int *)cs.ck.p : nullptr;
      C.d_uc_a = nnz ? (int *)cs.ca.p : nullptr;
      C.d_uc_b = nnz ? (int *)cs.cb.p : nullptr;
    }
  }
  tables(L);
  // host-formed levels: arrays and block tables in one buffer, one copy
  if (lh < L) {
    std::vector<int> stage;
    struct Ofs { size_t a[8]; size_t ub[kMaxLg + 1]; };
    std::vector<Ofs> ofs(L);
    for (int l = lh; l < L; ++l) {
      HostCpl &o = hc[l];
      const std::vector<int> *arr[8] = {&o.urow, &o.uptr, &o.ucol, &o.erow, &o.start, &o.ck, &o.ca, &o.cb};
      for (int k = 0; k < 8; ++k) {
        ofs[l].a[k] = stage.size();
        stage.insert(stage.end(), arr[k]->begin(), arr[k]->end());
        stage.resize((stage.size() + 63) & ~size_t(63));   // 256-byte aligned pieces
      }
      for (int lg = 0; lg <= kMaxLg; ++lg) {
        ofs[l].ub[lg] = stage.size();
        if (lg > lgmax) continue;
        std::vector<int> ub((size_t)s.lv[l].ublk_len[lg] * 2);
        host_ublk(sp.data() + sp_at[l], np, lg, boff.data() + boff_at[l * (kMaxLg + 1) + lg], o.urow, o.uptr,
                  ub.data());
        stage.insert(stage.end(), ub.begin(), ub.end());
        stage.resize((stage.size() + 63) & ~size_t(63));
      }
    }
    s.host_cpl.reserve(stage.size() * sizeof(int) + 256);
    int *base = (int *)s.host_cpl.p;
    SSAMG_HIP(hipMemcpyAsync(base, stage.data(), stage.size() * sizeof(int), hipMemcpyHostToDevice, st));
    for (int l = lh; l < L; ++l) {
      Level &C = s.lv[l];
      const bool any = C.nnz > 0;
      C.d_urow = any ? base + ofs[l].a[0] : nullptr;
      C.d_uptr = any ? base + ofs[l].a[1] : nullptr;
      C.d_ucol = any ? base + ofs[l].a[2] : nullptr;
      C.d_erow = any ? base + ofs[l].a[3] : nullptr;
      C.d_uc_start = any ? base + ofs[l].a[4] : nullptr;
      C.d_uc_k = any ? base + ofs[l].a[5] : nullptr;
      C.d_uc_a = any ? base + ofs[l].a[6] : nullptr;
      C.d_uc_b = any ? base + ofs[l].a[7] : nullptr;
      for (int lg = 0; lg <= kMaxLg; ++lg) C.d_ublk[lg] = lg <= lgmax ? base + ofs[l].ub[lg] : nullptr;
    }
    // the host vectors must outlive the asynchronous copy
    SSAMG_HIP(hipStreamSynchronize(st));
  }
  // block tables of the device-formed levels, all (level, lg) pairs in few launches
  {
    UblkJobs jobs{};
    int64_t nbx = 1;
    auto flush = [&] {
      launch_ublk(d_sp, np, d_boff, jobs, nbx, st);
      jobs.n = 0;
      nbx = 1;
    };
    for (int l = 0; l < lh; ++l) {
      Level &V = s.lv[l];
      int64_t maxchunk = 0;
      for (auto &q : V.parts) maxchunk = std::max<int64_t>(maxchunk, q.ncell);
      for (int lg = 0; lg <= kMaxLg; ++lg) {
        V.d_ublk[lg] = nullptr;
        if (lg > lgmax) continue;
        DevBuf &ub = s.store[l]->ublk[lg];
        ub.reserve((size_t)V.ublk_len[lg] * 2 * sizeof(int));
        V.d_ublk[lg] = (int *)ub.p;
        const int64_t chunks = (maxchunk + (kBlock >> lg) - 1) / (kBlock >> lg);
        nbx = std::max<int64_t>(nbx, (chunks + 1 + kBlock - 1) / kBlock);
        UblkJob &j = jobs.j[jobs.n++];
        j.urow = V.d_urow;
        j.uptr = V.d_uptr;
        j.out = (int *)ub.p;
        j.nrow = V.nrow;
        j.lg = lg;
        j.spat = (int)sp_at[l];
        j.boffat = (int)boff_at[l * (kMaxLg + 1) + lg];
        if (jobs.n == kUblkJobs) flush();
      }
    }
    flush();
  }
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipStreamSynchronize(st));
}

}  // namespace


void setup_symbolic(Solver &s) {
  const auto t0 = std::chrono::steady_clock::now();
  Problem &pr = *s.prob;
  const int np = pr.nparts;
  for (int p = 0; p < np; ++p) {
    if (vol(pr.dims[p]) <= 0) throw Error(SSAMG_ERR_STATE, "box of part " + std::to_string(p) + " not set");
    if (pr.stencil[p].empty() || !pr.coef_set[p] || !pr.coef[p])
      throw Error(SSAMG_ERR_STATE, "coefficients of part " + std::to_string(p) + " not set");
  }
  if (pr.ncell_total() >= (int64_t(1) << 31)) throw Error(SSAMG_ERR_UNSUPPORTED, "more than 2^31 cells");
  if (s.graph_exec) {
    (void)hipGraphExecDestroy(s.graph_exec);
    s.graph_exec = nullptr;
  }
  if (s.graph) {
    (void)hipGraphDestroy(s.graph);
    s.graph = nullptr;
  }
  if (s.ws_owned && s.ws) (void)hipFree(s.ws);
  s.ws = nullptr;
  s.ws_owned = false;
  s.lv.clear();
  s.state = 0;

  // level 0 from the problem
  Level L0;
  int64_t off = 0;
  for (int p = 0; p < np; ++p) {
    PartLevel q;
    q.n = pr.dims[p];
    q.off = off;
    q.ncell = vol(q.n);
    off += q.ncell;
    q.pat = pr.stencil[p];
    q.center = pr.center[p];
    q.coef64 = pr.coef[p];
    for (int f = 0; f < 6; ++f)
      if (pr.faces[p][f] == SSAMG_FACE_PART) q.faces |= 1 << f;
    L0.parts.push_back(q);
  }
  L0.N = off;
  L0.nrow = (int)pr.urow.size();
  L0.nnz = (int64_t)pr.ucol.size();
  L0.d_urow = pr.d_urow;
  L0.d_uptr = pr.d_uptr;
  L0.d_ucol = pr.d_ucol;

  // direction sums c_d on the device (the only round trip of the symbolic setup)
  {
    std::vector<PartDesc<double>> hd;
    int maxcell = 0;
    const int plain[kMaxLg + 1] = {1, 1, 1, 1, 1, 1};
    for (size_t p = 0; p < L0.parts.size(); ++p) {
      const PartLevel &q = L0.parts[p];
      hd.push_back(make_desc<double>(L0, q, p, q.coef64, nullptr, nullptr, nullptr, plain));
      maxcell = std::max<int64_t>(maxcell, q.ncell);
    }
    s.wsum_buf.reserve(np * sizeof(PartDesc<double>) + (size_t)np * 256 * 3 * 8 + np * 3 * 8 + 1024);
    char *base = (char *)s.wsum_buf.p;
    PartDesc<double> *dd = (PartDesc<double> *)base;
    double *part = (double *)(base + align_up(np * sizeof(PartDesc<double>)));
    double *out = part + (size_t)np * 256 * 3;
    if (pr.d_mpart && pr.metric_version == pr.coef_version) {
      // the finite-volume assembly formed the partial sums with the coefficients
      launch_wsum_final(pr.d_mpart, np, pr.mpart_nb, out, s.stream);
    } else {
      SSAMG_HIP(hipMemcpyAsync(dd, hd.data(), np * sizeof(PartDesc<double>), hipMemcpyHostToDevice, s.stream));
      launch_wsum(dd, np, maxcell, part, out, s.stream);
    }
    SSAMG_HIP(hipGetLastError());
    s.cd.assign((size_t)np * 3, 0.0);
    SSAMG_HIP(hipMemcpyAsync(s.cd.data(), out, np * 3 * sizeof(double), hipMemcpyDeviceToHost, s.stream));
    SSAMG_HIP(hipStreamSynchronize(s.stream));
  }
  const auto t_w = std::chrono::steady_clock::now();

  // W (Section 3.1) and Algorithm 1
  const int ndim = pr.ndim;
  int lgmax = 0;
  while ((1 << lgmax) < s.prm.max_nrhs) ++lgmax;
  std::vector<std::array<double, 3>> W(np);
  for (int p = 0; p < np; ++p) {
    double cmax = -kInf;
    for (int d = 0; d < ndim; ++d) cmax = std::max(cmax, s.cd[3 * p + d]);
    for (int d = 0; d < 3; ++d) {
      const double c = s.cd[3 * p + d];
      W[p][d] = (d < ndim && c > 0.0 && cmax > 0.0) ? std::sqrt(cmax / c) : kInf;
    }
  }
  std::vector<int> all_d(ndim);
  std::iota(all_d.begin(), all_d.end(), 0);
  s.lv.push_back(std::move(L0));
  while (true) {
    Level &L = s.lv.back();
    const int l = (int)s.lv.size() - 1;
    bool all_one = true;
    for (auto &q : L.parts) all_one = all_one && q.ncell == 1;
    // the hybrid tail (Section 3.5) ends the hierarchy at its switch level
    const int lmax = s.prm.hybrid_level > 0 ? std::min(s.prm.max_levels, s.prm.hybrid_level + 1)
                                            : s.prm.max_levels;
    const bool last = all_one || l >= lmax - 1 ||
                      (s.prm.min_coarse_size > 0 && L.N < s.prm.min_coarse_size);
    Level C;
    int64_t coff = 0;
    for (int p = 0; p < np; ++p) {
      PartLevel &q = L.parts[p];
      std::vector<int> cand;
      for (int d = 0; d < ndim; ++d)
        if (q.n[d] > 1) cand.push_back(d);
      int ds = -1;
      if (last || cand.empty()) {
        q.omega = relax_weight(W[p], argmin_tied(W[p], all_d), ndim);
      } else {
        ds = argmin_tied(W[p], cand);
        q.omega = relax_weight(W[p], ds, ndim);
        W[p][ds] *= 2.0;
      }
      if (s.prm.omega > 0.0) q.omega = s.prm.omega;
      q.dstar = ds;
      q.cn = q.n;
      q.fn = {0, 0, 0};
      q.nf = 0;
      if (ds >= 0) {
        q.cn[ds] = (q.n[ds] + 1) / 2;
        q.fn = q.n;
        q.fn[ds] = q.n[ds] / 2;
        q.nf = vol(q.fn);
      }
      q.cncell = vol(q.cn);
      q.coff = coff;
      coff += q.cncell;
      if (!last) {
        PartLevel c;
        c.n = q.cn;
        c.off = q.coff;
        c.ncell = q.cncell;
        c.faces = q.faces;
        c.pat = coarse_pattern(q.pat, ds);
        // non-Galerkin option: a star stencil keeps its star pattern
        if (nongalerkin(s, q)) {
          std::vector<std::array<int, 3>> star;
          for (const auto &t : c.pat)
            if ((t[0] != 0) + (t[1] != 0) + (t[2] != 0) <= 1) star.push_back(t);
          c.pat = std::move(star);
        }
        c.center = index_of(c.pat, {0, 0, 0});
        C.parts.push_back(std::move(c));   // Galerkin table: built in symbolic_couplings
      }
    }
    // weight buffer layout of this level
    int64_t w = 0;
    for (auto &q : L.parts) {
      q.wofs = w;
      w += 2 * q.nf;
    }
    L.nw = w;
    L.maxcell = L.maxcoarse = L.maxf = L.maxent = 0;
    for (auto &q : L.parts) {
      L.maxcell = std::max<int64_t>(L.maxcell, q.ncell);
      L.maxcoarse = std::max<int64_t>(L.maxcoarse, q.cncell);
      L.maxf = std::max<int64_t>(L.maxf, q.nf);
      L.maxent = std::max<int>(L.maxent, (int)q.pat.size());
    }
    if (last) break;
    C.N = coff;
    s.lv.push_back(std::move(C));
  }
  // skip option (Section 3.4): no relaxation where a part coarsens along the
  // same direction as n_d levels above
  for (int l = 0; l < (int)s.lv.size(); ++l)
    for (size_t p = 0; p < s.lv[l].parts.size(); ++p) {
      const int ds = s.lv[l].parts[p].dstar;
      s.lv[l].parts[p].skip =
          s.prm.skip && l >= ndim && ds >= 0 && ds == s.lv[l - ndim].parts[p].dstar;
    }
  if (s.prm.hybrid_level > 0 && s.lv.back().N > kDenseMax)
    throw Error(SSAMG_ERR_UNSUPPORTED, "the hybrid tail solves at most " + std::to_string(kDenseMax) +
                                           " unknowns exactly; level " + std::to_string(s.lv.size() - 1) +
                                           " has " + std::to_string(s.lv.back().N) + " (choose a coarser level)");
  if (s.prm.hybrid_level <= 0 && s.prm.coarse == SSAMG_COARSE_DIRECT && s.lv.back().N > kDirectMax)
    throw Error(SSAMG_ERR_UNSUPPORTED, "the direct coarsest solve takes at most " +
                                           std::to_string(kDirectMax) + " unknowns; the coarsest level has " +
                                           std::to_string(s.lv.back().N));
  const auto t_alg = std::chrono::steady_clock::now();
  symbolic_couplings(s, lgmax);
  const auto t_u = std::chrono::steady_clock::now();
  // collapse level: the first level >= 1 of at most collapse_cells cells, when
  // it is not the coarsest
  s.lk = -1;
  if (s.collapse_cells > 0 && s.prm.hybrid_level <= 0)
    for (int l = 1; l + 1 < (int)s.lv.size(); ++l)
      if (s.lv[l].N <= s.collapse_cells && s.lv[l].N <= kTailMax) {
        s.lk = l;
        break;
      }
  // sizing pass of the workspace
  Carver cv;
  carve(s, cv);
  s.ws_bytes = cv.off + 256;
  s.sig.clear();
  for (int l = 0; l < (int)s.lv.size(); ++l) s.sig.push_back(level_sig(s, l));
  s.state = 1;
  s.t_sym = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  s.t_num = 0.0;
  if (s.verbose) {
    size_t unnz = 0, contrib = 0;
    for (auto &L : s.lv) {
      unnz += L.nnz;
      contrib += L.ncontrib;
    }
    auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    fprintf(stderr, "[ssamg] symbolic setup: %.3f ms (metric %.3f, algorithm 1 + tables %.3f, "
            "couplings %.3f), %zu levels, %zu coupling entries, %zu Galerkin contributions, "
            "workspace %zu bytes\n",
            ms(t0, std::chrono::steady_clock::now()), ms(t0, t_w), ms(t_w, t_alg), ms(t_alg, t_u),
            s.lv.size(), unnz, contrib, s.ws_bytes);
  }
}

namespace {

// Assign every device buffer of the hierarchy from one workspace (base =
// nullptr: sizing only).  The order of takes must not depend on base.  The
// host-built tables come first, in one contiguous segment.
void carve(Solver &s, Carver &cv) {
  const bool mixed = s.prm.cycle_precision == SSAMG_FP32;
  const int L = (int)s.lv.size();
  const int nr = s.prm.max_nrhs;
  const int64_t N0 = s.lv[0].N;
  cv.off = align_up(cv.off);
  cv.tab_begin = cv.off;
  // TailLevel records of all levels, contiguous (the tail kernel walks them)
  const size_t tail_size = mixed ? sizeof(TailLevel<float>) : sizeof(TailLevel<double>);
  void *tail_all = cv.take<char>(tail_size * L);
  void *ctail_all = cv.take<char>(tail_size * L);   // the records the cycle reads (collapse level changed)
  for (int l = 0; l < L; ++l) {
    Level &V = s.lv[l];
    V.d_desc64 = cv.take<PartDesc<double>>(V.parts.size());
    V.d_desc32 = mixed ? cv.take<PartDesc<float>>(V.parts.size()) : nullptr;
    V.d_rapdesc = l < L - 1 ? cv.take<RapDesc>(V.parts.size()) : nullptr;
    V.d_tail = (char *)tail_all + (size_t)l * tail_size;
    V.d_ctail = (char *)ctail_all + (size_t)l * tail_size;
  }
  cv.off = align_up(cv.off);
  cv.tab_end = cv.off;
  // device-produced data
  s.r = cv.take<double>((size_t)N0 * nr);
  s.z = cv.take<double>((size_t)N0 * nr);
  s.p = cv.take<double>((size_t)N0 * nr);
  s.q = cv.take<double>((size_t)N0 * nr);
  s.partial = cv.take<double>((size_t)2 * kRedBlocks * kMaxRhs);
  {
    // partial sums of the dot products formed by level-0 kernels (p.q by the
    // FP64 product; r.z and z.q by the last sweep of a batched cycle): two
    // sets, widest case
    int64_t slots = 0;
    for (int lg = 0; (1 << lg) <= s.prm.max_nrhs; ++lg)
      slots = std::max<int64_t>(slots, (int64_t)s.lv[0].parts.size() * dot_slots(s.lv[0].maxcell, lg) << lg);
    s.dotp = slots > 0 ? cv.take<double>((size_t)2 * slots) : nullptr;
  }
  s.scal = cv.take<double>((size_t)kScalSlots * kMaxRhs);
  s.active = cv.take<int>(kMaxRhs);
  s.flag = cv.take<int>(1);
  const bool hybrid = s.prm.hybrid_level > 0;
  s.lv.back().d_ainv = !hybrid && s.prm.coarse == SSAMG_COARSE_DIRECT
                           ? cv.take<double>((size_t)s.lv.back().N * s.lv.back().N)
                           : nullptr;
  // hybrid tail: the coarsest level's dense inverse (padded), the Gauss-Jordan
  // scratch (transposed column panel, pivot block inverse) and the partial
  // sums of the applied product
  {
    const int64_t nc = s.lv.back().N, npad = hybrid ? dense_pad(nc) : 0;
    s.d_hyb = hybrid ? cv.take<double>((size_t)npad * npad) : nullptr;
    s.d_hyb_pt = hybrid ? cv.take<double>((size_t)64 * npad) : nullptr;
    s.d_hyb_dinv = hybrid ? cv.take<double>(64 * 64) : nullptr;
    s.d_hyb_part = hybrid ? cv.take<double>((size_t)dense_apply_chunks(nc) * nc * nr) : nullptr;
  }
  for (int l = 0; l < L; ++l)
    s.lv[l].d_mcyc = l == s.lk ? cv.take<double>((size_t)s.lv[l].N * s.lv[l].N) : nullptr;
  for (int l = 0; l < L; ++l) {
    Level &V = s.lv[l];
    const bool cyc32 = mixed && l < L - 1;
    V.cycle32 = mixed;   // the coarsest level of a mixed cycle keeps FP32 vectors
    for (auto &q : V.parts) {
      if (l > 0) q.coef64 = cv.take<double>((size_t)q.pat.size() * q.ncell);
      q.coef32 = cyc32 ? cv.take<float>((size_t)q.pat.size() * q.ncell) : nullptr;
    }
    V.d_w64 = l < L - 1 ? cv.take<double>(V.nw) : nullptr;
    V.d_w32 = (cyc32 && l < L - 1) ? cv.take<float>(V.nw) : nullptr;
    const size_t nnz = (size_t)V.nnz;
    V.d_uval64 = l == 0 ? s.prob->d_uval : cv.take<double>(nnz);
    V.d_uval32 = cyc32 ? cv.take<float>(nnz) : nullptr;
    V.d_rs64 = cv.take<double>((size_t)V.N);
    V.d_rs32 = cyc32 ? cv.take<float>((size_t)V.N) : nullptr;
    if (l >= 1 && l < L - 1 && V.N <= kTailMax) {   // pack of the coarse-end kernel
      const size_t n = (size_t)V.N, nc = (size_t)s.lv[l + 1].N, w = (size_t)V.maxent;
      V.d_pk_nb = cv.take<int>(w * n);
      V.d_pk_pi = cv.take<int>(2 * n);
      V.d_pk_ri = cv.take<int>(3 * nc);
      V.d_pk_row = cv.take<int>(n);
      if (mixed) {
        V.d_pk_ca = cv.take<float>(w * n);
        V.d_pk_pw = cv.take<float>(2 * n);
        V.d_pk_rw = cv.take<float>(2 * nc);
      } else {
        V.d_pk_ca = cv.take<double>(w * n);
        V.d_pk_pw = cv.take<double>(2 * n);
        V.d_pk_rw = cv.take<double>(2 * nc);
      }
    } else {
      V.d_pk_nb = V.d_pk_pi = V.d_pk_ri = V.d_pk_row = nullptr;
      V.d_pk_ca = V.d_pk_pw = V.d_pk_rw = nullptr;
    }
    const size_t nv = (size_t)V.N * nr;
    if (mixed) {
      V.vb = cv.take<float>(nv);
      V.vx = cv.take<float>(nv);
      V.vt = cv.take<float>(nv);
    } else {
      V.vb = l == 0 ? (void *)s.r : (void *)cv.take<double>(nv);
      V.vx = cv.take<double>(nv);
      V.vt = l == 0 ? (void *)s.z : (void *)cv.take<double>(nv);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- numeric

void setup_numeric(Solver &s, void *ws, size_t bytes) {
  if (s.state < 1) throw Error(SSAMG_ERR_STATE, "setup_symbolic must come first");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  if (ws) {
    if (bytes < s.ws_bytes) throw Error(SSAMG_ERR_ARG, "workspace smaller than ssamg_workspace_bytes");
    if (s.ws_owned && s.ws) (void)hipFree(s.ws);
    s.ws = ws;
    s.ws_owned = false;
  } else if (!s.ws || !s.ws_owned) {
    s.ws = dev_alloc<char>(s.ws_bytes);
    s.ws_owned = true;
  }
  if (s.graph_exec) {
    (void)hipGraphExecDestroy(s.graph_exec);
    s.graph_exec = nullptr;
  }
  if (s.graph) {
    (void)hipGraphDestroy(s.graph);
    s.graph = nullptr;
  }
  Carver cv;
  cv.base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(s.ws) + 255) & ~uintptr_t(255));
  carve(s, cv);
  const int L = (int)s.lv.size();
  const bool mixed = s.prm.cycle_precision == SSAMG_FP32;
  // every host-built table goes up in one copy
  // staged in pinned memory, so that the copy runs asynchronously; a copy of
  // an earlier call that did not end normally is waited for first
  const size_t tab_bytes = cv.tab_end - cv.tab_begin;
  if (s.h_tab_busy) {
    SSAMG_HIP(hipStreamSynchronize(st));
    s.h_tab_busy = false;
  }
  if (s.h_tab_cap < tab_bytes) {
    if (s.h_tab) (void)hipHostFree(s.h_tab);
    s.h_tab = nullptr;
    s.h_tab_cap = 0;
    SSAMG_HIP(hipHostMalloc(&s.h_tab, tab_bytes + 4096));
    s.h_tab_cap = tab_bytes + 4096;
  }
  char *stage = (char *)s.h_tab;
  std::memset(stage, 0, tab_bytes);
  auto put = [&](const void *dst, const void *src, size_t nbytes) {
    if (!nbytes) return;
    const size_t at = (size_t)((const char *)dst - cv.base) - cv.tab_begin;
    if (at + nbytes > tab_bytes) throw Error(SSAMG_ERR_STATE, "internal: table outside its segment");
    std::memcpy(stage + at, src, nbytes);
  };
  auto putv = [&](const void *dst, const auto &v) { put(dst, v.data(), v.size() * sizeof(v[0])); };
  for (int l = 0; l < L; ++l) {
    Level &V = s.lv[l];
    std::vector<PartDesc<double>> h64;
    std::vector<PartDesc<float>> h32;
    std::vector<RapDesc> hr;
    build_descs(s, l, h64, h32);
    for (size_t p = 0; p < V.parts.size(); ++p) {
      PartLevel &q = V.parts[p];
      if (l < L - 1) {
        RapDesc r{};
        r.out = s.lv[l + 1].parts[p].coef64;
        r.out32 = mixed && l + 1 < L - 1 ? s.lv[l + 1].parts[p].coef32 : nullptr;
        // the one-thread-per-coarse-cell kernel reads every coefficient of the
        // level: it also forms the L1 row sums and, on the finest level of a
        // mixed-precision cycle, the FP32 copy
        if (rap_per_cell((int)V.parts.size(), V.maxcoarse, s.rap_cell_min)) {
          r.l1 = s.prm.relax == SSAMG_RELAX_L1_JACOBI ? V.d_rs64 + q.off : nullptr;
          r.fine32 = l == 0 && mixed ? q.coef32 : nullptr;
        }
        r.nent = q.rap_nent;
        r.ng = q.rap_ng ? 1 : 0;
        r.wdir = -1;
        if (weights_fused(s, l + 1, p)) {
          const Level &C = s.lv[l + 1];
          const PartLevel &qc = C.parts[p];
          r.wdir = qc.dstar;
          r.wfaces = qc.faces;
          for (int a = 0; a < 3; ++a) r.wfn[a] = qc.fn[a];
          r.wm = C.d_w64 + qc.wofs;
          r.wp = C.d_w64 + qc.wofs + qc.nf;
          r.wm32 = mixed && C.d_w32 ? C.d_w32 + qc.wofs : nullptr;
          r.wp32 = mixed && C.d_w32 ? C.d_w32 + qc.wofs + qc.nf : nullptr;
          r.wflag = s.flag;
        }
        for (int o = 0; o < 27; ++o) {
          r.fmap[o] = q.rap_fmap[o];
          r.cmap[o] = q.rap_cmap[o];
          r.cofs[o] = q.rap_cofs[o];
        }
        hr.push_back(r);
      }
    }
    putv(V.d_desc64, h64);
    if (mixed) putv(V.d_desc32, h32);
    if (l < L - 1) putv(V.d_rapdesc, hr);
    // the levels' TailLevel records sit one after another in the workspace
    // only if consecutive takes are adjacent; they are written per level and
    // the tail kernel walks them through this level's pointer
    {
      auto rec = [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        TailLevel<T> t{};
        t.desc = mixed ? (const PartDesc<T> *)V.d_desc32 : (const PartDesc<T> *)V.d_desc64;
        t.ncell = V.N;
        t.nnext = l + 1 < L ? s.lv[l + 1].N : 0;
        t.np = (int)V.parts.size();
        t.nrow = V.nrow;
        t.nnz = (int)V.nnz;
        t.nw = V.maxent;
        t.urow = V.d_urow;
        t.uptr = V.d_uptr;
        t.ucol = V.d_ucol;
        t.uval = mixed ? (const T *)V.d_uval32 : (const T *)V.d_uval64;
        t.vb = (T *)V.vb;
        t.vt = (T *)V.vt;
        t.rs = mixed ? (const T *)V.d_rs32 : (const T *)V.d_rs64;
        t.rs64 = V.d_rs64;
        t.ainv = V.d_ainv;
        t.ndirect = V.d_ainv ? (int)V.N : 0;
        t.packed = V.d_pk_nb != nullptr;
        t.nb = V.d_pk_nb;
        t.ca = (T *)V.d_pk_ca;
        t.pi = V.d_pk_pi;
        t.pw = (T *)V.d_pk_pw;
        t.ri = V.d_pk_ri;
        t.rw = (T *)V.d_pk_rw;
        t.rowof = V.d_pk_row;
        put(V.d_tail, &t, sizeof(t));
        if (l == s.lk) {   // the cycle ends here: the collapsed operator as a direct solve
          t.ndirect = (int)V.N;
          t.ainv = V.d_mcyc;
          t.colmajor = 1;
        }
        put(V.d_ctail, &t, sizeof(t));
      };
      if (mixed)
        rec((float *)nullptr);
      else
        rec((double *)nullptr);
    }
  }
  if (tab_bytes) {
    s.h_tab_busy = true;
    SSAMG_HIP(hipMemcpyAsync(cv.base + cv.tab_begin, stage, tab_bytes, hipMemcpyHostToDevice, st));
  }
  SSAMG_HIP(hipMemsetAsync(s.flag, 0, sizeof(int), st));
  const auto t1 = std::chrono::steady_clock::now();
  // finest-level FP32 copies; coarser ones are written by the kernels below
  // per-cell smoother factors: omega_p / a_ii, or factor / sum_j |a_ij|
  const bool l1 = s.prm.relax == SSAMG_RELAX_L1_JACOBI;
  // levels whose Galerkin product runs one thread per coarse cell: that kernel
  // writes their L1 row sums (stencil part) and the finest FP32 copy
  auto fused = [&](int l) {
    return l < L - 1 && rap_per_cell((int)s.lv[l].parts.size(), s.lv[l].maxcoarse, s.rap_cell_min);
  };
  if (mixed && L > 1) {
    Level &V = s.lv[0];
    // otherwise the L1 factor pass writes them as it reads the coefficients
    if (!l1 && !fused(0))
      for (auto &q : V.parts) launch_cast_d2f(q.coef64, q.coef32, (int64_t)q.pat.size() * q.ncell, st);
    launch_cast_d2f(V.d_uval64, V.d_uval32, V.nnz, st);
  }
  const double l1_factor = s.prm.omega > 0.0 ? s.prm.omega : 1.5;
  auto smoother_scale = [&](int l) {
    Level &V = s.lv[l];
    float *rs32 = mixed && l < L - 1 ? V.d_rs32 : nullptr;
    launch_smoother_scale(l1, V.d_desc64, (int)V.parts.size(), V.maxcell, V.N, V.nrow, V.d_urow,
                          V.d_uptr, V.d_uval64, l1_factor, V.d_rs64, rs32, s.flag, st,
                          l == 0 && mixed && L > 1 && !fused(0) ? V.d_desc32 : nullptr, fused(l));
    // skipped parts: factor 0, so neither sweep changes their cells
    for (auto &q : V.parts) {
      if (!q.skip) continue;
      SSAMG_HIP(hipMemsetAsync(V.d_rs64 + q.off, 0, (size_t)q.ncell * sizeof(double), st));
      if (rs32) SSAMG_HIP(hipMemsetAsync(rs32 + q.off, 0, (size_t)q.ncell * sizeof(float), st));
    }
  };
  // level by level: weights, structured and unstructured Galerkin products,
  // then the level's smoother factors
  for (int l = 0; l + 1 < L; ++l) {
    Level &V = s.lv[l], &C = s.lv[l + 1];
    const int np = (int)V.parts.size();
    bool all_fused = true;
    for (int p = 0; p < np; ++p) all_fused = all_fused && (V.parts[p].dstar < 0 || weights_fused(s, l, p));
    if (!all_fused) launch_interp_weights(V.d_desc64, mixed ? V.d_desc32 : nullptr, np, V.maxf, s.flag, st);
    bool any_ng = false;
    for (const auto &q : V.parts) any_ng = any_ng || q.rap_ng;
    launch_rap(V.d_desc64, V.d_rapdesc, np, V.maxcoarse, C.maxent, s.rap_cell_min, any_ng, st);
    launch_uc_numeric(C.nnz, C.d_uc_start, C.d_uc_k, C.d_uc_a, C.d_uc_b, V.d_uval64,
                      V.d_w64, C.d_uval64, mixed && l + 1 < L - 1 ? C.d_uval32 : nullptr, st);
    smoother_scale(l);
  }
  smoother_scale(L - 1);
  // operator packs of the coarse-end kernel: levels l0 .. L-2 (consecutive
  // records; level sizes do not grow, so the packed levels are a suffix)
  {
    int l0 = L - 1;
    while (l0 - 1 >= 1 && s.lv[l0 - 1].d_pk_nb) --l0;
    if (l0 < L - 1) {
      if (mixed)
        launch_tail_pack<float>((TailLevel<float> *)s.lv[l0].d_tail, L - 1 - l0, s.lv[l0].N, st);
      else
        launch_tail_pack<double>((TailLevel<double> *)s.lv[l0].d_tail, L - 1 - l0, s.lv[l0].N, st);
    }
  }
  if (s.d_hyb) {
    Level &V = s.lv.back();
    launch_dense_inverse(V.d_desc64, (int)V.parts.size(), V.maxcell, V.N, V.nrow, V.d_urow, V.d_uptr,
                         V.d_ucol, V.d_uval64, s.d_hyb, s.d_hyb_pt, s.d_hyb_dinv, s.flag, st);
  } else if (s.prm.coarse == SSAMG_COARSE_DIRECT) {
    Level &V = s.lv.back();
    launch_direct_setup(V.d_desc64, (int)V.parts.size(), (int)V.N, V.nrow, V.d_urow, V.d_uptr, V.d_ucol,
                        V.d_uval64, V.d_ainv, s.flag, st);
  }
  // the collapsed cycle's matrix: the coarse end from level lk run once per
  // unit right-hand side (one workgroup each)
  if (s.lk >= 0) {
    Level &V = s.lv[s.lk];
    TailPlan pl;
    if (!tail_plan(s, s.lk, 0, pl)) throw Error(SSAMG_ERR_STATE, "internal: collapse level without a plan");
    if (mixed)
      launch_tail<float>((const TailLevel<float> *)V.d_tail, pl, 0, st, V.d_mcyc, (int)V.N);
    else
      launch_tail<double>((const TailLevel<double> *)V.d_tail, pl, 0, st, V.d_mcyc, (int)V.N);
  }
  SSAMG_HIP(hipGetLastError());
  int hflag = 0;
  SSAMG_HIP(hipMemcpyAsync(&hflag, s.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SSAMG_HIP(hipStreamSynchronize(st));
  s.h_tab_busy = false;
  const auto t2 = std::chrono::steady_clock::now();
  if (s.verbose)
    fprintf(stderr, "[ssamg] numeric setup: tables %.3f ms (%zu bytes), kernels %.3f ms\n",
            std::chrono::duration<double, std::milli>(t1 - t0).count(), tab_bytes,
            std::chrono::duration<double, std::milli>(t2 - t1).count());
  if (hflag == 2) throw Error(SSAMG_ERR_NUMERIC, "coarsest operator is not positive definite (direct solve)");
  if (hflag) throw Error(SSAMG_ERR_NUMERIC, "non-finite interpolation weight");
  s.t_num = std::chrono::duration<double>(t2 - t0).count();
  s.state = 2;
}

// ---------------------------------------------------------------- cycle

namespace {

template <typename T>
const PartDesc<T> *desc_of(const Level &V);
template <>
const PartDesc<double> *desc_of<double>(const Level &V) { return V.d_desc64; }
template <>
const PartDesc<float> *desc_of<float>(const Level &V) { return V.d_desc32; }

// Algorithmic bytes of one finest-level launch (each array element once).
double level0_bytes(const Solver &s, int kind, int lg, size_t tc, size_t tx, size_t tb, size_t to) {
  const Level &V = s.lv[0];
  const double nr = (double)(1 << lg);
  double by = 0.0;
  for (const auto &q : V.parts) {
    // the FP64 product streams the mirrored subset (see build_descs)
    const bool mir = kind == SSAMG_PROBE_MATVEC && mirrored(s) && q.pat.size() > 7;
    const double n = (double)q.ncell, ne = (double)streamed_entries(q, mir);
    switch (kind) {
      case SSAMG_PROBE_MATVEC: by += n * (ne * tc + nr * (tx + to)); break;
      case SSAMG_PROBE_SMOOTH0: by += n * (tc + nr * (tb + tx)); break;
      // coefficients + smoother factors; b read, x and r written
      case SSAMG_PROBE_RESID0: by += n * (ne * tc + tc + nr * (tb + tx + to)); break;
      // coefficients + smoother factors; x and b read, the output written
      case SSAMG_PROBE_JACOBI0: by += n * (ne * tc + tc + nr * (tx + tb + to)); break;
      case SSAMG_PROBE_RESTRICT0: by += nr * tx * (n + (double)q.cncell) + 2.0 * tc * (double)q.nf; break;
      case SSAMG_PROBE_INTERP0: by += nr * tx * (2.0 * n + (double)q.cncell) + 2.0 * tc * (double)q.nf; break;
      default: break;
    }
  }
  return by;
}

// HIP events of one launch of the probed kernel kind (recorded by the kernel's
// own dispatch); empty when this kind is not probed
struct Probe {
  LaunchEvents e;
  Probe(Solver &s, int kind, double bytes) {
    if (s.probe_kind != kind || s.pev_next + 2 > s.pev.size()) return;
    e.start = s.pev[s.pev_next];
    e.stop = s.pev[s.pev_next + 1];
    s.pev_next += 2;
    s.probe_launches += 1;
    s.probe_bytes += bytes;
  }
};

// First half of a level's down-sweep: x = w b (the first sweep of eq:relax0
// from zero) and t = b - A x.  One fused kernel that forms the iterate at each
// neighbour from its factor and right-hand side, except on large levels with
// more than 15-point stencils, and on levels of at least split_cells elements
// with four or more right-hand sides (then run four columns per thread), where
// the fused kernel's neighbour streams (coefficients, b, w) cost more than
// writing x and running the plain residual sweep.
// whether the finest level's one-column product and sweeps run two cells per
// thread (k_product2, k_sweep2): every part has the full 27-point stencil and
// an even number of cells along x (so a cell pair never straddles a row and
// every part starts at an even cell)
bool product2_ok(const Solver &s, int cpt = 2) {
  if (s.product2 == 0) return false;
  for (const auto &q : s.lv[0].parts)
    if (q.pat.size() != 27 || q.n[0] % cpt != 0 || q.off % cpt != 0) return false;
  return true;
}

bool first_sweep_split(const Solver &s, const Level &V, int lg, const TuneRec &o) {
  return o.split >= 0 ? o.split == 1
                      : (lg >= 2 ? (V.N << lg) >= s.split_cells : (V.maxent > 15 && V.N >= s.split_cells));
}

// x_ready: x = w b is already formed (by the residual update of PCG)
template <typename T, typename TB>
void down_sweep(Solver &s, const Level &V, const PartDesc<T> *d, int fine, int lg, const TB *b, T *x, T *t,
                const TuneRec &o, LaunchEvents ev = {}, bool x_ready = false) {
  const int np = (int)V.parts.size();
  const bool split = first_sweep_split(s, V, lg, o);
  if (split) {
    if (!x_ready) launch_smooth_zero<T, TB>(fine, d, np, V.maxcell, lg, b, x, s.stream);
    if constexpr (std::is_same<TB, double>::value) {
      if (sizeof(T) == 8 && fine && lg == 0 && s.sweepn && product2_ok(s, 16 / sizeof(T))) {
        launch_sweep2<T, T>(MODE_RESID, d, np, V.maxcell, x, b, t, s.stream, ev);
        return;
      }
    }
    launch_stencil<T, TB, T>(MODE_RESID, fine, V.maxent, d, np, V.maxcell, lg, x, b, t, s.stream, ev, o.cols4);
  } else {
    launch_smooth_resid<T, TB>(fine, V.maxent, d, np, V.maxcell, lg, b, x, t, s.stream, ev);
  }
}

}  // namespace

bool tail_plan(const Solver &s, int lt, int lg, TailPlan &pl, int lend) {
  const int L = lend >= 0 ? lend + 1 : (int)s.lv.size();   // levels lt .. L-1
  const size_t ts = s.prm.cycle_precision == SSAMG_FP32 ? sizeof(float) : sizeof(double);
  auto al = [](size_t v) { return (v + 15) & ~(size_t)15; };
  // every level above the coarsest needs its pack
  for (int l = lt; l < L - 1; ++l)
    if (!s.lv[l].d_pk_nb) return false;
  size_t nvec = 0, maxel = 1;
  for (int l = lt; l < L; ++l) {
    nvec += 2 * ((size_t)s.lv[l].N << lg);
    maxel = std::max(maxel, (size_t)s.lv[l].N << lg);
  }
  if (L - lt > 1 && maxel > (size_t)kTailMax) return false;
  pl = TailPlan{};
  pl.nl = L - lt;
  const int tt = ts == sizeof(double) ? kTailThreads / 2 : kTailThreads;
  pl.prodcap = kTailUPer * tt;
  size_t o = al(std::max(sizeof(TailLevel<double>), sizeof(TailLevel<float>)) * pl.nl);
  pl.off_tab = (int)o;
  o = al(o + sizeof(int) * pl.nl);
  pl.off_vec = (int)o;
  o = al(o + ts * nvec);
  pl.off_tv = (int)o;
  o = al(o + ts * maxel);
  pl.off_acc = (int)o;
  o = al(o + ts * maxel);
  pl.off_prod = (int)o;
  o = al(o + ts * (size_t)pl.prodcap);
  if (o > (size_t)kTailLds) return false;
  pl.maxel = (int)maxel;
  pl.bytes = (int)o;
  return true;
}

namespace {

// first level handled by the one-workgroup coarse-end kernel: the first level
// >= 1 with at most tail_elems (<= kTailMax; by default kTailElems, or
// kTailElemsBatched for four or more right-hand sides) elements whose coarse end fits in
// LDS; the coarsest level always is (when it alone does not fit, it runs as a
// grid kernel on global vectors)
int tail_start(const Solver &s, int lg) {
  const int L = (int)s.lv.size();
  if (s.d_hyb) return L - 1;   // hybrid tail: grid levels down to the dense solve
  TailPlan pl;
  const int64_t lim = s.tail_elems >= 0 ? s.tail_elems : (lg >= 2 ? kTailElemsBatched : kTailElems);
  for (int l = 1; l < L; ++l)
    if ((s.lv[l].N << lg) <= lim && tail_plan(s, l, lg, pl)) return l;
  return L - 1;
}

// first level handled by the coarse end (or a grid collapse); levels 1 .. end-1
// are grid levels.  With a collapse level above the coarse end's first level
// (wide batches), the grid levels stop there and its operator is applied as a
// grid kernel.
int grid_end(const Solver &s, int lg) {
  const int lt0 = tail_start(s, lg);
  return s.lk >= 1 && s.lk < lt0 ? s.lk : lt0;
}

// whether grid level l >= 1 takes its first sweep from zero from the
// restriction that forms its right-hand side (split down-sweep, one or two
// columns)
bool zero_in_restrict(const Solver &s, int l, int lg) {
  return s.fuse_zero && lg < 2 && l >= 1 && l < grid_end(s, lg) &&
         first_sweep_split(s, s.lv[l], lg, tune_rec(s, l, lg));
}

template <typename T>
const T *level_rs(const Level &V) {
  if constexpr (sizeof(T) == 4)
    return (const T *)V.d_rs32;
  else
    return (const T *)V.d_rs64;
}

// Levels l >= 1 of one V(1,1) cycle: from lv[1].vb into lv[1].vt (all in T,
// the coarsest level in FP64).  Captured in a HIP graph when use_graph is set.
template <typename T>
void run_tail(Solver &s, int lg) {
  hipStream_t st = s.stream;
  const int L = (int)s.lv.size();
  const int np = (int)s.lv[0].parts.size();
  const int lt0 = tail_start(s, lg);
  const bool grid_collapse = s.lk >= 1 && s.lk < lt0;
  const int lt = grid_end(s, lg);
  for (int l = 1; l < lt; ++l) {
    Level &V = s.lv[l];
    const PartDesc<T> *d = desc_of<T>(V);
    T *b = (T *)V.vb, *x = (T *)V.vx, *t = (T *)V.vt;
    down_sweep<T, T>(s, V, d, 0, lg, b, x, t, tune_rec(s, l, lg), {}, zero_in_restrict(s, l, lg));
    Level &C = s.lv[l + 1];
    const bool zn = zero_in_restrict(s, l + 1, lg);
    launch_restrict<T>(d, np, V.maxcoarse, lg, t, (T *)C.vb, st, {}, zn ? level_rs<T>(C) : nullptr,
                       zn ? (T *)C.vx : nullptr);
  }
  TailPlan pl;
  if (s.d_hyb)   // hybrid tail: the exact solve of the switch level, FP64 inverse
    launch_dense_apply<T>(s.d_hyb, s.lv[lt].N, lg, (const T *)s.lv[lt].vb, (T *)s.lv[lt].vt, s.d_hyb_part, st);
  else if (grid_collapse)
    launch_coarsest<T>((const TailLevel<T> *)s.lv[lt].d_ctail, s.lv[lt].N << lg, lg, st);
  else if (s.lk >= lt && tail_plan(s, lt, lg, pl, s.lk))   // the cycle ends at the collapse level
    launch_tail<T>((const TailLevel<T> *)s.lv[lt].d_ctail, pl, lg, st);
  else if (tail_plan(s, lt, lg, pl))
    launch_tail<T>((const TailLevel<T> *)s.lv[lt].d_tail, pl, lg, st);
  else   // a coarsest level too large for LDS
    launch_coarsest<T>((const TailLevel<T> *)s.lv[lt].d_tail, s.lv[lt].N << lg, lg, st);
  for (int l = lt - 1; l >= 1; --l) {
    Level &V = s.lv[l];
    const PartDesc<T> *d = desc_of<T>(V);
    T *b = (T *)V.vb, *x = (T *)V.vx, *t = (T *)V.vt;
    launch_interp_add<T>(d, np, V.maxcell, lg, (const T *)s.lv[l + 1].vt, x, st);
    launch_stencil<T, T, T>(MODE_JACOBI, 0, V.maxent, d, np, V.maxcell, lg, x, b, t, st, {},
                            tune_rec(s, l, lg).cols4);
  }
}

template <typename T>
void tail(Solver &s, int lg) {
  if (!s.prm.use_graph) {
    run_tail<T>(s, lg);
    return;
  }
  if (!s.graph_exec || s.graph_nrhs != (1 << lg)) {
    if (s.graph_exec) (void)hipGraphExecDestroy(s.graph_exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    s.graph_exec = nullptr;
    s.graph = nullptr;
    SSAMG_HIP(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
    run_tail<T>(s, lg);
    hipGraph_t g = nullptr;
    SSAMG_HIP(hipStreamEndCapture(s.stream, &g));
    s.graph = g;
    SSAMG_HIP(hipGraphInstantiate(&s.graph_exec, g, nullptr, nullptr, 0));
    s.graph_nrhs = 1 << lg;
  }
  SSAMG_HIP(hipGraphLaunch(s.graph_exec, s.stream));
}

// z = B r: one V(1,1) cycle from s.r into s.z.  Level 0 is launched directly
// (large kernels; in a mixed-precision cycle they read r and write z in FP64),
// the coarser levels as one graph.
// With dots (batched widths), the last sweep also forms r.z into S_RZN (after
// moving the old value to S_RZ) and, for flexible CG, z.q into S_ZQ.
template <typename T>
void precond_t(Solver &s, int lg, bool dots) {
  hipStream_t st = s.stream;
  const int L = (int)s.lv.size();
  const int np = (int)s.lv[0].parts.size();
  Level &V = s.lv[0];
  const PartDesc<T> *d = desc_of<T>(V);
  const size_t tc = sizeof(T), tx = sizeof(T);
  T *x = (T *)V.vx, *t = (T *)V.vt;
  if (L == 1 && s.d_hyb) {   // one level, solved exactly (hybrid tail at the finest level)
    launch_dense_apply<double>(s.d_hyb, V.N, lg, s.r, s.z, s.d_hyb_part, st);
    return;
  }
  if (L == 1) {
    const bool direct = V.d_ainv != nullptr;
    if (sizeof(T) == sizeof(float)) {
      launch_cast_d2f(s.r, (float *)V.vb, V.N << lg, st);
      if (direct)
        launch_coarsest<T>((const TailLevel<T> *)V.d_tail, V.N << lg, lg, st);
      else
        launch_coarse_mixed(V.d_desc64, np, V.maxcell, lg, (const float *)V.vb, (float *)V.vt, st);
      launch_cast_f2d((const float *)V.vt, s.z, V.N << lg, st);
    } else if (direct) {
      launch_coarsest<T>((const TailLevel<T> *)V.d_tail, V.N << lg, lg, st);   // vb = r, vt = z
    } else {
      launch_smooth_zero<double, double>(1, V.d_desc64, np, V.maxcell, lg, s.r, s.z, st);
    }
    return;
  }
  const TuneRec o = tune_rec(s, 0, lg);
  {
    Probe pr(s, SSAMG_PROBE_RESID0, level0_bytes(s, SSAMG_PROBE_RESID0, lg, tc, tx, 8, tx));
    const bool ready = s.x0_ready && lg == 0 && first_sweep_split(s, V, lg, o);
    s.x0_ready = false;
    down_sweep<T, double>(s, V, d, 1, lg, s.r, x, t, o, pr.e, ready);
  }
  {
    Probe pr(s, SSAMG_PROBE_RESTRICT0, level0_bytes(s, SSAMG_PROBE_RESTRICT0, lg, tc, tx, tx, tx));
    Level &C = s.lv[1];
    const bool zn = zero_in_restrict(s, 1, lg);
    launch_restrict<T>(d, np, V.maxcoarse, lg, t, (T *)C.vb, st, pr.e, zn ? level_rs<T>(C) : nullptr,
                       zn ? (T *)C.vx : nullptr);
  }
  tail<T>(s, lg);
  {
    Probe pr(s, SSAMG_PROBE_INTERP0, level0_bytes(s, SSAMG_PROBE_INTERP0, lg, tc, tx, tx, tx));
    launch_interp_add<T>(d, np, V.maxcell, lg, (const T *)s.lv[1].vt, x, st, pr.e);
  }
  const bool flexible = s.prm.cycle_precision == SSAMG_FP32;
  {
    // with dots the sweep also reads q (flexible CG)
    Probe pr(s, SSAMG_PROBE_JACOBI0, level0_bytes(s, SSAMG_PROBE_JACOBI0, lg, tc, tx, dots && flexible ? 16 : 8, 8));
    if (sizeof(T) == 8 && !dots && lg == 0 && s.sweepn && product2_ok(s, 16 / sizeof(T)))
      launch_sweep2<T, double>(MODE_JACOBI, d, np, V.maxcell, x, s.r, s.z, st, pr.e);
    else
      launch_stencil<T, double, double>(dots ? MODE_JACOBI_DOT : MODE_JACOBI, 1, V.maxent, d, np, V.maxcell, lg,
                                        x, s.r, s.z, st, pr.e, o.cols4, dots ? s.dotp : nullptr,
                                        dots && flexible ? s.q : nullptr);
  }
  if (dots) {
    const bool c4 = o.cols4 != 0 && stencil_cols4_ok<T>(lg, V.maxent);
    const int nset = flexible ? 2 : 1;
    launch_dot_groups(s.dotp, (int64_t)np * dot_slots(V.maxcell, lg) / 4, lg, c4 ? 1 : 4, nset, s.partial, st);
    launch_dot_final2(s.partial, kDotGroupBlocks, lg, s.scal, S_RZN, 1, S_ZQ, nset, st);
  }
}

void precond(Solver &s, int lg, bool dots = false) {
  if (s.prm.cycle_precision == SSAMG_FP32)
    precond_t<float>(s, lg, dots);
  else
    precond_t<double>(s, lg, dots);
}

// y = A x on level 0 in FP64; with dot_slot >= 0 the product also forms x.y
// per right-hand side into that scalar slot (two small reduction launches)
void apply_A0(Solver &s, int lg, const double *x, double *y, int dot_slot = -1) {
  Level &V = s.lv[0];
  const int np = (int)V.parts.size();
  const TuneRec o = tune_rec(s, 0, lg);
  const int cols4 = s.prm.cycle_precision == SSAMG_FP32 ? o.cols4_mv : o.cols4;
  const bool dot = dot_slot >= 0;
  if (dot && !s.dotp) throw Error(SSAMG_ERR_STATE, "internal: fused product dot needs a batch of 4+");
  {
    Probe pr(s, SSAMG_PROBE_MATVEC, level0_bytes(s, SSAMG_PROBE_MATVEC, lg, 8, 8, 8, 8));
    // the two-cell product always forms its p.q partials; without a dot they
    // go to the partial buffer unread (the true residual's product)
    if (lg == 0 && product2_ok(s) && s.dotp)
      launch_product2(V.d_desc64, np, V.maxcell, mirrored(s), s.product2 == 2, x, y, s.dotp, s.stream, pr.e);
    else
      launch_stencil<double, double, double>(dot ? MODE_APPLY_DOT : MODE_APPLY, 1, V.maxent, V.d_desc64, np,
                                             V.maxcell, lg, x, nullptr, y, s.stream, pr.e, cols4,
                                             dot ? s.dotp : nullptr, nullptr, mirrored(s));
  }
  if (dot) {
    const bool c4 = cols4 != 0 && stencil_cols4_ok<double>(lg, V.maxent);
    launch_dot_groups(s.dotp, (int64_t)np * dot_slots(V.maxcell, lg) / 4, lg, c4 ? 1 : 4, 1, s.partial, s.stream);
    launch_dot_final(s.partial, kDotGroupBlocks, lg, s.scal, dot_slot, s.stream);
  }
}

}  // namespace

void apply_level(Solver &s, int level, const double *x, double *y) {
  Level &V = s.lv[level];
  launch_stencil<double, double, double>(MODE_APPLY, level == 0, V.maxent, V.d_desc64, (int)V.parts.size(),
                                         V.maxcell, 0, x, nullptr, y, s.stream, {}, -1, nullptr, nullptr,
                                         mirrored(s));
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipStreamSynchronize(s.stream));
}

// ---------------------------------------------------------------- autotuner

namespace {

// Fastest of three timed launches (after one untimed), in milliseconds.
template <typename F>
double time_best(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F &&launch) {
  launch();
  double best = 1e30;
  for (int r = 0; r < 3; ++r) {
    SSAMG_HIP(hipEventRecord(e0, st));
    launch();
    SSAMG_HIP(hipEventRecord(e1, st));
    SSAMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    SSAMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, (double)ms);
  }
  return best;
}

// Strip counts worth timing for a level's four-column sweeps: more than one
// only when some part's blocks tile its z-planes and the grid's eight XCD
// ranges hold whole planes (otherwise every count gives the plain order).
std::vector<int> strip_candidates(const Level &V, int lg) {
  std::vector<int> c;
  const long long cpb = (long long)(kBlock * 4) >> lg;
  const long long nblk = (((long long)V.maxcell << lg) + kBlock * 4 - 1) / (kBlock * 4);
  bool tiles = false;
  for (const auto &q : V.parts) {
    const long long plane = (long long)q.n[0] * q.n[1];
    if (plane % cpb) continue;
    const long long bp = plane / cpb;
    if (bp >= 2 && nblk % 8 == 0 && (nblk / 8) % bp == 0) tiles = true;
  }
  if (tiles)
    for (int n : kTuneStrips)
      if (n > 1) c.push_back(n);
  return c;
}

// Times the launch options of every level of width 2^lg that runs grid kernels,
// holds at least kTuneMinElems elements and has no stored record, and stores
// the fastest: the stencil sweep (columns per thread, block order), the first
// sweep (split or fused), and on level 0 of a mixed-precision cycle the FP64
// product.  A candidate replaces the current choice only if it is at least 2 %
// faster.  The level's vectors are zeroed first; every option computes the
// same values, so the timing runs on the hierarchy itself.
template <typename T>
int autotune_t(Solver &s, int lg) {
  hipStream_t st = s.stream;
  const int np = (int)s.lv[0].parts.size();
  const bool mixed = sizeof(T) == sizeof(float);
  const int lt = tail_start(s, lg);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SSAMG_HIP(hipEventCreate(&e0));
  SSAMG_HIP(hipEventCreate(&e1));
  int ntuned = 0;
  try {
    for (int l = 0; l < lt; ++l) {
      Level &V = s.lv[l];
      const int64_t nel = V.N << lg;
      bool found = false;
      (void)tune_rec(s, l, lg, &found);
      if (nel < kTuneMinElems || found) continue;
      SSAMG_HIP(hipMemsetAsync(V.vx, 0, nel * sizeof(T), st));
      SSAMG_HIP(hipMemsetAsync(V.vb, 0, nel * sizeof(T), st));
      SSAMG_HIP(hipMemsetAsync(V.vt, 0, nel * sizeof(T), st));
      if (l == 0)
        for (double *v : {s.r, s.z, s.p, s.q}) SSAMG_HIP(hipMemsetAsync(v, 0, nel * sizeof(double), st));
      T *x = (T *)V.vx, *b = (T *)V.vb, *t = (T *)V.vt;
      TuneRec best;
      auto pick = [&](std::vector<TuneRec> cand, auto &&run) {
        tune_store(s, l, lg, best);
        double tb = time_best(st, e0, e1, run);
        for (const TuneRec &r : cand) {
          tune_store(s, l, lg, r);
          const double tr = time_best(st, e0, e1, run);
          if (tr < 0.98 * tb) {
            best = r;
            tb = tr;
          }
        }
        tune_store(s, l, lg, best);
      };
      // stencil sweep of the cycle
      {
        std::vector<TuneRec> cand;
        TuneRec r = best;
        r.cols4 = 0;
        cand.push_back(r);
        if (stencil_cols4_ok<T>(lg, V.maxent))
          for (int n : strip_candidates(V, lg)) {
            r.cols4 = 1;
            r.strips = n;
            cand.push_back(r);
          }
        pick(cand, [&] {
          const TuneRec o = tune_rec(s, l, lg);
          const PartDesc<T> *d = desc_of<T>(V);
          if (l == 0)
            launch_stencil<T, double, double>(MODE_JACOBI, 1, V.maxent, d, np, V.maxcell, lg, x, s.r, s.z, st,
                                              {}, o.cols4);
          else
            launch_stencil<T, T, T>(MODE_JACOBI, 0, V.maxent, d, np, V.maxcell, lg, x, b, t, st, {}, o.cols4);
        });
      }
      // first sweep: split from the residual or fused with it
      {
        std::vector<TuneRec> cand;
        for (int sp = 0; sp <= 1; ++sp) {
          TuneRec r = best;
          r.split = sp;
          cand.push_back(r);
        }
        pick(cand, [&] {
          const TuneRec o = tune_rec(s, l, lg);
          const PartDesc<T> *d = desc_of<T>(V);
          if (l == 0)
            down_sweep<T, double>(s, V, d, 1, lg, s.r, x, t, o);
          else
            down_sweep<T, T>(s, V, d, 0, lg, b, x, t, o);
        });
      }
      // FP64 product of PCG (its own descriptors in a mixed-precision cycle)
      if (l == 0 && mixed) {
        std::vector<TuneRec> cand;
        TuneRec r = best;
        r.cols4_mv = 0;
        cand.push_back(r);
        if (stencil_cols4_ok<double>(lg, V.maxent))
          for (int n : strip_candidates(V, lg)) {
            r.cols4_mv = 1;
            r.strips_mv = n;
            cand.push_back(r);
          }
        pick(cand, [&] {
          const TuneRec o = tune_rec(s, 0, lg);
          launch_stencil<double, double, double>(MODE_APPLY_DOT, 1, V.maxent, V.d_desc64, np, V.maxcell, lg,
                                                 s.p, nullptr, s.q, st, {}, o.cols4_mv, s.dotp, nullptr,
                                                 mirrored(s));
        });
      }
      ++ntuned;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  SSAMG_HIP(hipEventDestroy(e0));
  SSAMG_HIP(hipEventDestroy(e1));
  return ntuned;
}

}  // namespace

int autotune(Solver &s, int lg) {
  if (s.state < 2) throw Error(SSAMG_ERR_STATE, "autotuning needs the numeric setup");
  if (lg < 2) return 0;   // the options concern batches of four or more right-hand sides
  const auto t0 = std::chrono::steady_clock::now();
  const int n = s.prm.cycle_precision == SSAMG_FP32 ? autotune_t<float>(s, lg) : autotune_t<double>(s, lg);
  SSAMG_HIP(hipGetLastError());
  s.tune_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return n;
}

bool tuned(const Solver &s, int lg) {
  if (lg < 2) return true;
  const int lt = tail_start(s, lg);
  for (int l = 0; l < lt; ++l) {
    bool found = false;
    (void)tune_rec(s, l, lg, &found);
    if ((s.lv[l].N << lg) >= kTuneMinElems && !found) return false;
  }
  return true;
}

void probe_set(Solver &s, int kind) {
  if (kind >= 0 && s.pev.empty()) {
    s.pev.resize(4096);
    for (auto &e : s.pev) SSAMG_HIP(hipEventCreate(&e));
  }
  s.probe_kind = kind;
  s.pev_next = 0;
  s.probe_launches = 0;
  s.probe_bytes = 0.0;
}

void probe_read(Solver &s, int64_t *launches, double *ms, double *bytes) {
  SSAMG_HIP(hipStreamSynchronize(s.stream));
  double total = 0.0;
  for (size_t i = 0; i + 1 < s.pev_next; i += 2) {
    float t = 0.f;
    SSAMG_HIP(hipEventElapsedTime(&t, s.pev[i], s.pev[i + 1]));
    total += t;
  }
  *launches = s.probe_launches;
  *ms = total;
  *bytes = s.probe_bytes;
  s.pev_next = 0;
  s.probe_launches = 0;
  s.probe_bytes = 0.0;
}

void apply_precond(Solver &s, const double *r, double *z) {
  const int64_t N = s.lv[0].N;
  s.x0_ready = false;
  launch_copy(r, s.r, N, s.stream);
  precond(s, 0);
  launch_copy(s.z, z, N, s.stream);
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipStreamSynchronize(s.stream));
}

// ---------------------------------------------------------------- PCG

ssamg_status pcg_solve(Solver &s, int nrhs, const double *b, double *x, ssamg_info *info) {
  int lg = 0;
  while ((1 << lg) < nrhs) ++lg;
  if (s.prm.autotune && !tuned(s, lg)) autotune(s, lg);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  const int64_t nel = s.lv[0].N << lg;
  const bool flexible = s.prm.cycle_precision == SSAMG_FP32;
  double *h = s.h_pin;   // [kScalSlots][kMaxRhs] mirror
  std::vector<int> act(kMaxRhs, 0), iters(nrhs, 0), conv(nrhs, 0);
  std::vector<double> bb(nrhs), relres(nrhs, 0.0);

  s.x0_ready = false;
  // one column with a split finest down-sweep: the residual update also forms
  // that sweep's x = w r for the next cycle
  const Level &V0 = s.lv[0];
  const bool fuse0 = s.fuse_zero && lg == 0 && s.lv.size() > 1 && V0.d_rs64 &&
                     first_sweep_split(s, V0, 0, tune_rec(s, 0, 0)) &&
                     (s.prm.cycle_precision == SSAMG_FP32 ? V0.d_rs32 != nullptr : true);
  launch_fill(x, 0.0, nel, st);
  launch_copy(b, s.r, nel, st);
  launch_dot(b, b, nel, lg, s.partial, s.scal, S_BB, 0, st);
  SSAMG_HIP(hipMemcpyAsync(h, s.scal, kScalSlots * kMaxRhs * sizeof(double), hipMemcpyDeviceToHost, st));
  SSAMG_HIP(hipEventRecord(s.ev_scal, st));
  // the first direction does not depend on which right-hand sides are zero
  // (none of its kernels reads the active mask): queued before |b| is read
  precond(s, lg);
  launch_copy(s.z, s.p, nel, st);
  launch_dot(s.r, s.z, nel, lg, s.partial, s.scal, S_RZN, 0, st);
  SSAMG_HIP(hipEventSynchronize(s.ev_scal));
  int nact = 0;
  for (int k = 0; k < nrhs; ++k) {
    bb[k] = h[S_BB * kMaxRhs + k];
    if (!std::isfinite(bb[k])) throw Error(SSAMG_ERR_NUMERIC, "non-finite right-hand side");
    act[k] = bb[k] > 0.0;
    conv[k] = !act[k];
    nact += act[k];
  }
  SSAMG_HIP(hipMemcpyAsync(s.active, act.data(), kMaxRhs * sizeof(int), hipMemcpyHostToDevice, st));
  const double tol = s.prm.tol;
  bool pending_x = false;            // x += alpha p of the last iteration not yet applied
  // z = B r, the dot products and the x/p update of the next direction
  auto next_direction = [&] {
    if (lg >= 2 && s.lv.size() > 1) {
      precond(s, lg, true);                 // r.z (and z.q) formed by the last sweep
    } else {
      precond(s, lg);
      if (flexible)
        launch_dot2(s.r, s.z, s.q, nel, lg, s.partial, s.scal, S_RZN, 1, S_ZQ, st);
      else
        launch_dot(s.r, s.z, nel, lg, s.partial, s.scal, S_RZN, 1, st);
    }
    launch_pcg_xp(nel, lg, s.scal, s.active, flexible ? 1 : 0, s.z, s.p, x, st);
    pending_x = false;
  };
  // residual history per right-hand side, to predict whether the next
  // iteration is needed
  std::vector<double> rel1(nrhs, 1.0), rel2(nrhs, 1.0);   // x0 = 0: the initial relative residual is 1
  for (int it = 1; it <= s.prm.max_iter && nact > 0; ++it) {
    apply_A0(s, lg, s.p, s.q, S_PQ);        // p.q formed by the product itself
    if (fuse0 && s.prm.cycle_precision == SSAMG_FP32)
      launch_pcg_r(nel, lg, s.scal, s.active, s.r, s.q, s.partial, st, V0.d_rs32, (float *)V0.vx);
    else if (fuse0)
      launch_pcg_r(nel, lg, s.scal, s.active, s.r, s.q, s.partial, st, nullptr, nullptr, V0.d_rs64,
                   (double *)V0.vx);
    else
      launch_pcg_r(nel, lg, s.scal, s.active, s.r, s.q, s.partial, st);
    s.x0_ready = fuse0;
    pending_x = true;
    SSAMG_HIP(hipMemcpyAsync(h, s.scal, kScalSlots * kMaxRhs * sizeof(double), hipMemcpyDeviceToHost, st));
    SSAMG_HIP(hipEventRecord(s.ev_scal, st));
    // Speculation: when some active right-hand side is predicted (from the
    // ratio of its last two residuals) to stay above the tolerance, the next
    // direction is queued before this iteration's residual is read, so the
    // device does not idle during the read.  Always correct: a right-hand side
    // that has converged meanwhile still gets its last x += alpha p (beta and
    // p are discarded, its later alphas are 0); only when every one has
    // converged is the queued preconditioner wasted.
    bool spec = false;
    if (it < s.prm.max_iter)
      for (int k = 0; k < nrhs && !spec; ++k) {
        if (!act[k]) continue;
        const double rho = rel2[k] > 0.0 ? std::min(1.0, rel1[k] / rel2[k]) : 0.0;
        spec = rel1[k] * rho > 4.0 * tol;
      }
    if (spec) next_direction();
    SSAMG_HIP(hipEventSynchronize(s.ev_scal));
    bool changed = false;
    for (int k = 0; k < nrhs; ++k) {
      if (!act[k]) continue;
      const double pq = h[S_PQ * kMaxRhs + k], rr = h[S_RR * kMaxRhs + k];
      if (!(pq > 0.0) || !std::isfinite(pq)) throw Error(SSAMG_ERR_NUMERIC, "PCG breakdown: p^T A p <= 0");
      if (!std::isfinite(rr)) throw Error(SSAMG_ERR_NUMERIC, "non-finite residual");
      iters[k] = it;
      relres[k] = std::sqrt(rr / bb[k]);
      rel2[k] = rel1[k];
      rel1[k] = relres[k];
      if (relres[k] < tol) {
        act[k] = 0;
        conv[k] = 1;
        --nact;
        changed = true;
      }
    }
    if (changed)
      SSAMG_HIP(hipMemcpyAsync(s.active, act.data(), kMaxRhs * sizeof(int), hipMemcpyHostToDevice, st));
    if (nact == 0 || it == s.prm.max_iter) break;
    if (!spec) next_direction();
  }
  s.x0_ready = false;
  if (pending_x) launch_pcg_x(nel, lg, s.scal, s.p, x, st);
  // true residual
  apply_A0(s, lg, x, s.q);
  launch_resid_norm(b, s.q, nel, lg, s.partial, s.scal, S_TR, st);
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipMemcpyAsync(h, s.scal, kScalSlots * kMaxRhs * sizeof(double), hipMemcpyDeviceToHost, st));
  SSAMG_HIP(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  bool all = true;
  for (int k = 0; k < nrhs; ++k) all = all && conv[k];
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->nrhs = nrhs;
    for (int k = 0; k < nrhs; ++k) {
      info->iters[k] = iters[k];
      info->relres[k] = relres[k];
      info->true_relres[k] = bb[k] > 0.0 ? std::sqrt(h[S_TR * kMaxRhs + k] / bb[k]) : 0.0;
      info->converged[k] = conv[k];
    }
    info->t_setup = s.t_sym + s.t_num;
    info->t_solve = std::chrono::duration<double>(t1 - t0).count();
  }
  return all ? SSAMG_OK : SSAMG_NOT_CONVERGED;
}

}  // namespace ssamg
