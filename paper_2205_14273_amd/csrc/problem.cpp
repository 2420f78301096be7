// Problem description (Section 2: grid of boxes, per-part stencils, inter-part
// couplings U, per-cell coefficients) and the C ABI calls that fill it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "capi_common.h"
#include "ssamg_impl.h"

namespace ssamg {

int64_t Problem::ncell_total() const {
  int64_t n = 0;
  for (auto &d : dims) n += (int64_t)d[0] * d[1] * d[2];
  return n;
}

std::vector<int64_t> Problem::offsets() const {
  std::vector<int64_t> off(nparts + 1, 0);
  for (int p = 0; p < nparts; ++p) off[p + 1] = off[p] + (int64_t)dims[p][0] * dims[p][1] * dims[p][2];
  return off;
}

bool Problem::has_topology() const {
  for (int p = 0; p < nparts; ++p) {
    if (!boxes[p].empty()) return true;
    for (int f = 0; f < 6; ++f)
      if (glue[p][f].part >= 0) return true;
  }
  return false;
}

void Problem::free_device() {
  for (auto &c : coef) {
    if (c) (void)hipFree(c);
    c = nullptr;
  }
  for (void *p : {(void *)d_urow, (void *)d_uptr, (void *)d_ucol, (void *)d_uval, (void *)d_kappa,
                  (void *)d_aniso, (void *)d_ucode, (void *)d_geom, (void *)d_cptr, (void *)d_mpart,
                  (void *)d_csum, (void *)d_csoff})
    if (p) (void)hipFree(p);
  d_mpart = nullptr;
  mpart_cap = 0;
  d_csum = nullptr;
  csum_cap = 0;
  d_csoff = nullptr;
  csum_off.clear();
  metric_version = 0;
  d_urow = d_uptr = d_ucol = d_ucode = d_geom = nullptr;
  d_cptr = nullptr;
  fv_structure_ready = false;
  d_uval = d_kappa = d_aniso = nullptr;
}

namespace {

Problem *P(ssamg_problem h) {
  if (!h) throw Error(SSAMG_ERR_ARG, "NULL problem");
  return reinterpret_cast<Problem *>(h);
}

void check_part(const Problem *pr, int part) {
  if (part < 0 || part >= pr->nparts) throw Error(SSAMG_ERR_ARG, "part index out of range");
}

void check_box(const Problem *pr, int part) {
  auto &d = pr->dims[part];
  if (d[0] <= 0 || d[1] <= 0 || d[2] <= 0) throw Error(SSAMG_ERR_STATE, "box of part not set");
}

int center_of(const std::vector<std::array<int, 3>> &st) {
  for (size_t e = 0; e < st.size(); ++e)
    if (st[e][0] == 0 && st[e][1] == 0 && st[e][2] == 0) return (int)e;
  return -1;
}

// Build the canonical compressed-row CSR from COO (sorted by row, then col;
// duplicates summed).
void canonical_csr(int64_t nnz, const int64_t *row, const int64_t *col, const double *val,
                   std::vector<int> &urow, std::vector<int> &uptr, std::vector<int> &ucol,
                   std::vector<double> &uval) {
  std::vector<int64_t> idx(nnz);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return row[a] != row[b] ? row[a] < row[b] : col[a] < col[b];
  });
  urow.clear();
  uptr.assign(1, 0);
  ucol.clear();
  uval.clear();
  int64_t pr = -1, pc = -1;
  for (int64_t t = 0; t < nnz; ++t) {
    const int64_t k = idx[t];
    if (row[k] == pr && col[k] == pc) {
      uval.back() += val[k];
      continue;
    }
    if (row[k] != pr) {
      if (!urow.empty()) uptr.push_back((int)ucol.size());
      urow.push_back((int)row[k]);
    }
    ucol.push_back((int)col[k]);
    uval.push_back(val[k]);
    pr = row[k];
    pc = col[k];
  }
  if (!urow.empty()) uptr.push_back((int)ucol.size());
}

// cells of part p's box that lie in one of its boxes (all without a box list)
std::vector<char> active_mask(const Problem *pr, int p) {
  const auto &n = pr->dims[p];
  const int64_t nc = (int64_t)n[0] * n[1] * n[2];
  if (pr->boxes[p].empty()) return std::vector<char>(nc, 1);
  std::vector<char> m(nc, 0);
  for (const auto &b : pr->boxes[p])
    for (int k = b[2]; k <= b[5]; ++k)
      for (int j = b[1]; j <= b[4]; ++j)
        for (int i = b[0]; i <= b[3]; ++i) m[i + (int64_t)n[0] * (j + (int64_t)n[1] * k)] = 1;
  return m;
}

// canonical CSR of the couplings: the given COO plus every part's entries
// moved across glued faces; rows and columns must be cells of different parts
// and active (not ghost) cells
void rebuild_coupling(Problem *pr) {
  const auto off = pr->offsets();
  const int64_t N = off.back();
  auto part_of = [&](int64_t id) {
    return (int)(std::upper_bound(off.begin(), off.end(), id) - off.begin()) - 1;
  };
  std::vector<int64_t> row(pr->ucoo_row), col(pr->ucoo_col);
  std::vector<double> val(pr->ucoo_val);
  for (int p = 0; p < pr->nparts; ++p) {
    row.insert(row.end(), pr->ux_row[p].begin(), pr->ux_row[p].end());
    col.insert(col.end(), pr->ux_col[p].begin(), pr->ux_col[p].end());
    val.insert(val.end(), pr->ux_val[p].begin(), pr->ux_val[p].end());
  }
  std::vector<std::vector<char>> act(pr->nparts);
  bool any_boxes = false;
  for (int p = 0; p < pr->nparts; ++p) any_boxes = any_boxes || !pr->boxes[p].empty();
  if (any_boxes)
    for (int p = 0; p < pr->nparts; ++p) act[p] = active_mask(pr, p);
  for (size_t k = 0; k < row.size(); ++k) {
    if (row[k] < 0 || row[k] >= N || col[k] < 0 || col[k] >= N)
      throw Error(SSAMG_ERR_ARG, "coupling index out of range");
    const int pr_ = part_of(row[k]), pc = part_of(col[k]);
    if (pr_ == pc) throw Error(SSAMG_ERR_ARG, "coupling inside one part (U must couple different parts)");
    if (!std::isfinite(val[k])) throw Error(SSAMG_ERR_NUMERIC, "non-finite coupling value");
    if (any_boxes && (!act[pr_][row[k] - off[pr_]] || !act[pc][col[k] - off[pc]]))
      throw Error(SSAMG_ERR_ARG, "coupling touches a ghost cell (a cell in none of its part's boxes)");
  }
  canonical_csr((int64_t)row.size(), row.data(), col.data(), val.data(), pr->urow, pr->uptr, pr->ucol,
                pr->uval_host);
  dev_upload(pr->d_urow, pr->urow);
  dev_upload(pr->d_uptr, pr->uptr);
  dev_upload(pr->d_ucol, pr->ucol);
  dev_upload(pr->d_uval, pr->uval_host);
  pr->coupling_set = true;
  pr->fv_structure_ready = false;
}

// Stencil values of part p given topology (host, [nent][ncell], changed in
// place): ghost cells get an identity row; entries pointing at a ghost cell are
// dropped; an entry leaving the box goes, in face order, through the first
// glued face it crosses whose image is an active cell of that face's
// neighbour, and is moved to the part's crossing couplings.
void apply_topology(Problem *pr, int p, std::vector<double> &h) {
  const auto &n = pr->dims[p];
  const int64_t nc = (int64_t)n[0] * n[1] * n[2];
  const auto &st = pr->stencil[p];
  const int nent = (int)st.size(), center = pr->center[p];
  const auto off = pr->offsets();
  const auto act = active_mask(pr, p);
  std::vector<std::vector<char>> nact(pr->nparts);
  for (int f = 0; f < 6; ++f) {
    const int q = pr->glue[p][f].part;
    if (q >= 0 && nact[q].empty()) nact[q] = active_mask(pr, q);
  }
  auto &xr = pr->ux_row[p], &xc = pr->ux_col[p];
  auto &xv = pr->ux_val[p];
  xr.clear();
  xc.clear();
  xv.clear();
  for (int64_t c = 0; c < nc; ++c) {
    if (!act[c]) {
      for (int e = 0; e < nent; ++e) h[(size_t)e * nc + c] = e == center ? 1.0 : 0.0;
      continue;
    }
    const int x[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
    for (int e = 0; e < nent; ++e) {
      if (e == center) continue;
      const int t[3] = {x[0] + st[e][0], x[1] + st[e][1], x[2] + st[e][2]};
      double &a = h[(size_t)e * nc + c];
      const bool inside = t[0] >= 0 && t[0] < n[0] && t[1] >= 0 && t[1] < n[1] && t[2] >= 0 && t[2] < n[2];
      if (inside) {
        if (!act[t[0] + (int64_t)n[0] * (t[1] + (int64_t)n[1] * t[2])]) a = 0.0;
        continue;
      }
      for (int f = 0; f < 6; ++f) {
        const Problem::Glue &g = pr->glue[p][f];
        const int ax = f / 2;
        const bool crossed = (f & 1) ? t[ax] >= n[ax] : t[ax] < 0;
        if (g.part < 0 || !crossed) continue;
        int y[3];
        for (int d = 0; d < 3; ++d) y[g.map[d]] = g.nbr_at[g.map[d]] + g.dir[d] * (t[d] - g.at[d]);
        const auto &m = pr->dims[g.part];
        if (y[0] < 0 || y[0] >= m[0] || y[1] < 0 || y[1] >= m[1] || y[2] < 0 || y[2] >= m[2]) continue;
        const int64_t yc = y[0] + (int64_t)m[0] * (y[1] + (int64_t)m[1] * y[2]);
        if (!nact[g.part][yc]) continue;
        xr.push_back(off[p] + c);
        xc.push_back(off[g.part] + yc);
        xv.push_back(a);
        break;
      }
      a = 0.0;   // moved to U, or dropped (Dirichlet)
    }
  }
}

}  // namespace

// face kind from placement: PART when the layer of cells just across the face
// overlaps another part's box
void derive_faces(Problem *pr) {
  for (int p = 0; p < pr->nparts; ++p) {
    for (int f = 0; f < 6; ++f) {
      const int ax = f / 2, sg = (f & 1) ? 1 : -1;
      if (ax >= pr->ndim) {
        pr->faces[p][f] = SSAMG_FACE_PHYSICAL;
        continue;
      }
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        lo[d] = pr->origin[p][d];
        hi[d] = pr->origin[p][d] + pr->dims[p][d] - 1;
      }
      if (sg < 0)
        lo[ax] = hi[ax] = pr->origin[p][ax] - 1;
      else
        lo[ax] = hi[ax] = pr->origin[p][ax] + pr->dims[p][ax];
      int kind = SSAMG_FACE_PHYSICAL;
      for (int q = 0; q < pr->nparts && kind == SSAMG_FACE_PHYSICAL; ++q) {
        if (q == p) continue;
        bool over = true;
        for (int d = 0; d < 3; ++d) {
          const int qlo = pr->origin[q][d], qhi = pr->origin[q][d] + pr->dims[q][d] - 1;
          over = over && lo[d] <= qhi && qlo <= hi[d];
        }
        if (over) kind = SSAMG_FACE_PART;
      }
      pr->faces[p][f] = kind;
    }
  }
}

// canonical finite-volume stencil: center first, then (dz, dy, dx) ascending
std::vector<std::array<int, 3>> fv_offsets(int kind, int ndim) {
  std::vector<std::array<int, 3>> out = {{0, 0, 0}};
  const int zl = ndim == 3 ? -1 : 0, zh = ndim == 3 ? 1 : 0;
  for (int dz = zl; dz <= zh; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
        if (nnz == 0) continue;
        if ((kind == 7 || kind == 5) && nnz > 1) continue;
        out.push_back({dx, dy, dz});
      }
  return out;
}

}  // namespace ssamg

using namespace ssamg;

extern "C" {

ssamg_status ssamg_problem_create(int ndim, int nparts, ssamg_problem *out) {
  API_BEGIN
  if (!out) throw Error(SSAMG_ERR_ARG, "NULL output");
  if (ndim != 2 && ndim != 3) throw Error(SSAMG_ERR_ARG, "ndim must be 2 or 3");
  if (nparts <= 0 || nparts > 8191) throw Error(SSAMG_ERR_ARG, "nparts must be in 1..8191");
  auto *pr = new Problem();
  pr->ndim = ndim;
  pr->nparts = nparts;
  pr->dims.assign(nparts, {0, 0, 0});
  pr->origin.assign(nparts, {0, 0, 0});
  pr->has_origin.assign(nparts, 0);
  pr->faces.assign(nparts, {0, 0, 0, 0, 0, 0});
  pr->stencil.assign(nparts, {});
  pr->center.assign(nparts, -1);
  pr->coef.assign(nparts, nullptr);
  pr->coef_set.assign(nparts, 0);
  pr->sym_ok.assign(nparts, 1);
  pr->boxes.assign(nparts, {});
  pr->glue.assign(nparts, {});
  pr->ux_row.assign(nparts, {});
  pr->ux_col.assign(nparts, {});
  pr->ux_val.assign(nparts, {});
  *out = reinterpret_cast<ssamg_problem>(pr);
  API_END
}

ssamg_status ssamg_problem_destroy(ssamg_problem prob) {
  API_BEGIN
  delete reinterpret_cast<Problem *>(prob);
  API_END
}

ssamg_status ssamg_problem_set_box(ssamg_problem prob, int part, const int lo[3], const int hi[3]) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  if (!lo || !hi) throw Error(SSAMG_ERR_ARG, "NULL corner");
  if (lo[0] != 0 || lo[1] != 0 || lo[2] != 0)
    throw Error(SSAMG_ERR_UNSUPPORTED, "box lower corner must be (0,0,0)");
  for (int d = 0; d < 3; ++d)
    if (hi[d] < lo[d]) throw Error(SSAMG_ERR_ARG, "empty box");
  if (pr->ndim == 2 && hi[2] != 0) throw Error(SSAMG_ERR_ARG, "2D box must have nz = 1");
  std::array<int, 3> n = {hi[0] + 1, hi[1] + 1, hi[2] + 1};
  if ((int64_t)n[0] * n[1] * n[2] >= (int64_t(1) << 31)) throw Error(SSAMG_ERR_UNSUPPORTED, "box too large");
  if (pr->dims[part] != n) {
    pr->dims[part] = n;
    if (pr->coef[part]) (void)hipFree(pr->coef[part]);
    pr->coef[part] = nullptr;
    pr->coef_set[part] = 0;
    pr->coef_version++;
    pr->fv_structure_ready = false;
  }
  API_END
}

ssamg_status ssamg_problem_set_origin(ssamg_problem prob, int part, const int origin[3]) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  if (!origin) throw Error(SSAMG_ERR_ARG, "NULL origin");
  pr->origin[part] = {origin[0], origin[1], pr->ndim == 2 ? 0 : origin[2]};
  pr->has_origin[part] = 1;
  pr->fv_structure_ready = false;
  API_END
}

ssamg_status ssamg_problem_set_face(ssamg_problem prob, int part, int face, int kind) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  if (face < 0 || face > 5) throw Error(SSAMG_ERR_ARG, "face must be 0..5");
  if (kind != SSAMG_FACE_PHYSICAL && kind != SSAMG_FACE_PART) throw Error(SSAMG_ERR_ARG, "bad face kind");
  pr->faces[part][face] = kind;
  pr->fv_structure_ready = false;
  API_END
}

// every part's coefficients depend on the boxes and glued faces of the parts
// they reach: topology changes ask for the coefficients again
static void topology_changed(Problem *pr) {
  for (int p = 0; p < pr->nparts; ++p) pr->coef_set[p] = 0;
  pr->coef_version++;
  pr->fv_structure_ready = false;
}

ssamg_status ssamg_problem_add_box(ssamg_problem prob, int part, const int lo[3], const int hi[3]) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  check_box(pr, part);
  if (!lo || !hi) throw Error(SSAMG_ERR_ARG, "NULL corner");
  const auto &n = pr->dims[part];
  for (int d = 0; d < 3; ++d)
    if (lo[d] < 0 || hi[d] >= n[d] || lo[d] > hi[d])
      throw Error(SSAMG_ERR_ARG, "box must be non-empty and lie in the part's box");
  pr->boxes[part].push_back({lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]});
  topology_changed(pr);
  API_END
}

ssamg_status ssamg_problem_set_neighbor(ssamg_problem prob, int part, int face, int nbr_part, const int at[3],
                                        const int nbr_at[3], const int map[3], const int dir[3]) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  check_part(pr, nbr_part);
  check_box(pr, part);
  check_box(pr, nbr_part);
  if (nbr_part == part) throw Error(SSAMG_ERR_ARG, "a face glued to its own part would put couplings inside it");
  if (face < 0 || face > 5 || face / 2 >= pr->ndim) throw Error(SSAMG_ERR_ARG, "bad face");
  if (!at || !nbr_at || !map || !dir) throw Error(SSAMG_ERR_ARG, "NULL argument");
  const auto &n = pr->dims[part], &m = pr->dims[nbr_part];
  int seen = 0;
  for (int d = 0; d < 3; ++d) {
    if (map[d] < 0 || map[d] > 2 || (seen >> map[d]) & 1) throw Error(SSAMG_ERR_ARG, "map must be a permutation");
    seen |= 1 << map[d];
    if (dir[d] != 1 && dir[d] != -1) throw Error(SSAMG_ERR_ARG, "dir must be +1 or -1");
    if (nbr_at[d] < 0 || nbr_at[d] >= m[d]) throw Error(SSAMG_ERR_ARG, "nbr_at must lie in the neighbour's box");
  }
  const int ax = face / 2;
  for (int d = 0; d < 3; ++d) {
    const bool ok = d == ax ? at[d] == ((face & 1) ? n[d] : -1) : (at[d] >= 0 && at[d] < n[d]);
    if (!ok) throw Error(SSAMG_ERR_ARG, "at must be a point just across the face");
  }
  Problem::Glue &g = pr->glue[part][face];
  g.part = nbr_part;
  for (int d = 0; d < 3; ++d) {
    g.at[d] = at[d];
    g.nbr_at[d] = nbr_at[d];
    g.map[d] = map[d];
    g.dir[d] = dir[d];
  }
  pr->faces[part][face] = SSAMG_FACE_PART;
  topology_changed(pr);
  API_END
}

ssamg_status ssamg_problem_set_stencil(ssamg_problem prob, int part, int nent, const int *off) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  if (!off || nent <= 0) throw Error(SSAMG_ERR_ARG, "empty stencil");
  if (nent > kMaxEnt) throw Error(SSAMG_ERR_UNSUPPORTED, "more than 27 stencil entries");
  std::vector<std::array<int, 3>> st;
  for (int e = 0; e < nent; ++e) {
    std::array<int, 3> o = {off[3 * e], off[3 * e + 1], off[3 * e + 2]};
    for (int d = 0; d < 3; ++d)
      if (o[d] < -1 || o[d] > 1)
        throw Error(SSAMG_ERR_UNSUPPORTED, "stencil offsets must lie in {-1,0,1}^3");
    if (pr->ndim == 2 && o[2] != 0) throw Error(SSAMG_ERR_ARG, "2D stencil with dz != 0");
    if (std::find(st.begin(), st.end(), o) != st.end()) throw Error(SSAMG_ERR_ARG, "repeated stencil offset");
    st.push_back(o);
  }
  const int c = center_of(st);
  if (c < 0) throw Error(SSAMG_ERR_ARG, "stencil lacks the (0,0,0) entry");
  if (pr->stencil[part] != st) {
    pr->stencil[part] = st;
    pr->center[part] = c;
    if (pr->coef[part]) (void)hipFree(pr->coef[part]);
    pr->coef[part] = nullptr;
    pr->coef_set[part] = 0;
    pr->coef_version++;
    pr->fv_structure_ready = false;
  }
  API_END
}

ssamg_status ssamg_problem_set_coeffs(ssamg_problem prob, int part, const double *vals, int where,
                                      int constant) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  check_box(pr, part);
  if (pr->stencil[part].empty()) throw Error(SSAMG_ERR_STATE, "stencil of part not set");
  if (!vals) throw Error(SSAMG_ERR_ARG, "NULL coefficients");
  if (where != SSAMG_MEM_HOST && where != SSAMG_MEM_DEVICE) throw Error(SSAMG_ERR_ARG, "bad memory kind");
  const int nent = (int)pr->stencil[part].size();
  const int64_t ncell = (int64_t)pr->dims[part][0] * pr->dims[part][1] * pr->dims[part][2];
  if (!pr->coef[part]) pr->coef[part] = dev_alloc<double>((size_t)nent * ncell);
  double *dst = pr->coef[part];
  bool topo = !pr->boxes[part].empty();
  for (int f = 0; f < 6; ++f) topo = topo || pr->glue[part][f].part >= 0;
  if (topo) {
    // ghost cells and glued faces: the values are rearranged on the host
    for (int f = 0; f < 6; ++f)
      if (pr->glue[part][f].part >= 0) check_box(pr, pr->glue[part][f].part);
    std::vector<double> h((size_t)nent * ncell);
    if (constant) {
      std::vector<double> cv(nent);
      if (where == SSAMG_MEM_HOST)
        std::memcpy(cv.data(), vals, nent * sizeof(double));
      else
        SSAMG_HIP(hipMemcpy(cv.data(), vals, nent * sizeof(double), hipMemcpyDeviceToHost));
      for (int e = 0; e < nent; ++e) std::fill(h.begin() + e * ncell, h.begin() + (e + 1) * ncell, cv[e]);
    } else if (where == SSAMG_MEM_HOST) {
      std::memcpy(h.data(), vals, h.size() * sizeof(double));
    } else {
      SSAMG_HIP(hipMemcpy(h.data(), vals, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    apply_topology(pr, part, h);
    SSAMG_HIP(hipMemcpy(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  } else if (constant) {
    std::vector<double> host(nent);
    if (where == SSAMG_MEM_HOST)
      std::memcpy(host.data(), vals, nent * sizeof(double));
    else
      SSAMG_HIP(hipMemcpy(host.data(), vals, nent * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> full((size_t)nent * ncell);
    for (int e = 0; e < nent; ++e) std::fill(full.begin() + e * ncell, full.begin() + (e + 1) * ncell, host[e]);
    SSAMG_HIP(hipMemcpy(dst, full.data(), full.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    SSAMG_HIP(hipMemcpy(dst, vals, (size_t)nent * ncell * sizeof(double),
                        where == SSAMG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice));
  }
  if (!topo) {
    pr->ux_row[part].clear();
    pr->ux_col[part].clear();
    pr->ux_val[part].clear();
  }
  BoxStencil bs{};
  for (int d = 0; d < 3; ++d) bs.n[d] = pr->dims[part][d];
  bs.nent = nent;
  bs.center = pr->center[part];
  bs.ncell = ncell;
  for (int e = 0; e < nent; ++e) {
    const auto &o = pr->stencil[part][e];
    bs.code[e] = pack_off(o[0], o[1], o[2]);
    bs.lin[e] = o[0] + bs.n[0] * (o[1] + bs.n[1] * o[2]);
    bs.mir[e] = -1;
    for (int f = 0; f < nent; ++f) {
      const auto &t = pr->stencil[part][f];
      if (t[0] == -o[0] && t[1] == -o[1] && t[2] == -o[2]) bs.mir[e] = f;
    }
  }
  bs.coef = dst;
  int *flag = dev_alloc<int>(2);
  SSAMG_HIP(hipMemset(flag, 0, 2 * sizeof(int)));
  launch_normalise(bs, flag, nullptr);
  int hflag[2] = {0, 0};
  SSAMG_HIP(hipMemcpy(hflag, flag, 2 * sizeof(int), hipMemcpyDeviceToHost));
  (void)hipFree(flag);
  SSAMG_HIP(hipGetLastError());
  pr->coef_set[part] = 1;
  pr->coef_version++;
  pr->sym_ok[part] = hflag[1] == 0;
  pr->fv_structure_ready = false;
  if (hflag[0]) throw Error(SSAMG_ERR_NUMERIC, "nonpositive diagonal or non-finite coefficient");
  if (topo || pr->has_topology()) rebuild_coupling(pr);
  API_END
}

ssamg_status ssamg_problem_set_coupling(ssamg_problem prob, int64_t nnz, const int64_t *row,
                                        const int64_t *col, const double *val, int where) {
  API_BEGIN
  Problem *pr = P(prob);
  if (nnz < 0) throw Error(SSAMG_ERR_ARG, "negative nnz");
  if (nnz > 0 && (!row || !col || !val)) throw Error(SSAMG_ERR_ARG, "NULL coupling arrays");
  if (where != SSAMG_MEM_HOST && where != SSAMG_MEM_DEVICE) throw Error(SSAMG_ERR_ARG, "bad memory kind");
  for (int p = 0; p < pr->nparts; ++p) check_box(pr, p);
  // device COO: the canonical form is built on the host from a copy
  std::vector<int64_t> hrow, hcol;
  std::vector<double> hval;
  if (where == SSAMG_MEM_DEVICE && nnz > 0) {
    hrow.resize(nnz);
    hcol.resize(nnz);
    hval.resize(nnz);
    SSAMG_HIP(hipMemcpy(hrow.data(), row, nnz * sizeof(int64_t), hipMemcpyDeviceToHost));
    SSAMG_HIP(hipMemcpy(hcol.data(), col, nnz * sizeof(int64_t), hipMemcpyDeviceToHost));
    SSAMG_HIP(hipMemcpy(hval.data(), val, nnz * sizeof(double), hipMemcpyDeviceToHost));
    row = hrow.data();
    col = hcol.data();
    val = hval.data();
  }
  const auto off = pr->offsets();
  const int64_t N = off.back();
  auto part_of = [&](int64_t id) {
    return (int)(std::upper_bound(off.begin(), off.end(), id) - off.begin()) - 1;
  };
  for (int64_t k = 0; k < nnz; ++k) {
    if (row[k] < 0 || row[k] >= N || col[k] < 0 || col[k] >= N)
      throw Error(SSAMG_ERR_ARG, "coupling index out of range");
    if (part_of(row[k]) == part_of(col[k]))
      throw Error(SSAMG_ERR_ARG, "coupling inside one part (U must couple different parts)");
    if (!std::isfinite(val[k])) throw Error(SSAMG_ERR_NUMERIC, "non-finite coupling value");
  }
  pr->ucoo_row.assign(row, row + nnz);
  pr->ucoo_col.assign(col, col + nnz);
  pr->ucoo_val.assign(val, val + nnz);
  rebuild_coupling(pr);
  API_END
}

ssamg_status ssamg_problem_num_cells(ssamg_problem prob, int64_t *n) {
  API_BEGIN
  Problem *pr = P(prob);
  if (!n) throw Error(SSAMG_ERR_ARG, "NULL output");
  *n = pr->ncell_total();
  API_END
}

ssamg_status ssamg_problem_num_parts(ssamg_problem prob, int *nparts) {
  API_BEGIN
  Problem *pr = P(prob);
  if (!nparts) throw Error(SSAMG_ERR_ARG, "NULL output");
  *nparts = pr->nparts;
  API_END
}

ssamg_status ssamg_problem_part_size(ssamg_problem prob, int part, int *nent, int64_t *ncell) {
  API_BEGIN
  Problem *pr = P(prob);
  check_part(pr, part);
  if (!nent || !ncell) throw Error(SSAMG_ERR_ARG, "NULL output");
  *nent = (int)pr->stencil[part].size();
  *ncell = (int64_t)pr->dims[part][0] * pr->dims[part][1] * pr->dims[part][2];
  API_END
}

ssamg_status ssamg_problem_fv_assemble(ssamg_problem prob, const double *kappa, const double *aniso,
                                       int stencil, void *hip_stream) {
  API_BEGIN
  Problem *pr = P(prob);
  hipStream_t st = (hipStream_t)hip_stream;
  if (!kappa || !aniso) throw Error(SSAMG_ERR_ARG, "NULL kappa or aniso");
  const bool ok3 = pr->ndim == 3 && (stencil == 7 || stencil == 27);
  const bool ok2 = pr->ndim == 2 && (stencil == 5 || stencil == 9);
  if (!ok3 && !ok2) throw Error(SSAMG_ERR_ARG, "stencil must be 7|27 (3D) or 5|9 (2D)");
  if (pr->has_topology())
    throw Error(SSAMG_ERR_UNSUPPORTED, "fv_assemble places parts by origins: parts of several boxes and "
                                       "glued faces take set_coeffs and set_coupling");
  for (int p = 0; p < pr->nparts; ++p) {
    check_box(pr, p);
    if (!pr->has_origin[p]) throw Error(SSAMG_ERR_STATE, "origin of every part is needed");
    for (int d = 0; d < 3; ++d)
      if (!(aniso[3 * p + d] > 0.0) || !std::isfinite(aniso[3 * p + d]))
        throw Error(SSAMG_ERR_ARG, "aniso factors must be positive");
  }
  // parts must not overlap in the global index space
  for (int p = 0; p < pr->nparts; ++p)
    for (int q = p + 1; q < pr->nparts; ++q) {
      bool over = true;
      for (int d = 0; d < 3; ++d)
        over = over && pr->origin[p][d] < pr->origin[q][d] + pr->dims[q][d] &&
               pr->origin[q][d] < pr->origin[p][d] + pr->dims[p][d];
      if (over) throw Error(SSAMG_ERR_ARG, "parts overlap in the global index space");
    }
  const auto st_off = fv_offsets(stencil, pr->ndim);
  const int nent = (int)st_off.size();
  const auto off = pr->offsets();
  const int64_t N = off.back();
  int maxcell = 0;
  for (int p = 0; p < pr->nparts; ++p) {
    const int64_t nc = off[p + 1] - off[p];
    maxcell = std::max<int64_t>(maxcell, nc);
    if (pr->stencil[p] != st_off || !pr->coef[p]) {
      if (pr->coef[p]) (void)hipFree(pr->coef[p]);
      pr->coef[p] = dev_alloc<double>((size_t)nent * nc);
      pr->fv_structure_ready = false;
    }
    pr->stencil[p] = st_off;
    pr->center[p] = 0;
    pr->coef_set[p] = 1;
    pr->sym_ok[p] = 1;   // two-point conductances are symmetric by construction
  }
  // the face kinds, the geometry table and the coupling structure depend on
  // the placement and the stencil only: rebuilt when those change
  std::vector<int> sig = {pr->ndim, pr->nparts, stencil};
  for (int p = 0; p < pr->nparts; ++p)
    for (int d = 0; d < 3; ++d) {
      sig.push_back(pr->dims[p][d]);
      sig.push_back(pr->origin[p][d]);
    }
  const bool same_geometry = pr->fv_structure_ready && sig == pr->fv_signature;
  if (!same_geometry) {
  pr->fv_structure_ready = false;
  derive_faces(pr);
  // geometry table
  std::vector<int> geom(7 * pr->nparts);
  for (int p = 0; p < pr->nparts; ++p) {
    for (int d = 0; d < 3; ++d) {
      geom[7 * p + d] = pr->origin[p][d];
      geom[7 * p + 3 + d] = pr->dims[p][d];
    }
    geom[7 * p + 6] = (int)off[p];
  }
  dev_upload(pr->d_geom, geom);
  // coupling structure from placement: boundary cells whose neighbour lies in
  // another part
  std::vector<int64_t> crow, ccol;
  std::vector<int> ccode_raw;
  for (int p = 0; p < pr->nparts; ++p) {
    const auto &n = pr->dims[p];
    const auto &o = pr->origin[p];
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j) {
        const bool edge_jk = (j == 0 || j == n[1] - 1 || k == 0 || k == n[2] - 1);
        for (int i = 0; i < n[0]; ++i) {
          if (!edge_jk && i != 0 && i != n[0] - 1) {
            i = n[0] - 2;   // skip to the last cell of the row
            continue;
          }
          for (int e = 1; e < nent; ++e) {
            const int lc[3] = {i + st_off[e][0], j + st_off[e][1], k + st_off[e][2]};
            if (lc[0] >= 0 && lc[0] < n[0] && lc[1] >= 0 && lc[1] < n[1] && lc[2] >= 0 && lc[2] < n[2])
              continue;
            const int G[3] = {o[0] + lc[0], o[1] + lc[1], o[2] + lc[2]};
            for (int q = 0; q < pr->nparts; ++q) {
              if (q == p) continue;
              const auto &h = pr->origin[q];
              const auto &m = pr->dims[q];
              if (G[0] >= h[0] && G[0] < h[0] + m[0] && G[1] >= h[1] && G[1] < h[1] + m[1] &&
                  G[2] >= h[2] && G[2] < h[2] + m[2]) {
                const int64_t jid = off[q] + (G[0] - h[0]) + (int64_t)m[0] * ((G[1] - h[1]) + (int64_t)m[1] * (G[2] - h[2]));
                crow.push_back(off[p] + i + (int64_t)n[0] * (j + (int64_t)n[1] * k));
                ccol.push_back(jid);
                // link code: offset (6 bits), row part, column part (13 bits each)
                ccode_raw.push_back((int)((unsigned)pack_off(st_off[e][0], st_off[e][1], st_off[e][2]) |
                                          ((unsigned)p << 6) | ((unsigned)q << 19)));
                break;
              }
            }
          }
        }
      }
  }
  // canonical order (rows ascending already; sort entries inside each row)
  std::vector<int64_t> idx(crow.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return crow[a] != crow[b] ? crow[a] < crow[b] : ccol[a] < ccol[b];
  });
  pr->urow.clear();
  pr->uptr.assign(1, 0);
  pr->ucol.clear();
  std::vector<int> ucode;
  for (int64_t t = 0; t < (int64_t)idx.size(); ++t) {
    const int64_t k = idx[t];
    if (pr->urow.empty() || pr->urow.back() != (int)crow[k]) {
      if (!pr->urow.empty()) pr->uptr.push_back((int)pr->ucol.size());
      pr->urow.push_back((int)crow[k]);
    }
    pr->ucol.push_back((int)ccol[k]);
    ucode.push_back(ccode_raw[k]);
  }
  if (!pr->urow.empty()) pr->uptr.push_back((int)pr->ucol.size());
  pr->uval_host.assign(pr->ucol.size(), 0.0);
  dev_upload(pr->d_urow, pr->urow);
  dev_upload(pr->d_uptr, pr->uptr);
  dev_upload(pr->d_ucol, pr->ucol);
  dev_upload(pr->d_ucode, ucode);
  if (pr->d_uval) (void)hipFree(pr->d_uval);
  pr->d_uval = dev_alloc<double>(pr->ucol.size());
  pr->coupling_set = true;
  std::vector<double *> cptr(pr->coef.begin(), pr->coef.end());
  dev_upload(pr->d_cptr, cptr);
  if (pr->d_kappa) (void)hipFree(pr->d_kappa);
  pr->d_kappa = dev_alloc<double>(N);
  if (pr->d_aniso) (void)hipFree(pr->d_aniso);
  pr->d_aniso = dev_alloc<double>(3 * pr->nparts);
  pr->fv_signature = sig;
  pr->fv_structure_ready = true;
  }
  // conductivity and anisotropy copies
  SSAMG_HIP(hipMemcpyAsync(pr->d_kappa, kappa, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  SSAMG_HIP(hipMemcpyAsync(pr->d_aniso, aniso, 3 * pr->nparts * sizeof(double), hipMemcpyHostToDevice, st));
  pr->fv_stencil = stencil;
  // kernels
  FvArgs fa{};
  fa.geom = pr->d_geom;
  fa.nparts = pr->nparts;
  fa.nent = nent;
  for (int e = 0; e < nent; ++e) fa.code[e] = pack_off(st_off[e][0], st_off[e][1], st_off[e][2]);
  const size_t mbytes = (size_t)pr->nparts * fv_blocks((int)maxcell) * 3 * sizeof(double);
  if (pr->mpart_cap < mbytes) {
    if (pr->d_mpart) (void)hipFree(pr->d_mpart);
    pr->d_mpart = nullptr;
    pr->mpart_cap = 0;
    pr->d_mpart = dev_alloc<double>(mbytes / sizeof(double));
    pr->mpart_cap = mbytes;
  }
  // collapse sums: per part and direction d, three blocks of the cells odd along d
  {
    std::vector<long long> off((size_t)3 * pr->nparts);
    long long tot = 0;
    for (int p = 0; p < pr->nparts; ++p) {
      const auto &n = pr->dims[p];
      for (int d = 0; d < 3; ++d) {
        off[3 * p + d] = tot;
        tot += 3LL * (n[d] / 2) * n[(d + 1) % 3] * n[(d + 2) % 3];
      }
    }
    const size_t cbytes = (size_t)std::max<long long>(tot, 1) * sizeof(double);
    if (pr->csum_cap < cbytes) {
      if (pr->d_csum) (void)hipFree(pr->d_csum);
      pr->d_csum = nullptr;
      pr->csum_cap = 0;
      pr->d_csum = dev_alloc<double>(cbytes / sizeof(double));
      pr->csum_cap = cbytes;
    }
    if (off != pr->csum_off || !pr->d_csoff) {
      dev_upload(pr->d_csoff, off);
      pr->csum_off = off;
    }
  }
  launch_fv_stencil(fa, maxcell, pr->d_kappa, pr->d_aniso, pr->d_cptr, pr->d_mpart, pr->d_csum, pr->d_csoff,
                    st);
  launch_fv_coupling((int)pr->urow.size(), pr->d_urow, pr->d_uptr, pr->d_ucol, pr->d_ucode,
                     pr->d_kappa, pr->d_aniso, pr->d_uval, st);
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipStreamSynchronize(st));
  pr->coef_version++;
  pr->metric_version = pr->coef_version;
  pr->mpart_nb = fv_blocks((int)maxcell);
  API_END
}

ssamg_status ssamg_problem_fv_grad(ssamg_problem prob, int nrhs, const double *lambda, const double *x,
                                   double *grad, void *hip_stream) {
  API_BEGIN
  Problem *pr = P(prob);
  if (!pr->fv_stencil) throw Error(SSAMG_ERR_STATE, "fv_assemble has not been called");
  if (!lambda || !x || !grad) throw Error(SSAMG_ERR_ARG, "NULL vector");
  if (nrhs < 1 || nrhs > kMaxRhs) throw Error(SSAMG_ERR_ARG, "nrhs must be in 1..32");
  hipStream_t st = (hipStream_t)hip_stream;
  const auto st_off = fv_offsets(pr->fv_stencil, pr->ndim);
  FvArgs fa{};
  fa.geom = pr->d_geom;
  fa.nparts = pr->nparts;
  fa.nent = (int)st_off.size();
  for (int e = 0; e < fa.nent; ++e) fa.code[e] = pack_off(st_off[e][0], st_off[e][1], st_off[e][2]);
  const auto off = pr->offsets();
  int64_t maxcell = 0;
  for (int p = 0; p < pr->nparts; ++p) maxcell = std::max(maxcell, off[p + 1] - off[p]);
  launch_fv_grad(fa, (int)maxcell, pr->d_kappa, pr->d_aniso, lambda, x, nrhs, grad, (int)pr->urow.size(),
                 pr->d_urow, pr->d_uptr, pr->d_ucol, pr->d_ucode, st);
  SSAMG_HIP(hipGetLastError());
  SSAMG_HIP(hipStreamSynchronize(st));
  API_END
}

}  // extern "C"
