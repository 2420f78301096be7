// C ABI of the solver object (include/ssamg.h).
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "capi_common.h"
#include "ssamg_impl.h"

using namespace ssamg;

namespace ssamg {
extern thread_local std::string g_last_error;
}

namespace {

Solver *S(ssamg_solver h) {
  if (!h) throw Error(SSAMG_ERR_ARG, "NULL solver");
  return reinterpret_cast<Solver *>(h);
}

void need(const Solver *s, int state, const char *what) {
  if (s->state < state) throw Error(SSAMG_ERR_STATE, what);
}

void check_level(const Solver *s, int level) {
  if (level < 0 || level >= (int)s->lv.size()) throw Error(SSAMG_ERR_ARG, "level out of range");
}

void check_part(const Solver *s, int level, int part) {
  check_level(s, level);
  if (part < 0 || part >= (int)s->lv[level].parts.size()) throw Error(SSAMG_ERR_ARG, "part out of range");
}

int width_lg(const Solver *s, int nrhs) {
  if (nrhs < 1 || nrhs > s->prm.max_nrhs || (nrhs & (nrhs - 1)))
    throw Error(SSAMG_ERR_ARG, "nrhs must be a power of two <= max_nrhs");
  int lg = 0;
  while ((1 << lg) < nrhs) ++lg;
  return lg;
}

// Autotuner cache: a JSON object whose "records" array holds one object per
// line, {"key": ..., "strips": ..., "cols4": ..., "split": ..., "strips_mv":
// ..., "cols4_mv": ...}, keys in this order (the file is written here).
const char *kCacheFormat = "ssamg-autotune-1";

std::map<std::string, TuneRec> read_cache(const char *path) {
  std::map<std::string, TuneRec> out;
  std::ifstream f(path);
  if (!f) return out;                 // no file yet
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  if (text.find(kCacheFormat) == std::string::npos)
    throw Error(SSAMG_ERR_ARG, std::string("not an autotuner cache: ") + path);
  size_t at = 0;
  while ((at = text.find("{\"key\":", at)) != std::string::npos) {
    char key[1024];
    TuneRec r;
    const int n = std::sscanf(text.c_str() + at,
                              "{\"key\": \"%1023[^\"]\", \"strips\": %d, \"cols4\": %d, \"split\": %d, "
                              "\"strips_mv\": %d, \"cols4_mv\": %d}",
                              key, &r.strips, &r.cols4, &r.split, &r.strips_mv, &r.cols4_mv);
    if (n != 6) throw Error(SSAMG_ERR_ARG, std::string("malformed record in ") + path);
    out[key] = r;
    ++at;
  }
  return out;
}

void write_cache(const char *path, const std::map<std::string, TuneRec> &recs) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) throw Error(SSAMG_ERR_ARG, std::string("cannot write ") + tmp);
    f << "{\"format\": \"" << kCacheFormat << "\", \"records\": [\n";
    size_t i = 0;
    for (const auto &kv : recs) {
      const TuneRec &r = kv.second;
      f << "  {\"key\": \"" << kv.first << "\", \"strips\": " << r.strips << ", \"cols4\": " << r.cols4
        << ", \"split\": " << r.split << ", \"strips_mv\": " << r.strips_mv << ", \"cols4_mv\": " << r.cols4_mv
        << "}" << (++i < recs.size() ? "," : "") << "\n";
    }
    f << "]}\n";
    if (!f) throw Error(SSAMG_ERR_ARG, std::string("cannot write ") + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) throw Error(SSAMG_ERR_ARG, std::string("cannot write ") + path);
}

}  // namespace

extern "C" {

const char *ssamg_last_error(void) { return ssamg::g_last_error.c_str(); }

ssamg_status ssamg_params_default(ssamg_params *p) {
  API_BEGIN
  if (!p) throw Error(SSAMG_ERR_ARG, "NULL params");
  std::memset(p, 0, sizeof(*p));
  p->max_levels = 64;
  p->min_coarse_size = 0;
  p->relax = SSAMG_RELAX_JACOBI;
  p->omega = 0.0;
  p->coarse = SSAMG_COARSE_SWEEP;
  p->cycle_precision = SSAMG_FP64;
  p->tol = 1e-8;
  p->max_iter = 100;
  p->max_nrhs = 1;
  p->use_graph = 1;
  p->skip = 0;
  p->autotune = 0;
  p->symmetric = 1;
  p->pb_interp = SSAMG_PB_ONE;
  p->hybrid_level = 0;
  p->coarse_op = SSAMG_COARSE_OP_GALERKIN;
  API_END
}

ssamg_status ssamg_solver_create(ssamg_problem prob, const ssamg_params *params, void *hip_stream,
                                 ssamg_solver *out) {
  API_BEGIN
  if (!prob || !out) throw Error(SSAMG_ERR_ARG, "NULL problem or output");
  ssamg_params p;
  if (params)
    p = *params;
  else
    ssamg_params_default(&p);
  if (p.max_levels < 1) throw Error(SSAMG_ERR_ARG, "max_levels must be >= 1");
  if (p.min_coarse_size < 0) throw Error(SSAMG_ERR_ARG, "min_coarse_size must be >= 0");
  if (p.relax != SSAMG_RELAX_JACOBI && p.relax != SSAMG_RELAX_L1_JACOBI)
    throw Error(SSAMG_ERR_ARG, "relax must be SSAMG_RELAX_JACOBI or SSAMG_RELAX_L1_JACOBI");
  if (p.coarse != SSAMG_COARSE_SWEEP && p.coarse != SSAMG_COARSE_DIRECT)
    throw Error(SSAMG_ERR_ARG, "coarse must be SSAMG_COARSE_SWEEP or SSAMG_COARSE_DIRECT");
  if (p.skip != 0 && p.skip != 1) throw Error(SSAMG_ERR_ARG, "skip must be 0 or 1");
  if (p.autotune != 0 && p.autotune != 1) throw Error(SSAMG_ERR_ARG, "autotune must be 0 or 1");
  if (p.symmetric != 0 && p.symmetric != 1) throw Error(SSAMG_ERR_ARG, "symmetric must be 0 or 1");
  if (p.hybrid_level < 0) throw Error(SSAMG_ERR_ARG, "hybrid_level must be >= 0");
  if (p.coarse_op != SSAMG_COARSE_OP_GALERKIN && p.coarse_op != SSAMG_COARSE_OP_NONGALERKIN)
    throw Error(SSAMG_ERR_ARG, "coarse_op must be SSAMG_COARSE_OP_GALERKIN or SSAMG_COARSE_OP_NONGALERKIN");
  if (p.pb_interp != SSAMG_PB_ONE && p.pb_interp != SSAMG_PB_LUMP)
    throw Error(SSAMG_ERR_ARG, "pb_interp must be SSAMG_PB_ONE or SSAMG_PB_LUMP");
  if (p.cycle_precision != SSAMG_FP64 && p.cycle_precision != SSAMG_FP32)
    throw Error(SSAMG_ERR_ARG, "cycle_precision must be SSAMG_FP64 or SSAMG_FP32");
  if (!(p.tol > 0.0) || !std::isfinite(p.tol)) throw Error(SSAMG_ERR_ARG, "tol must be positive");
  if (p.max_iter < 1) throw Error(SSAMG_ERR_ARG, "max_iter must be >= 1");
  if (p.max_nrhs < 1 || p.max_nrhs > kMaxRhs || (p.max_nrhs & (p.max_nrhs - 1)))
    throw Error(SSAMG_ERR_ARG, "max_nrhs must be a power of two <= 32");
  if (!std::isfinite(p.omega) || p.omega >= 2.0) throw Error(SSAMG_ERR_ARG, "omega must be < 2");
  auto *s = new Solver();
  s->prob = reinterpret_cast<Problem *>(prob);
  s->prm = p;
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&s->stream) != hipSuccess) {
      delete s;
      throw Error(SSAMG_ERR_DEVICE, "hipStreamCreate failed");
    }
    s->own_stream = true;
  }
  const char *verbose = std::getenv("SSAMG_VERBOSE");
  s->verbose = verbose && verbose[0] && verbose[0] != '0';
  // cycle levels of at most this many elements run in the one-workgroup kernel
  const char *tail = std::getenv("SSAMG_TAIL_ELEMS");
  if (tail && tail[0]) s->tail_elems = std::min<int64_t>(kTailMax, std::max<int64_t>(0, std::atoll(tail)));
  const char *split = std::getenv("SSAMG_SPLIT_CELLS");
  if (split && split[0]) s->split_cells = std::max<int64_t>(0, std::atoll(split));
  const char *coll = std::getenv("SSAMG_COLLAPSE_CELLS");
  if (coll && coll[0]) s->collapse_cells = std::max<int64_t>(0, std::atoll(coll));
  const char *rapmin = std::getenv("SSAMG_RAP_CELL_MIN");
  if (rapmin && rapmin[0]) s->rap_cell_min = std::max<int64_t>(0, std::atoll(rapmin));
  const char *prod2 = std::getenv("SSAMG_PRODUCT2");
  if (prod2 && prod2[0]) s->product2 = std::max(0, std::min(2, std::atoi(prod2)));
  const char *sweepn = std::getenv("SSAMG_SWEEPN");
  if (sweepn && sweepn[0]) s->sweepn = std::atoi(sweepn) != 0;
  const char *fuse = std::getenv("SSAMG_FUSE_ZERO");
  if (fuse && fuse[0]) s->fuse_zero = std::atoi(fuse) != 0;
  const char *rsort = std::getenv("SSAMG_ROW_SORT");
  if (rsort && rsort[0]) s->scratch.row_sort = std::max<int64_t>(0, std::atoll(rsort));
  const char *hsym = std::getenv("SSAMG_HOST_SYM");
  if (hsym && hsym[0]) s->host_sym = std::max<int64_t>(0, std::atoll(hsym));
  void *pin = nullptr;
  if (hipHostMalloc(&pin, kScalSlots * kMaxRhs * sizeof(double)) != hipSuccess) {
    delete s;
    throw Error(SSAMG_ERR_ALLOC, "hipHostMalloc failed");
  }
  s->h_pin = (double *)pin;
  if (hipEventCreateWithFlags(&s->ev_scal, hipEventDisableTiming) != hipSuccess) {
    delete s;
    throw Error(SSAMG_ERR_DEVICE, "hipEventCreateWithFlags failed");
  }
  *out = reinterpret_cast<ssamg_solver>(s);
  API_END
}

ssamg_status ssamg_solver_destroy(ssamg_solver s) {
  API_BEGIN
  delete reinterpret_cast<Solver *>(s);
  API_END
}

ssamg_status ssamg_setup_symbolic(ssamg_solver h) {
  API_BEGIN
  setup_symbolic(*S(h));
  API_END
}

ssamg_status ssamg_workspace_bytes(ssamg_solver h, size_t *bytes) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  if (!bytes) throw Error(SSAMG_ERR_ARG, "NULL output");
  *bytes = s->ws_bytes;
  API_END
}

ssamg_status ssamg_setup_numeric(ssamg_solver h, void *ws, size_t bytes) {
  API_BEGIN
  setup_numeric(*S(h), ws, bytes);
  API_END
}

ssamg_status ssamg_update_coeffs(ssamg_solver h, int part, const double *vals, int where) {
  API_BEGIN
  Solver *s = S(h);
  const ssamg_status st = ssamg_problem_set_coeffs((ssamg_problem)s->prob, part, vals, where, 0);
  if (st != SSAMG_OK) return st;
  s->state = 0;
  API_END
}

ssamg_status ssamg_solve(ssamg_solver h, int nrhs, const double *b, double *x, int layout,
                         ssamg_info *info) {
  Solver *s = nullptr;
  try {
    s = S(h);
    need(s, 2, "setup_numeric must come first");
    if (!b || !x) throw Error(SSAMG_ERR_ARG, "NULL vector");
    if (nrhs < 1 || nrhs > s->prm.max_nrhs || (nrhs & (nrhs - 1)))
      throw Error(SSAMG_ERR_ARG, "nrhs must be a power of two <= max_nrhs");
    if (layout != SSAMG_LAYOUT_CELL_MAJOR && layout != SSAMG_LAYOUT_RHS_MAJOR)
      throw Error(SSAMG_ERR_ARG, "layout must be SSAMG_LAYOUT_CELL_MAJOR or SSAMG_LAYOUT_RHS_MAJOR");
    ssamg_status st;
    if (layout == SSAMG_LAYOUT_RHS_MAJOR && nrhs > 1) {
      const int lg = width_lg(s, nrhs);
      const int64_t n = s->lv[0].N;
      const size_t bytes = (size_t)n * nrhs * sizeof(double);
      s->lay_b.reserve(bytes);
      s->lay_x.reserve(bytes);
      double *bt = (double *)s->lay_b.p, *xt = (double *)s->lay_x.p;
      launch_transpose(b, bt, n, lg, 1, s->stream);
      SSAMG_HIP(hipGetLastError());
      st = pcg_solve(*s, nrhs, bt, xt, info);
      launch_transpose(xt, x, n, lg, 0, s->stream);
      SSAMG_HIP(hipGetLastError());
      SSAMG_HIP(hipStreamSynchronize(s->stream));
    } else {
      st = pcg_solve(*s, nrhs, b, x, info);
    }
    set_last_error(st == SSAMG_OK ? "" : "not converged within max_iter");
    return st;
  } catch (const Error &e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return SSAMG_ERR_ARG;
  }
}

ssamg_status ssamg_autotune(ssamg_solver h, int nrhs, const char *cache_path) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  const int lg = width_lg(s, nrhs);
  std::map<std::string, TuneRec> file;
  if (cache_path) {
    file = read_cache(cache_path);
    for (int l = 0; l < (int)s->lv.size(); ++l) {
      bool have = false;
      (void)tune_rec(*s, l, lg, &have);
      auto it = file.find(tune_key(*s, l, lg));
      if (!have && it != file.end()) tune_store(*s, l, lg, it->second);
    }
  }
  autotune(*s, lg);
  if (cache_path) {
    for (const auto &kv : s->tune) file[kv.first] = kv.second;
    write_cache(cache_path, file);
  }
  API_END
}

ssamg_status ssamg_tune_get(ssamg_solver h, int level, int nrhs, int rec[6]) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  check_level(s, level);
  if (!rec) throw Error(SSAMG_ERR_ARG, "NULL output");
  bool found = false;
  const TuneRec r = tune_rec(*s, level, width_lg(s, nrhs), &found);
  rec[0] = r.strips;
  rec[1] = r.cols4;
  rec[2] = r.split;
  rec[3] = r.strips_mv;
  rec[4] = r.cols4_mv;
  rec[5] = found ? 1 : 0;
  API_END
}

ssamg_status ssamg_tune_set(ssamg_solver h, int level, int nrhs, const int rec[5]) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  check_level(s, level);
  if (!rec) throw Error(SSAMG_ERR_ARG, "NULL record");
  TuneRec r;
  r.strips = rec[0];
  r.cols4 = rec[1];
  r.split = rec[2];
  r.strips_mv = rec[3];
  r.cols4_mv = rec[4];
  tune_store(*s, level, width_lg(s, nrhs), r);
  API_END
}

ssamg_status ssamg_apply_A(ssamg_solver h, int level, const double *x, double *y) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  check_level(s, level);
  if (!x || !y) throw Error(SSAMG_ERR_ARG, "NULL vector");
  apply_level(*s, level, x, y);
  API_END
}

ssamg_status ssamg_apply_precond(ssamg_solver h, const double *r, double *z) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  if (!r || !z) throw Error(SSAMG_ERR_ARG, "NULL vector");
  apply_precond(*s, r, z);
  API_END
}

ssamg_status ssamg_level_cells(ssamg_solver h, int level, int64_t *ncell) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  check_level(s, level);
  if (!ncell) throw Error(SSAMG_ERR_ARG, "NULL output");
  *ncell = s->lv[level].N;
  API_END
}

ssamg_status ssamg_num_levels(ssamg_solver h, int *nlevels) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  if (!nlevels) throw Error(SSAMG_ERR_ARG, "NULL output");
  *nlevels = (int)s->lv.size();
  API_END
}

ssamg_status ssamg_level_info(ssamg_solver h, int level, int part, ssamg_level_desc *info) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  check_part(s, level, part);
  if (!info) throw Error(SSAMG_ERR_ARG, "NULL output");
  const PartLevel &q = s->lv[level].parts[part];
  std::memset(info, 0, sizeof(*info));
  for (int d = 0; d < 3; ++d) {
    info->dims[d] = q.n[d];
    info->fdims[d] = q.fn[d];
  }
  info->offset = q.off;
  info->dstar = q.dstar;
  info->omega = q.omega;
  info->nent = (int)q.pat.size();
  info->skip = q.skip ? 1 : 0;
  for (size_t e = 0; e < q.pat.size(); ++e)
    for (int d = 0; d < 3; ++d) info->pattern[e][d] = q.pat[e][d];
  API_END
}

ssamg_status ssamg_direction_sums(ssamg_solver h, double *c_out) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  if (!c_out) throw Error(SSAMG_ERR_ARG, "NULL output");
  std::memcpy(c_out, s->cd.data(), s->cd.size() * sizeof(double));
  API_END
}

ssamg_status ssamg_copy_stencil(ssamg_solver h, int level, int part, double *vals) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  check_part(s, level, part);
  if (!vals) throw Error(SSAMG_ERR_ARG, "NULL output");
  const PartLevel &q = s->lv[level].parts[part];
  SSAMG_HIP(hipStreamSynchronize(s->stream));
  SSAMG_HIP(hipMemcpy(vals, q.coef64, q.pat.size() * q.ncell * sizeof(double), hipMemcpyDeviceToHost));
  API_END
}

ssamg_status ssamg_copy_interp(ssamg_solver h, int level, int part, double *wm, double *wp) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  check_part(s, level, part);
  if (!wm || !wp) throw Error(SSAMG_ERR_ARG, "NULL output");
  const Level &V = s->lv[level];
  const PartLevel &q = V.parts[part];
  if (q.nf == 0) return SSAMG_OK;
  SSAMG_HIP(hipStreamSynchronize(s->stream));
  SSAMG_HIP(hipMemcpy(wm, V.d_w64 + q.wofs, q.nf * sizeof(double), hipMemcpyDeviceToHost));
  SSAMG_HIP(hipMemcpy(wp, V.d_w64 + q.wofs + q.nf, q.nf * sizeof(double), hipMemcpyDeviceToHost));
  API_END
}

ssamg_status ssamg_probe_set(ssamg_solver h, int kind) {
  API_BEGIN
  Solver *s = S(h);
  if (kind < SSAMG_PROBE_NONE || kind > SSAMG_PROBE_JACOBI0) throw Error(SSAMG_ERR_ARG, "bad probe kind");
  probe_set(*s, kind);
  API_END
}

ssamg_status ssamg_probe_read(ssamg_solver h, int64_t *launches, double *total_ms, double *alg_bytes) {
  API_BEGIN
  Solver *s = S(h);
  if (!launches || !total_ms || !alg_bytes) throw Error(SSAMG_ERR_ARG, "NULL output");
  probe_read(*s, launches, total_ms, alg_bytes);
  API_END
}

ssamg_status ssamg_coupling_nnz(ssamg_solver h, int level, int64_t *nnz) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 1, "setup_symbolic must come first");
  check_level(s, level);
  if (!nnz) throw Error(SSAMG_ERR_ARG, "NULL output");
  *nnz = s->lv[level].nnz;
  API_END
}

ssamg_status ssamg_copy_coupling(ssamg_solver h, int level, int64_t *rowptr, int64_t *col, double *val) {
  API_BEGIN
  Solver *s = S(h);
  need(s, 2, "setup_numeric must come first");
  check_level(s, level);
  if (!rowptr || !col || !val) throw Error(SSAMG_ERR_ARG, "NULL output");
  const Level &V = s->lv[level];
  const size_t nnz = (size_t)V.nnz, nrow = (size_t)V.nrow;
  std::vector<double> hv(nnz);
  std::vector<int> urow(nrow), uptr(nrow + 1, 0), ucol(nnz);
  SSAMG_HIP(hipStreamSynchronize(s->stream));
  if (nnz) {
    SSAMG_HIP(hipMemcpy(hv.data(), V.d_uval64, nnz * sizeof(double), hipMemcpyDeviceToHost));
    SSAMG_HIP(hipMemcpy(urow.data(), V.d_urow, nrow * sizeof(int), hipMemcpyDeviceToHost));
    SSAMG_HIP(hipMemcpy(uptr.data(), V.d_uptr, (nrow + 1) * sizeof(int), hipMemcpyDeviceToHost));
    SSAMG_HIP(hipMemcpy(ucol.data(), V.d_ucol, nnz * sizeof(int), hipMemcpyDeviceToHost));
  }
  for (int64_t i = 0; i <= V.N; ++i) rowptr[i] = 0;
  for (size_t r = 0; r < nrow; ++r) rowptr[urow[r] + 1] = uptr[r + 1] - uptr[r];
  for (int64_t i = 0; i < V.N; ++i) rowptr[i + 1] += rowptr[i];
  for (size_t k = 0; k < nnz; ++k) {
    col[k] = ucol[k];
    val[k] = hv[k];
  }
  API_END
}

}  // extern "C"
