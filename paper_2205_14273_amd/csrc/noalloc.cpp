// A solve that allocates no device memory (ssamg_solve_noalloc): the PCG work
// vectors, the reduction partials and scalars and, for right-hand-side-major
// vectors, the layout staging come from one fixed device array per GPU instead
// of the solver's workspace or the layout buffers ssamg_solve allocates.
#include <cstring>
#include <mutex>

#include "capi_common.h"
#include "ssamg_impl.h"

using namespace ssamg;

namespace {

constexpr size_t kScratchBytes = SSAMG_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchAlign = 256;

// Every GPU that loads the library holds its own copy of this array until the
// process ends.  In host code `scratch` only names the symbol: its device
// address on the current GPU comes from hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of the current GPU's array, looked up once per device with
// that device current.
void *scratch_ptr() {
  int dev = 0;
  SSAMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(SSAMG_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    SSAMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(SSAMG_ERR_DEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

// Carves the fixed array like the workspace (base = nullptr: sizing only).
struct Bump {
  char *base = nullptr;
  size_t off = 0;
  template <typename T>
  T *take(size_t n) {
    off = (off + kScratchAlign - 1) & ~(kScratchAlign - 1);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

struct SolveScratch {
  double *r, *z, *p, *q, *partial, *dotp, *scal, *bt, *xt;
  int *active;
};

// The buffers one solve of width 2^lg reads and writes besides b and x: the
// same list, in the same sizes for that width, as the workspace holds.
SolveScratch carve_solve(const Solver &s, Bump &bp, int lg, bool staging) {
  const size_t nel = (size_t)s.lv[0].N << lg;
  SolveScratch c{};
  c.r = bp.take<double>(nel);
  c.z = bp.take<double>(nel);
  c.p = bp.take<double>(nel);
  c.q = bp.take<double>(nel);
  c.partial = bp.take<double>((size_t)2 * kRedBlocks * kMaxRhs);
  const int64_t slots = (int64_t)s.lv[0].parts.size() * dot_slots(s.lv[0].maxcell, lg) << lg;
  c.dotp = bp.take<double>((size_t)2 * slots);
  c.scal = bp.take<double>((size_t)kScalSlots * kMaxRhs);
  c.active = bp.take<int>(kMaxRhs);
  c.bt = staging ? bp.take<double>(nel) : nullptr;
  c.xt = staging ? bp.take<double>(nel) : nullptr;
  return c;
}

// Points the solver's PCG buffers at the scratch for the duration of one call.
// A cycle graph not yet instantiated for this width is not built here (that
// would allocate): the call then launches the coarse levels directly.
struct Redirect {
  Solver &s;
  double *r, *z, *p, *q, *partial, *dotp, *scal;
  int *active;
  int use_graph;
  Redirect(Solver &sv, const SolveScratch &c, int nrhs)
      : s(sv), r(sv.r), z(sv.z), p(sv.p), q(sv.q), partial(sv.partial), dotp(sv.dotp), scal(sv.scal),
        active(sv.active), use_graph(sv.prm.use_graph) {
    if (!s.graph_exec || s.graph_nrhs != nrhs) s.prm.use_graph = 0;
    s.r = c.r;
    s.z = c.z;
    s.p = c.p;
    s.q = c.q;
    s.partial = c.partial;
    s.dotp = c.dotp;
    s.scal = c.scal;
    s.active = c.active;
  }
  ~Redirect() {
    s.prm.use_graph = use_graph;
    s.r = r;
    s.z = z;
    s.p = p;
    s.q = q;
    s.partial = partial;
    s.dotp = dotp;
    s.scal = scal;
    s.active = active;
  }
};

}  // namespace

extern "C" {

ssamg_status ssamg_solve_noalloc(ssamg_solver h, int nrhs, const double *b, double *x, int layout,
                                 ssamg_info *info) {
  try {
    if (!h) throw Error(SSAMG_ERR_ARG, "NULL solver");
    Solver &s = *reinterpret_cast<Solver *>(h);
    if (s.state < 2) throw Error(SSAMG_ERR_STATE, "setup_numeric must come first");
    if (!b || !x) throw Error(SSAMG_ERR_ARG, "NULL vector");
    if (nrhs < 1 || nrhs > s.prm.max_nrhs || (nrhs & (nrhs - 1)))
      throw Error(SSAMG_ERR_ARG, "nrhs must be a power of two <= max_nrhs");
    if (layout != SSAMG_LAYOUT_CELL_MAJOR && layout != SSAMG_LAYOUT_RHS_MAJOR)
      throw Error(SSAMG_ERR_ARG, "layout must be SSAMG_LAYOUT_CELL_MAJOR or SSAMG_LAYOUT_RHS_MAJOR");
    int lg = 0;
    while ((1 << lg) < nrhs) ++lg;
    if (s.prm.autotune && !tuned(s, lg))
      throw Error(SSAMG_ERR_STATE, "autotune = 1: run ssamg_autotune (or ssamg_solve) for this width first");
    const bool staging = layout == SSAMG_LAYOUT_RHS_MAJOR && nrhs > 1;
    Bump sizing;
    (void)carve_solve(s, sizing, lg, staging);
    if (sizing.off > kScratchBytes)
      throw Error(SSAMG_ERR_ARG, "this solve needs " + std::to_string(sizing.off) +
                                     " bytes of scratch; the fixed array holds " +
                                     std::to_string(kScratchBytes) + " (use ssamg_solve)");
    Bump bp;
    bp.base = static_cast<char *>(scratch_ptr());
    const SolveScratch c = carve_solve(s, bp, lg, staging);
    ssamg_status st;
    {
      Redirect red(s, c, nrhs);
      if (staging) {
        const int64_t n = s.lv[0].N;
        launch_transpose(b, c.bt, n, lg, 1, s.stream);
        SSAMG_HIP(hipGetLastError());
        st = pcg_solve(s, nrhs, c.bt, c.xt, info);
        launch_transpose(c.xt, x, n, lg, 0, s.stream);
        SSAMG_HIP(hipGetLastError());
        SSAMG_HIP(hipStreamSynchronize(s.stream));
      } else {
        st = pcg_solve(s, nrhs, b, x, info);
      }
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

}  // extern "C"
