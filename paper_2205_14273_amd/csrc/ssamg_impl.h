// Internal declarations of the SSAMG library: host-side hierarchy objects,
// the device-side per-part descriptors read by every kernel, and the kernel
// launchers.  Not part of the ABI (include/ssamg.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <memory>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ssamg.h"

namespace ssamg {

struct Error : std::runtime_error {
  ssamg_status code;
  Error(ssamg_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define SSAMG_HIP(call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::ssamg::Error(SSAMG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxEnt = 27;      // stencils live in the 27-point neighbourhood
constexpr int kBlock = 256;      // threads per block of every grid-over-cells kernel
constexpr int kRedBlocks = 2048; // fixed grid of the deterministic reductions (8 per CU)
constexpr int kMaxRhs = 32;
constexpr int kMaxLg = 5;        // log2(kMaxRhs)
// The coarse end of the cycle runs in one workgroup of kTailThreads threads
// (half of them in FP64): the coarsest level and the levels of at most
// tail_elems elements (cells x right-hand sides; never more than kTailMax).
// The levels' vectors live in LDS (at most kTailLds bytes; fewer levels are
// taken when they do not fit) and their operators are packed in level-wide
// arrays, so each phase of the kernel waits on one round of coalesced loads
// and LDS gathers instead of a launch and a chain of dependent loads.
// kTailUPer coupling products per thread are staged per pass.
constexpr int kTailThreads = 1024;
constexpr int kTailMax = 4096;
constexpr int kTailUPer = 4;   // coupling products staged per thread and pass (4096 in FP32, 2048 in FP64)
constexpr int64_t kTailElems = 1024;          // one or two right-hand sides
constexpr int64_t kTailElemsBatched = 2048;   // four or more (measured on 2 x 96^3, 32 rhs)
constexpr int kTailLds = 65536;
// The cycle below the first level of at most kCollapseCells cells (when that
// level is not the coarsest) is a fixed linear map of its right-hand side; it
// is formed at numeric setup as a dense FP64 matrix (one column per unit
// right-hand side, by the coarse-end kernel itself) and applied in its place.
constexpr int64_t kCollapseCells = 128;
// coarse coupling structures whose product emits at most this many records
// (four per fine entry) are formed on the host: below it a handful of
// microseconds of host work beats the ten launches and the synchronisation
// of the device sort
constexpr int64_t kHostSymRecords = 16384;
// coupling-product records of a coarse row ranked in LDS (rows with more are
// ranked from memory); SSAMG_ROW_SORT lowers it (0: every row from memory)
constexpr int64_t kRowSortRecords = 512;
// levels with more than 15-point stencils and at least this many cells run the
// first smoothing sweep and the residual as two kernels instead of one
constexpr int64_t kSplitCells = 1 << 20;
// largest coarsest level the direct solve accepts (its inverse is formed in LDS)
constexpr int kDirectMax = 64;
// largest switch level of the hybrid tail (dense FP64 inverse of at most 2 GiB)
constexpr int64_t kDenseMax = 16384;
// coarse levels of at least this many cells (over all parts) take the
// one-thread-per-coarse-cell Galerkin kernel; smaller ones one thread per
// (coarse cell, entry), whose shorter gather chains win when threads are few
constexpr int64_t kRapCellMin = 3 << 16;
// the autotuner times a level's launch options only if the level holds at
// least this many (cell, right-hand side) elements; below it launches are
// latency-bound and the defaults stand
constexpr int64_t kTuneMinElems = 1 << 16;
// strip counts per z-plane the autotuner tries for the four-column sweeps
constexpr int kTuneStrips[] = {1, 2, 3, 4, 6, 8};

// Launch options of one level's cycle for one batch width (autotuned, or set
// through the C ABI); every option gives bit-identical results.
struct TuneRec {
  int strips = 1;      // z-plane strips of the four-column sweeps' block order (1: plain order)
  int cols4 = -1;      // stencil sweeps: four columns per thread (1), one (0), default (-1)
  int split = -1;      // first sweep: split from the residual (1), fused (0), default rule (-1)
  int strips_mv = 1;   // level 0, FP64 product of PCG in a mixed-precision cycle: strips
  int cols4_mv = -1;   // and its columns per thread
};

// Packed stencil offset: (dx+1) | (dy+1) << 2 | (dz+1) << 4.
inline int pack_off(int dx, int dy, int dz) { return (dx + 1) | ((dy + 1) << 2) | ((dz + 1) << 4); }

// One part at one level, as seen by the kernels (lives in device memory; every
// kernel indexes it with blockIdx.y, so its fields are wave-uniform).
template <typename T>
struct PartDesc {
  int n[3];            // box extents
  int nent;            // stencil entries
  int center;          // index of (0,0,0) in the stencil
  int dstar;           // semicoarsening direction to the next level, -1: identity
  int faces;           // bit f set: face f (-x,+x,-y,+y,-z,+z) is a part boundary
  int fn[3];           // F-box extents (cells odd along dstar)
  int cn[3];           // coarse box extents
  int pblump;          // 1: lumped part-boundary interpolation (SSAMG_PB_LUMP)
  long long off;       // first cell of the part in the level vector
  long long ncell;
  long long coff;      // first cell of the part in the next level vector
  long long cncell;
  long long nf;        // cells of the F-box
  T omega;             // relaxation weight
  const T *coef;       // [nent][ncell]
  const T *wm;         // [nf] weight toward the -dstar coarse neighbour
  const T *wp;         // [nf] weight toward the +dstar coarse neighbour
  // couplings U of the level (compressed rows, shared by all parts); the rows
  // of the part's block `b` of a grid-over-cells launch with 1 << lg
  // right-hand sides are urow[ublk[lg][2b] .. ublk[lg][2b+2]) and their
  // entries ucol[ublk[lg][2b+1] .. ublk[lg][2b+3])
  const int *urow;     // cell id of each stored row (ascending)
  const int *uptr;
  const int *ucol;
  const T *uval;
  const int *ublk[kMaxLg + 1];
  // block order of the four-columns-per-thread sweeps at each lg: blocks per
  // z-plane (0: planes do not split into whole blocks) and strip width in
  // blocks (0: plain order)
  int tbp[kMaxLg + 1];
  int tsb[kMaxLg + 1];
  // per-cell smoother factor (weighted L1-Jacobi: factor / sum_j |a_ij|);
  // null: weighted Jacobi omega / a_ii
  const T *rs;
  int lin[kMaxEnt];    // dx + nx*(dy + ny*dz)
  int code[kMaxEnt];   // pack_off(dx, dy, dz)
  // where the cycle and product kernels read a_s(c): entry mir[s] at cell
  // c + mlin[s].  Symmetric stencils: an entry with a negative offset s is
  // read as the mirrored entry -s of the neighbour c + s (a_s(c) = a_{-s}(c+s)),
  // so only the center and the positive half are streamed; otherwise mir[s] =
  // s, mlin[s] = 0.
  int mir[kMaxEnt];
  int mlin[kMaxEnt];
  // interpolation weights (FP64 descriptors only): the collapse sums take the
  // entries in the order wsum[0 .. nent) (the order in which the Galerkin
  // product forms a coarse row, so both kernels round alike); wfused: that
  // product has already written this part's weights
  int wsum[kMaxEnt];
  int wfused;
  // finest level of an assembled problem: the collapse sums along dstar
  // (den, sm, sp blocks of nf) that the assembly formed in the order of wsum,
  // or null
  const double *csum;
  // lin[s] * 64 + code[s] (code < 64): the small-level sweeps read one scalar
  // per entry, which keeps the 27-point tables within the scalar registers
  int lc[kMaxEnt];
  // entry of each offset, cube index (dx+1) + 3(dy+1) + 9(dz+1); -1: none
  int cube[27];
};

// ------------------------------------------------------------------ problem

struct Problem {
  int ndim = 3, nparts = 0;
  std::vector<std::array<int, 3>> dims;
  std::vector<std::array<int, 3>> origin;
  std::vector<int> has_origin;
  std::vector<std::array<int, 6>> faces;
  std::vector<std::vector<std::array<int, 3>>> stencil;
  std::vector<int> center;
  std::vector<double *> coef;        // device [nent][ncell] per part, problem-owned
  std::vector<int> coef_set;
  // every change of coefficients bumps coef_version; finite-volume assembly
  // also leaves the per-block partial sums of the direction metric c_d
  // (Section 3.1; [part][block][3], mpart_nb blocks per part), valid while
  // metric_version == coef_version
  uint64_t coef_version = 1, metric_version = 0;
  double *d_mpart = nullptr;
  size_t mpart_cap = 0;
  int mpart_nb = 0;
  // the same assembly's collapse sums of every cell odd along a direction d,
  // per part and direction in that direction's F-box order: den, sm and sp
  // (as the interpolation weights take them), each of nf_d doubles, from
  // d_csum + csum_off[3 p + d]; valid with the metric
  double *d_csum = nullptr;
  size_t csum_cap = 0;
  long long *d_csoff = nullptr;
  std::vector<long long> csum_off;
  // 1: the part's given coefficients satisfy a_s(c) = a_{-s}(c+s) to a relative
  // 1e-12 (checked by set_coeffs; finite-volume assembly is symmetric)
  std::vector<int> sym_ok;
  // parts of several boxes: inclusive sub-boxes {lo[3], hi[3]} of the part's
  // box (empty: the whole box); cells in none of them are ghost unknowns
  std::vector<std::vector<std::array<int, 6>>> boxes;
  // glued faces: face f of part p continues into part `part` through an
  // index map (point `at` across the face is `nbr_at` there; axis d maps to
  // axis map[d] with direction dir[d])
  struct Glue {
    int part = -1;
    int at[3], nbr_at[3], map[3], dir[3];
  };
  std::vector<std::array<Glue, 6>> glue;
  // couplings as given (COO, host) and the entries of each part's stencils
  // that cross a glued face, moved to U by set_coeffs
  std::vector<int64_t> ucoo_row, ucoo_col;
  std::vector<double> ucoo_val;
  std::vector<std::vector<int64_t>> ux_row, ux_col;
  std::vector<std::vector<double>> ux_val;
  bool has_topology() const;
  // couplings, canonical compressed-row CSR (host copy + device copy)
  std::vector<int> urow, uptr, ucol;
  std::vector<double> uval_host;
  int *d_urow = nullptr, *d_uptr = nullptr, *d_ucol = nullptr;
  double *d_uval = nullptr;
  bool coupling_set = false;
  // finite-volume description of the last fv_assemble
  int fv_stencil = 0;
  double *d_kappa = nullptr;
  double *d_aniso = nullptr;
  int *d_ucode = nullptr;            // per coupling entry: offset code | p_i << 6 | p_j << 19
  int *d_geom = nullptr;             // per part: origin[3], dims[3], offset
  double **d_cptr = nullptr;         // device copy of coef[]
  std::vector<int> fv_signature;     // placement + stencil the FV structure was built for
  bool fv_structure_ready = false;
  int64_t ncell_total() const;
  std::vector<int64_t> offsets() const;
  void free_device();
  ~Problem() { free_device(); }
};

// ------------------------------------------------------------------ hierarchy

struct PartLevel {
  std::array<int, 3> n{}, fn{}, cn{};
  int64_t off = 0, ncell = 0, coff = 0, cncell = 0, nf = 0;
  int dstar = -1;
  double omega = 0.0;
  int faces = 0;
  bool skip = false;                 // no relaxation on this part at this level (skip option)
  std::vector<std::array<int, 3>> pat;
  int center = 0;
  double *coef64 = nullptr;
  float *coef32 = nullptr;
  int64_t wofs = 0;                  // offset of wm in the level weight buffer (wp at +nf)
  // Galerkin product toward the next level: entry maps over the 27 offsets
  // (see RapDesc)
  std::array<int, 27> rap_fmap{}, rap_cmap{}, rap_cofs{};
  int rap_nent = 0;
  bool rap_ng = false;               // non-Galerkin coarse stencil (SSAMG_COARSE_OP_NONGALERKIN)
};

// Growable device buffer (kept across setups; reallocated only to grow).
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  void reserve(size_t bytes);
  ~DevBuf();
};

// Part geometry read by the symbolic coupling kernels.
struct SymPart {
  int n[3], cn[3], fn[3];
  int dstar;
  long long off, ncell, coff, nf, wofs;
};

// Device structure of one level's couplings and its Galerkin recipe.
struct CouplingStore {
  DevBuf urow, uptr, ucol, erow, start, ck, ca, cb;
  int64_t ncontrib = 0;
};

struct LevelStore {
  CouplingStore cpl;
  DevBuf ublk[kMaxLg + 1];
};

// Scratch of the device sort.
struct SymScratch {
  DevBuf key0, key1, idx0, idx1, rk, ra, rb, ent, temp, rcnt, roff, rinfo, rscan;
  int *host_small = nullptr;         // pinned, coherent: the three sizes of the last call
  int *dev_small = nullptr;          // its device address
  int64_t row_sort = kRowSortRecords; // rows of at most this many records are ranked in LDS
  // rcnt and rinfo are all zero between calls (each call leaves them so); the
  // allocation (pointer, capacity) that was last cleared, null when unknown
  const void *rcnt_zero = nullptr, *rinfo_zero = nullptr;
  size_t rcnt_zcap = 0, rinfo_zcap = 0;
  ~SymScratch() {
    if (host_small) (void)hipHostFree(host_small);
  }
};

struct Level {
  std::vector<PartLevel> parts;
  int64_t N = 0;
  int maxcell = 0, maxcoarse = 0, maxf = 0, maxent = 0;
  // couplings (compressed rows, device; level 0 belongs to the problem)
  int nrow = 0;
  int64_t nnz = 0, ncontrib = 0;
  int *d_urow = nullptr, *d_uptr = nullptr, *d_ucol = nullptr;
  int *d_erow = nullptr;             // row cell of every entry
  double *d_uval64 = nullptr;
  float *d_uval32 = nullptr;
  // per-cell smoother factors of weighted L1-Jacobi (null for weighted Jacobi)
  double *d_rs64 = nullptr;
  float *d_rs32 = nullptr;
  // first coupling row of every block of a grid-over-cells launch, per lg
  int64_t ublk_len[kMaxLg + 1] = {};
  std::vector<int64_t> ublk_off[kMaxLg + 1];   // per part
  int *d_ublk[kMaxLg + 1] = {};
  // recipe of this level's U as P^T U P from the previous level
  int *d_uc_start = nullptr, *d_uc_k = nullptr, *d_uc_a = nullptr, *d_uc_b = nullptr;
  // interpolation weights of all parts toward the next level
  int64_t nw = 0;
  double *d_w64 = nullptr;
  float *d_w32 = nullptr;
  PartDesc<double> *d_desc64 = nullptr;
  PartDesc<float> *d_desc32 = nullptr;
  struct RapDesc *d_rapdesc = nullptr;
  double *d_ainv = nullptr;          // coarsest level, direct solve: dense inverse
  void *d_tail = nullptr;            // TailLevel<cycle precision> of this level
  void *d_ctail = nullptr;           // the same, except at the collapse level (its operator as the end)
  double *d_mcyc = nullptr;          // collapse level: the collapsed cycle's matrix, [N][N] by columns
  // operator pack of the coarse-end kernel (levels 1 .. L-2 of at most
  // kTailMax cells; see TailLevel), cycle precision
  int *d_pk_nb = nullptr, *d_pk_pi = nullptr, *d_pk_ri = nullptr, *d_pk_row = nullptr;
  void *d_pk_ca = nullptr, *d_pk_pw = nullptr, *d_pk_rw = nullptr;
  // V-cycle vectors in the cycle precision: [N][max_nrhs]
  void *vb = nullptr, *vx = nullptr, *vt = nullptr;
  bool cycle32 = false;              // this level's cycle runs in FP32
};

struct Solver {
  Problem *prob = nullptr;
  ssamg_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool verbose = false;              // SSAMG_VERBOSE: phase timings on stderr
  int64_t tail_elems = -1;           // SSAMG_TAIL_ELEMS overrides (-1: kTailElems / kTailElemsBatched)
  int64_t split_cells = kSplitCells; // SSAMG_SPLIT_CELLS overrides
  int64_t host_sym = kHostSymRecords; // SSAMG_HOST_SYM overrides (0: device only)
  int64_t collapse_cells = kCollapseCells;   // SSAMG_COLLAPSE_CELLS overrides (0: off)
  int64_t rap_cell_min = kRapCellMin;        // SSAMG_RAP_CELL_MIN overrides (0: per-cell kernel always)
  bool x0_ready = false;                     // the finest level's x = w r is formed (next cycle skips it)
  bool fuse_zero = true;                     // SSAMG_FUSE_ZERO=0: first sweeps from zero run on their own
                                             // (not formed by PCG's residual update or the restriction)
  int product2 = 1;                          // SSAMG_PRODUCT2=0: the one-cell product and sweeps everywhere;
                                             // 1: two-cell product loading its row neighbours;
                                             // 2: ... taking them from the adjacent lanes
  int sweepn = 1;                            // SSAMG_SWEEPN=0: the one-cell finest sweeps
  int lk = -1;                       // collapse level (-1: none)
  DevBuf host_cpl;                   // couplings and block tables of the host-formed levels
  hipEvent_t ev_scal = nullptr;      // PCG: the scalars of an iteration have reached the host
  int state = 0;                     // 0 created, 1 symbolic done, 2 numeric done
  double t_sym = 0.0, t_num = 0.0;   // host seconds of the last symbolic and numeric setup
  // RHS-major solves: the right-hand sides and solutions in [N][nrhs] order
  DevBuf lay_b, lay_x;
  std::vector<Level> lv;
  std::vector<double> cd;            // direction sums c[p][d]
  // device buffers of the symbolic setup, kept across setups
  std::vector<std::unique_ptr<LevelStore>> store;
  SymScratch scratch;
  DevBuf symtab, wsum_buf;
  // workspace
  size_t ws_bytes = 0;
  void *ws = nullptr;
  bool ws_owned = false;
  // PCG vectors (FP64, [N0][max_nrhs])
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *partial = nullptr;         // [2][kRedBlocks][kMaxRhs]
  double *dotp = nullptr;            // p.q partials of the batched FP64 product (MODE_APPLY_DOT)
  double *scal = nullptr;            // [kScalSlots][kMaxRhs]
  int *active = nullptr;             // [kMaxRhs]
  int *flag = nullptr;               // device error flag
  double *h_pin = nullptr;           // pinned host mirror of a few scalar slots
  // pinned staging of the numeric setup's host-built tables (one asynchronous
  // copy); busy while a copy from it may still be in flight
  void *h_tab = nullptr;
  size_t h_tab_cap = 0;
  bool h_tab_busy = false;
  // hybrid tail (hybrid_level > 0): dense inverse of the coarsest level, padded
  // to a multiple of 64 (row-major, symmetric), and its scratch
  double *d_hyb = nullptr, *d_hyb_pt = nullptr, *d_hyb_dinv = nullptr, *d_hyb_part = nullptr;
  // graph of one V-cycle
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_nrhs = 0;
  // HIP-event timing of one finest-level kernel kind (SSAMG_PROBE_*)
  int probe_kind = -1;
  std::vector<hipEvent_t> pev;
  size_t pev_next = 0;
  int64_t probe_launches = 0;
  double probe_bytes = 0.0;
  // autotuned launch options, keyed by level signature and lg (kept across
  // setups: a level with the same shape finds its record again)
  std::map<std::string, TuneRec> tune;
  std::vector<std::string> sig;      // signature of each level of the current hierarchy
  double tune_s = 0.0;               // seconds spent timing candidates
  ~Solver();
};

void setup_symbolic(Solver &s);
void setup_numeric(Solver &s, void *ws, size_t bytes);
void apply_level(Solver &s, int level, const double *x, double *y);
void apply_precond(Solver &s, const double *r, double *z);
ssamg_status pcg_solve(Solver &s, int nrhs, const double *b, double *x, ssamg_info *info);
void probe_set(Solver &s, int kind);
void probe_read(Solver &s, int64_t *launches, double *ms, double *bytes);
// launch options of level l for width 2^lg: the stored record or defaults
TuneRec tune_rec(const Solver &s, int l, int lg, bool *found = nullptr);
void tune_store(Solver &s, int l, int lg, const TuneRec &r);   // validates, re-uploads descriptors
int autotune(Solver &s, int lg);   // times candidates of every untuned level; returns levels tuned
bool tuned(const Solver &s, int lg);
std::string tune_key(const Solver &s, int l, int lg);

enum ScalSlot { S_RZ = 0, S_RZN, S_PQ, S_RR, S_ZQ, S_BB, S_TR, S_ALPHA, kScalSlots };

// ------------------------------------------------------------------ launchers

// one part's box + stencil, passed by value to the per-part setup kernels
struct BoxStencil {
  int n[3];
  int nent;
  int center;
  int pad;
  long long ncell;
  int code[kMaxEnt];
  int lin[kMaxEnt];    // dx + nx*(dy + ny*dz)
  int mir[kMaxEnt];    // entry with the opposite offset, -1 if none
  double *coef;
};

// One level of the coarse end of the cycle run by the one-workgroup kernel.
// Levels 1 .. of at most kTailMax cells also carry a pack of their operators
// in level-wide arrays (written by k_tail_pack at numeric setup), so that the
// kernel finds every operand from the cell index alone: the stencil as
// (neighbour cell, coefficient) pairs, P and P^T as index and weight lists.
// Absent entries point at the cell itself with weight 0, which leaves the
// sums of the grid kernels unchanged.
template <typename T>
struct TailLevel {
  const PartDesc<T> *desc;          // parts of the level (cycle precision; read by the pack kernel)
  long long ncell, nnext;           // cells of the level and of the next one (0 for the coarsest)
  int np, nrow, nnz, nw;            // parts, stored rows of U, entries of U, stencil width of the pack
  const int *urow, *uptr, *ucol;
  const T *uval;
  T *vb, *vt;                       // right-hand side and output of the level (global)
  const T *rs;                      // smoother factors (cycle precision; null on the coarsest)
  const double *rs64;               // FP64 smoother factors (the coarsest level's sweep)
  const double *ainv;               // coarsest level, direct solve: A^{-1} (row-major), else null
  int ndirect, packed;              // its order (0: one relaxation sweep); 1 if the pack below is set
  int colmajor, pad1;               // 1: ainv is stored by columns (the collapsed cycle operator)
  int *nb;                          // [nw][ncell] neighbour cell of entry s (the cell itself if absent)
  T *ca;                            // [nw][ncell] its coefficient (0 if absent)
  int *pi;                          // [2][ncell] interpolation: the two next-level cells
  T *pw;                            // [2][ncell] and their weights
  int *ri;                          // [3][nnext] restriction: the three cells of this level
  T *rw;                            // [2][nnext] and the weights of the second and third
  int *rowof;                       // [ncell] row of U holding the cell, -1 if none
};

// Dynamic LDS layout of the coarse-end kernel for nl levels (byte offsets, 16
// aligned): the TailLevel records, the vector offset table, the b and x
// vectors of every level, then a scratch and a sum vector of maxel elements
// and prodcap coupling products.
struct TailPlan {
  int nl, maxel, prodcap;
  int off_tab, off_vec, off_tv, off_acc, off_prod, bytes;
};

// per-part Galerkin product toward the next level (device array indexed by
// part).  Offsets are cube indices (dx+1) + 3(dy+1) + 9(dz+1).
struct RapDesc {
  double *out;         // coarse coefficients [nent][cncell]
  float *out32;        // FP32 copy of them (mixed-precision cycle) or null
  double *l1;          // one-thread-per-coarse-cell kernel: sum_s |a_s(f)| of every fine cell (part slice) or null
  float *fine32;       // that kernel: FP32 copy of the fine coefficients [nent_f][ncell] or null
  int nent;            // coarse entries
  int ng;              // 1: non-Galerkin coarse stencil of a star part (see rap_ng_value)
  int fmap[27];        // fine entry of each offset, -1: not in the fine stencil
  int cmap[27];        // coarse entry of each offset, -1: not in the coarse stencil
  int cofs[27];        // offset of each coarse entry
  // one-thread-per-coarse-cell kernel: the coarse part's own interpolation
  // weights (toward the level after) from each coarse row as it is formed:
  // its coarsening direction (-1: not formed here), faces, F-box extents,
  // the weight arrays (FP32 copies or null) and the error flag
  int wdir;
  int wfaces;
  int wfn[3];
  double *wm, *wp;
  float *wm32, *wp32;
  int *wflag;
};

// blocks per part of the finite-volume stencil kernel (its metric partials)
inline int fv_blocks(int maxcell) { return (maxcell + kBlock - 1) / kBlock > 0 ? (maxcell + kBlock - 1) / kBlock : 1; }

// finite-volume assembly arguments
struct FvArgs {
  const int *geom;     // per part: origin[3], dims[3], cell offset
  int nparts;
  int nent;
  int code[kMaxEnt];   // stencil offsets, entry 0 = center
};

// MODE_APPLY_DOT (FP64 only): y = A x and the per-right-hand-side partial sums
// of x.y: per block of 256 (cell, rhs) elements in the one-column kernel, per
// group of four such blocks in the four-column kernel (see dot_slots)
// MODE_JACOBI_DOT (finest level, FP64 b = r and output z): the sweep and the
// partial sums of r.z (first set) and, when aux = q is given, z.q (second set)
enum StencilMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2, MODE_APPLY_DOT = 3, MODE_JACOBI_DOT = 4 };

// Partial slots of MODE_APPLY_DOT per part: the one-column grid's blocks of
// 256 elements, rounded up to a multiple of 4, so that every group of four
// slots is one block of the four-column kernel; slot (part * dot_slots +
// block) holds 1 << lg sums (the four-column kernel fills the first quarter
// of the buffer with one sum per group).
inline int64_t dot_slots(int64_t maxcell, int lg) {
  const int64_t nb = (((maxcell << lg) + kBlock - 1) / kBlock);
  return 4 * ((nb + 3) / 4);
}

// Optional timing of one launch: when start is set the kernel is dispatched
// with hipExtLaunchKernelGGL, which records the two events with the kernel's
// own dispatch (its execution time, without the gaps around it).
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// kernels_cycle.hip
// Stencil sweeps of batched solves (lg >= 2) run four right-hand-side columns
// per thread unless cols4 is 0; never for FP64 27-point stencils, whose 108
// neighbour values would not fit the register file.
template <typename T>
inline bool stencil_cols4_ok(int lg, int maxent) {
  return lg >= 2 && !(sizeof(T) == 8 && maxent > 15);
}
template <typename T, typename TB, typename TO>
void launch_stencil(int mode, int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell,
                    int lg, const T *x, const TB *b, TO *y, hipStream_t st, LaunchEvents ev = {},
                    int cols4 = -1, double *dotp = nullptr, const double *aux = nullptr,
                    bool mir = false);
// The FP64 product of PCG with its p.q partials (MODE_APPLY_DOT, one
// right-hand side) on a finest level whose parts all have the full 27-point
// stencil and an even number of cells along x, two cells per thread
// (k_product2); same partial slots as the one-column kernel.  nb1: that
// kernel's blocks per part.
void launch_product2(const PartDesc<double> *desc, int nparts, int maxcell, bool mir, bool share,
                     const double *x, double *y, double *dotp, hipStream_t st, LaunchEvents ev = {});
// The finest level's residual (MODE_RESID) or post-smoothing sweep
// (MODE_JACOBI) for one right-hand side with b in FP64, 16 / sizeof(T) cells
// per thread (k_sweepN): every part has the full 27-point stencil and a
// multiple of that many cells along x.  Taken by the FP64 cycle only: in
// FP32 the four-cell form measured slower than one cell per thread (C3
// post-sweep 491 against 434 us; two waves per SIMD instead of four).
template <typename T, typename TO>
void launch_sweep2(int mode, const PartDesc<T> *desc, int nparts, int maxcell, const T *x, const double *b, TO *y,
                   hipStream_t st, LaunchEvents ev = {});
// First pass of the fused product dot: kDotGroupBlocks partial sums per
// right-hand side into partial[b][k] (row stride kMaxRhs) from ngroups groups
// of dotp (per = 4 one-column slots each, or per = 1 group sum); k_dot_final
// (launch_dot_final) finishes it.
constexpr int kDotGroupBlocks = 512;
void launch_dot_groups(const double *dotp, int64_t ngroups, int lg, int per, int nset, double *partial,
                       hipStream_t st);
void launch_dot_final(const double *partial, int nblk, int lg, double *scal, int slot, hipStream_t st);
// the first set into slot_a (with the S_RZN -> S_RZ shift when shift_rz) and,
// with nset = 2, the second into slot_b
void launch_dot_final2(const double *partial, int nblk, int lg, double *scal, int slot_a, int shift_rz,
                       int slot_b, int nset, hipStream_t st);
// the coarse end of one cycle (levels tl[0 .. pl.nl), LDS-resident); with
// mcol, pl.nl = levels from a level of n cells to the coarsest: one workgroup
// per unit right-hand side e_j writes column j of that coarse end's operator
// (FP64, by columns) to mcol instead
template <typename T>
void launch_tail(const TailLevel<T> *tl, const TailPlan &pl, int lg, hipStream_t st, double *mcol = nullptr,
                 int n = 1);
// one coarsest level of nel elements, any size (vectors in global memory): a
// sweep from zero or the direct solve, vb into vt
template <typename T>
void launch_coarsest(const TailLevel<T> *tl, int64_t nel, int lg, hipStream_t st);
// writes the packs of the nlev consecutive records tl[0 .. nlev) (maxcell: their largest level)
template <typename T>
void launch_tail_pack(TailLevel<T> *tl, int nlev, int64_t maxcell, hipStream_t st);
// LDS layout of the coarse end from level lt at width 2^lg; false when it
// exceeds kTailLds bytes
// ... for the levels lt .. lend (default: to the coarsest)
bool tail_plan(const Solver &s, int lt, int lg, TailPlan &pl, int lend = -1);
template <typename T, typename TB>
void launch_smooth_zero(int fine, const PartDesc<T> *desc, int nparts, int maxcell, int lg, const TB *b,
                        T *x, hipStream_t st);
template <typename T>
// wn, xn (one or two columns): also the next level's first sweep from zero,
// xn = wn b_c, with that level's smoother factors wn (level vector)
void launch_restrict(const PartDesc<T> *desc, int nparts, int maxcoarse, int lg, const T *r, T *bc,
                     hipStream_t st, LaunchEvents ev = {}, const T *wn = nullptr, T *xn = nullptr);
template <typename T>
void launch_interp_add(const PartDesc<T> *desc, int nparts, int maxcell, int lg, const T *xc, T *x,
                       hipStream_t st, LaunchEvents ev = {});
void launch_coarse_mixed(const PartDesc<double> *desc, int nparts, int maxcell, int lg, const float *b,
                         float *x, hipStream_t st);
// [nrhs][n] -> [n][nrhs] (to_cell_major = 1) or back, nrhs = 1 << lg <= kMaxRhs
void launch_transpose(const double *in, double *out, int64_t n, int lg, int to_cell_major, hipStream_t st);
void launch_cast_d2f(const double *in, float *out, int64_t n, hipStream_t st);
void launch_cast_f2d(const float *in, double *out, int64_t n, hipStream_t st);
void launch_fill(double *x, double v, int64_t n, hipStream_t st);
void launch_copy(const double *in, double *out, int64_t n, hipStream_t st);
void launch_dot(const double *a, const double *b, int64_t nel, int lg, double *partial, double *scal,
                int slot, int shift_rz, hipStream_t st);
// a.b into slot_ab (shift_rz as launch_dot) and b.c into slot_bc in one pass;
// partial holds 2 * kRedBlocks * kMaxRhs doubles
void launch_dot2(const double *a, const double *b, const double *c, int64_t nel, int lg, double *partial,
                 double *scal, int slot_ab, int shift_rz, int slot_bc, hipStream_t st);
// x32 / x64 (one column): also x0 = w r, the finest level's first sweep from
// zero of the next cycle, with the level's smoother factors w32 / w64
void launch_pcg_r(int64_t nel, int lg, double *scal, const int *active, double *r, const double *q,
                  double *partial, hipStream_t st, const float *w32 = nullptr, float *x32 = nullptr,
                  const double *w64 = nullptr, double *x64 = nullptr);
void launch_pcg_xp(int64_t nel, int lg, const double *scal, const int *active, int flexible,
                   const double *z, double *p, double *x, hipStream_t st);
void launch_pcg_x(int64_t nel, int lg, const double *scal, const double *p, double *x, hipStream_t st);
void launch_resid_norm(const double *b, const double *ax, int64_t nel, int lg, double *partial,
                       double *scal, int slot, hipStream_t st);

// kernels_setup.hip
// flag[0] = 1: nonpositive diagonal or non-finite coefficient; flag[1] = 1: some
// in-box pair a_s(c), a_{-s}(c+s) differs by more than a relative 1e-12
void launch_normalise(const BoxStencil &bs, int *flag, hipStream_t st);
void launch_wsum(const PartDesc<double> *desc, int nparts, int maxcell, double *partial, double *out,
                 hipStream_t st);
// c_d from per-block partial sums [part][nblk][3] (those of fv_assemble)
void launch_wsum_final(const double *partial, int nparts, int nblk, double *out, hipStream_t st);
void launch_interp_weights(const PartDesc<double> *desc, const PartDesc<float> *desc32, int nparts,
                           int maxf, int *flag, hipStream_t st);
// one thread per coarse cell when the level has at least cell_min coarse cells
// (over all parts), else one thread per (coarse cell, entry); the same values
// bit for bit either way
void launch_rap(const PartDesc<double> *desc, const RapDesc *rd, int nparts, int maxcoarse,
                int maxent_c, int64_t cell_min, bool any_ng, hipStream_t st);
// whether launch_rap takes the one-thread-per-coarse-cell kernel (which also
// writes the fine level's L1 row sums and FP32 copy when asked to)
bool rap_per_cell(int nparts, int maxcoarse, int64_t cell_min);
// weighted L1-Jacobi: cast32 (finest level, mixed precision) also receives
// the FP32 copy of the coefficients the pass reads; stencil_sums_done: rs
// already holds the stencil part of the row sums (written by the Galerkin
// kernel)
void launch_smoother_scale(bool l1, const PartDesc<double> *desc, int nparts, int maxcell, int64_t n,
                           int nrow, const int *urow, const int *uptr, const double *uval,
                           double factor, double *rs, float *rs32, int *flag, hipStream_t st,
                           const PartDesc<float> *cast32 = nullptr, bool stencil_sums_done = false);
template <typename T, typename TB>
void launch_smooth_resid(int fine, int maxent, const PartDesc<T> *desc, int nparts, int maxcell, int lg,
                         const TB *b, T *x, T *r, hipStream_t st, LaunchEvents ev = {});
void launch_direct_setup(const PartDesc<double> *desc, int np, int n, int nrow, const int *urow,
                         const int *uptr, const int *ucol, const double *uval, double *ainv, int *flag,
                         hipStream_t st);
void launch_uc_numeric(int64_t nnz, const int *start, const int *k, const int *a, const int *b,
                       const double *uprev, const double *w, double *uval, float *uval32,
                       hipStream_t st);

// kernels_symbolic.hip
void coarse_coupling_device(SymScratch &w, const SymPart *sp, int np, int64_t nnz, const int *erow,
                            const int *ucol, int64_t nc, CouplingStore &out, int64_t &out_nnz,
                            int &out_nrow, hipStream_t st,
                            const std::function<void()> &before_sync = {});
void launch_entry_rows(int nrow, const int *urow, const int *uptr, int *erow, hipStream_t st);
// block tables of several (level, lg) pairs in one launch: the level's part
// records start at sp + spat, its block offsets at boff + boffat; nbx: blocks
// of kBlock chunks that cover the largest part
struct UblkJob {
  const int *urow, *uptr;
  int *out;
  int nrow, lg, spat, boffat;
};
constexpr int kUblkJobs = 48;
struct UblkJobs {
  int n;
  UblkJob j[kUblkJobs];
};
void launch_ublk(const SymPart *sp, int np, const long long *boff, const UblkJobs &jobs, int64_t nbx,
                 hipStream_t st);

// kernels_dense.hip: exact solve of the hybrid tail's switch level
int64_t dense_pad(int64_t n);            // order of the padded dense matrix
int64_t dense_apply_chunks(int64_t n);   // column chunks of the applied product
// the level's operator (FP64 descriptors and couplings) assembled densely into
// a (npad x npad) and inverted in place; pt: 64 * npad, dinv: 64 * 64 doubles;
// flag = 2 when a pivot block is not positive definite
void launch_dense_inverse(const PartDesc<double> *desc, int nparts, int maxcell, int64_t n, int nrow,
                          const int *urow, const int *uptr, const int *ucol, const double *uval, double *a,
                          double *pt, double *dinv, int *flag, hipStream_t st);
// vt = M vb for 1 << lg right-hand sides ([cell][rhs]); part holds
// dense_apply_chunks(n) * n << lg doubles
template <typename T>
void launch_dense_apply(const double *m, int64_t n, int lg, const T *vb, T *vt, double *part, hipStream_t st);

// kernels_fv.hip
void launch_fv_stencil(const FvArgs &fa, int maxcell, const double *kappa, const double *aniso,
                       double *const *coef, double *mpart, double *csum, const long long *csoff,
                       hipStream_t st);
void launch_fv_coupling(int nrow, const int *urow, const int *uptr, const int *ucol,
                        const int *ucode, const double *kappa, const double *aniso, double *uval,
                        hipStream_t st);
void launch_fv_grad(const FvArgs &fa, int maxcell, const double *kappa, const double *aniso,
                    const double *lam, const double *x, int nrhs, double *grad, int nrow, const int *urow,
                    const int *uptr, const int *ucol, const int *ucode, hipStream_t st);

}  // namespace ssamg
