/*
 * ssamg.h - C ABI of a semi-structured algebraic multigrid (SSAMG) solver for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is that of Magri, Falgout and Yang, "A New Semi-Structured
 * Algebraic Multigrid Method" (arXiv 2205.14273):
 *   - the problem is A x = b with A = S + U on a semi-structured grid
 *     (Section 2): n_p parts, each a box of cells with its own index space,
 *     a per-part stencil S with per-cell coefficients, and a sparse matrix U
 *     holding the couplings between parts;
 *   - setup (Section 3): grid-spacing metric W and Algorithm 1 (semicoarsening
 *     direction per level and part), two-point operator-collapse interpolation
 *     (Section 3.2, eq:prolEx), Galerkin coarse operators
 *     A_c = P^T S P + P^T U P (Section 3.3, eq:galerkin);
 *   - solve: PCG preconditioned by one V(1,1) cycle of weighted Jacobi with the
 *     per-part weights of eq:relax1 / eq:alpha-beta (Sections 3.4 and 4).
 *
 * Conventions shared by every call:
 *   - every function returns ssamg_status; nothing throws across the ABI; the
 *     text of the last error of the calling thread is ssamg_last_error();
 *   - cells are numbered part-major and, inside a part, lexicographically with
 *     x fastest: id = offset[p] + i + nx*(j + ny*k); every box has lower corner
 *     (0,0,0) in its part's own index space (other lower corners are
 *     SSAMG_ERR_UNSUPPORTED: only the parity of the index matters to the
 *     method, and a shifted box is the same problem);
 *   - pointers tagged "device" are HIP device pointers on the current device;
 *     "host" pointers are ordinary memory; the library copies what it keeps
 *     and never frees caller memory;
 *   - all device work is ordered on the HIP stream given at creation (NULL =
 *     the null stream); calls that return results to the host synchronize it;
 *   - total cells of a problem must stay below 2^31.
 */
#ifndef SSAMG_H
#define SSAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSAMG_OK = 0,
  SSAMG_NOT_CONVERGED = 1,     /* max_iter reached; x and info are filled */
  SSAMG_ERR_ARG = -1,          /* bad argument (index, size, NULL, layout) */
  SSAMG_ERR_STATE = -2,        /* call out of order (e.g. solve before setup) */
  SSAMG_ERR_UNSUPPORTED = -3,  /* valid request outside this implementation */
  SSAMG_ERR_NUMERIC = -4,      /* nonpositive diagonal or collapse denominator,
                                  NaN/Inf, PCG breakdown (p^T A p <= 0) */
  SSAMG_ERR_DEVICE = -5,       /* a HIP runtime call failed */
  SSAMG_ERR_ALLOC = -6         /* device or host allocation failed */
} ssamg_status;

enum { SSAMG_FACE_PHYSICAL = 0, SSAMG_FACE_PART = 1 };
enum { SSAMG_MEM_HOST = 0, SSAMG_MEM_DEVICE = 1 };
enum { SSAMG_RELAX_JACOBI = 0, SSAMG_RELAX_L1_JACOBI = 1 };
enum { SSAMG_COARSE_SWEEP = 0, SSAMG_COARSE_DIRECT = 1 };
enum { SSAMG_FP64 = 0, SSAMG_FP32 = 1 };
enum { SSAMG_PB_ONE = 0, SSAMG_PB_LUMP = 1 };
enum { SSAMG_COARSE_OP_GALERKIN = 0, SSAMG_COARSE_OP_NONGALERKIN = 1 };
enum { SSAMG_LAYOUT_CELL_MAJOR = 0, SSAMG_LAYOUT_RHS_MAJOR = 1 };

typedef struct ssamg_problem_s *ssamg_problem;
typedef struct ssamg_solver_s *ssamg_solver;

/* ---------------------------------------------------------------- problem */

/* Create an empty problem of n_p = nparts parts in ndim (2 or 3) dimensions.
 * In 2D every box has nz = 1 and stencil offsets have dz = 0 (Section 2). */
ssamg_status ssamg_problem_create(int ndim, int nparts, ssamg_problem *out);
ssamg_status ssamg_problem_destroy(ssamg_problem prob);

/* Box of part `part`: cells lo[d] .. hi[d] inclusive, lo must be {0,0,0}.
 * This is the part's index-space box (its bounding box, on which Algorithm 1
 * coarsens); the part's cells are all of it unless ssamg_problem_add_box
 * lists the boxes the part is made of (Section 2). */
ssamg_status ssamg_problem_set_box(ssamg_problem prob, int part, const int lo[3],
                                   const int hi[3]);

/* A part made of several boxes (Section 2): adds the box lo .. hi (inclusive,
 * inside the part's box) to the part's list.  When a part has a list, each of
 * its cells in none of the listed boxes is a ghost unknown (the treatment of
 * coarse cells under a refined patch in adaptive refinement, Section 4): its
 * row is the identity (set_coeffs replaces its given coefficients), every
 * stencil entry pointing at it is dropped, and no coupling may touch it.
 * Vectors still span the part's whole box; with b = 0 on ghost cells, x is
 * zero there up to the solver's tolerance.  Boxes may overlap.  Invalidates every part's coefficients (call
 * set_coeffs again).  Needs set_box first. */
ssamg_status ssamg_problem_add_box(ssamg_problem prob, int part, const int lo[3], const int hi[3]);

/* Glue face `face` (0..5 = -x,+x,-y,+y,-z,+z) of part `part` to part
 * `nbr_part` (another part) for non-Cartesian connectivity (Section 2; the
 * rotated index spaces of Section 4's three-part intersection): a point x just
 * across the face, in part's index space, is the point y of the neighbour's
 * index space with y[map[d]] = nbr_at[map[d]] + dir[d] * (x[d] - at[d]), where
 * `at` is a point just across the face (at[axis] = -1 or n[axis], the other
 * components inside the box), `nbr_at` its image (inside the neighbour's box),
 * map a permutation of {0,1,2} and dir[d] = +-1.  set_coeffs then moves every
 * stencil entry a_s(c) whose neighbour c + s leaves the box through a glued
 * face into the couplings, U(c, y) = a_s(c) (entries leaving through two faces
 * at an edge or corner take the first glued face, in face order, whose image
 * is an active cell of its neighbour; all others are dropped as Dirichlet).
 * The face becomes SSAMG_FACE_PART.  The caller glues both sides, with
 * symmetric coefficients, to keep A symmetric.  Invalidates every part's
 * coefficients.  SSAMG_ERR_ARG for a bad map, a point not across the face or
 * an image outside the neighbour's box. */
ssamg_status ssamg_problem_set_neighbor(ssamg_problem prob, int part, int face, int nbr_part,
                                        const int at[3], const int nbr_at[3], const int map[3],
                                        const int dir[3]);

/* Placement of part `part` in a shared global index space.  Used only by
 * ssamg_problem_fv_assemble (neighbour lookup across parts) and to derive
 * face kinds; not needed for problems given through set_coeffs/set_coupling. */
ssamg_status ssamg_problem_set_origin(ssamg_problem prob, int part, const int origin[3]);

/* Kind of face `face` (0..5 = -x,+x,-y,+y,-z,+z) of part `part`:
 * SSAMG_FACE_PART marks a part boundary that is not a physical boundary, where
 * the interpolation rule of Section 3.2 (crossing weight 0, opposite weight 1)
 * applies.  Default SSAMG_FACE_PHYSICAL. */
ssamg_status ssamg_problem_set_face(ssamg_problem prob, int part, int face, int kind);

/* Stencil of part `part` (Section 2): nent offsets off[nent][3] in
 * {-1,0,1}^3 (the 27-point neighbourhood, Section 3.1), distinct, including
 * (0,0,0).  Offsets outside the neighbourhood are SSAMG_ERR_UNSUPPORTED. */
ssamg_status ssamg_problem_set_stencil(ssamg_problem prob, int part, int nent,
                                       const int *off);

/* Coefficients of part `part` for its stencil: vals[nent][nz][ny][nx] (x
 * fastest), or vals[nent] when constant = 1 (one value per stencil entry for
 * the whole part, Section 2).  `where` = SSAMG_MEM_HOST or SSAMG_MEM_DEVICE.
 * Copied.  Entries whose neighbour lies outside the box are discarded
 * (Dirichlet elimination) or, across a glued face, moved to the couplings;
 * ghost cells of a part of several boxes get identity rows.  Requires
 * set_box and set_stencil first, and the boxes and glued faces of every part
 * when there are any. */
ssamg_status ssamg_problem_set_coeffs(ssamg_problem prob, int part, const double *vals,
                                      int where, int constant);

/* Inter-part couplings U (Section 2): nnz entries (row[k], col[k], val[k]) with
 * global cell ids, in COO form; `where` = SSAMG_MEM_HOST or SSAMG_MEM_DEVICE
 * for all three arrays; copied; duplicates are summed (also with the entries
 * moved across glued faces), explicit zeros kept as structure.  An entry
 * inside one part or on a ghost cell is SSAMG_ERR_ARG (the first is an
 * assumption of the theorem of Section 3.3); a non-finite value
 * SSAMG_ERR_NUMERIC.  A second call replaces the given couplings; nnz = 0
 * means none. */
ssamg_status ssamg_problem_set_coupling(ssamg_problem prob, int64_t nnz, const int64_t *row,
                                        const int64_t *col, const double *val, int where);

/* Finite-volume diffusion operator from per-cell conductivity (the synthetic
 * workloads): kappa (device, N doubles, copied), aniso (host, [nparts][3]
 * directional factors), stencil 7 or 27 (5 or 9 in 2D).  For neighbour offset
 * s the conductance is t = g_s * H(a_{p(i),s} kappa_i, a_{p(j),s} kappa_j),
 * H(x,y) = 2xy/(x+y), g_s = 1, 1/2, 1/4 for faces, edges, corners, a_{p,s} the
 * mean of the part's factors over the nonzero components of s; neighbours
 * outside every part are zero-Dirichlet ghosts with kappa_j = kappa_i.
 * A_ii = sum of t, A_ij = -t; same-part entries go to S, the rest to U.  Needs
 * boxes and origins of every part; sets the stencils, the face kinds and U.
 * Problems with add_box or set_neighbor are SSAMG_ERR_UNSUPPORTED here. */
ssamg_status ssamg_problem_fv_assemble(ssamg_problem prob, const double *kappa,
                                       const double *aniso, int stencil, void *hip_stream);

/* Gradient of L(x(kappa)) for the operator of the last fv_assemble (adjoint
 * method): grad[c] = -sum_k lambda_k^T (dA/dkappa_c) x_k over the nrhs columns
 * (1..32), where lambda_k solves A lambda_k = dL/dx_k.  lambda, x: device,
 * [N][nrhs] doubles (right-hand side fastest); grad: device, N doubles,
 * overwritten. */
ssamg_status ssamg_problem_fv_grad(ssamg_problem prob, int nrhs, const double *lambda, const double *x,
                                   double *grad, void *hip_stream);

/* Number of cells N of the problem, and its number of parts. */
ssamg_status ssamg_problem_num_cells(ssamg_problem prob, int64_t *n);
ssamg_status ssamg_problem_num_parts(ssamg_problem prob, int *nparts);

/* Stencil entries (0 before set_stencil) and cells of part `part`, so that a
 * caller can size the coefficient array of set_coeffs. */
ssamg_status ssamg_problem_part_size(ssamg_problem prob, int part, int *nent, int64_t *ncell);

/* ---------------------------------------------------------------- solver */

typedef struct {
  int max_levels;            /* l_max of Section 3.1 (default 64) */
  int64_t min_coarse_size;   /* s_max of Section 3.1: stop at the first level with
                                fewer cells (default 0: coarsen to one cell/part) */
  int relax;                 /* SSAMG_RELAX_JACOBI (default): x += omega D^{-1} (b - Ax);
                                SSAMG_RELAX_L1_JACOBI: x += factor M^{-1} (b - Ax) with
                                M_ii = sum_j |a_ij| over S and U (Section 3.4) */
  double omega;              /* JACOBI: > 0 fixed weight, <= 0 per-part omega_p of
                                eq:relax1 (default); L1_JACOBI: > 0 the factor, <= 0 3/2
                                (the paper's SSAMG-base setting) */
  int coarse;                /* SSAMG_COARSE_SWEEP (default, Section 3.5): one sweep
                                from zero; SSAMG_COARSE_DIRECT: exact solve with the
                                coarsest operator's inverse, formed at setup_numeric
                                (at most 64 unknowns, else setup_symbolic returns
                                SSAMG_ERR_UNSUPPORTED; SSAMG_ERR_NUMERIC when the
                                operator is not positive definite) */
  int cycle_precision;       /* SSAMG_FP64 (default) or SSAMG_FP32: V-cycle in FP32
                                inside FP64 PCG, coarsest level in FP64 */
  double tol;                /* ||r||_2 < tol ||b||_2 (default 1e-8) */
  int max_iter;              /* default 100 */
  int max_nrhs;              /* right-hand sides per solve, power of two <= 32 (default 1) */
  int use_graph;             /* capture the V-cycle in a HIP graph (default 1) */
  int skip;                  /* 1: the "skip" option of Section 3.4 - a part does not
                                relax at level l >= n_d where it coarsens along the
                                same direction as at level l - n_d (default 0) */
  int autotune;              /* 1: the first solve of each batch width >= 4 times the
                                launch options of its larger levels and keeps the
                                fastest (ssamg_autotune); 0: defaults (default 0) */
  int symmetric;             /* 1 (default): A is symmetric, as conjugate gradients
                                requires, so within each part a_s(c) = a_{-s}(c+s);
                                the FP64 product of PCG (and ssamg_apply_A) on
                                stencils of more than 7 points reads the center and
                                the entries of positive offset (last nonzero
                                component of (dx, dy, dz) positive) and takes every
                                other entry from the neighbour's mirrored one,
                                halving its coefficient traffic (parts whose
                                pattern lacks a mirror read every entry, and so
                                does every part of a problem whose given
                                coefficients are not symmetric to a relative
                                1e-12).  The V-cycle always reads every entry.
                                0: the product reads every entry too */
  int pb_interp;             /* interpolation at a part face crossed along d* (Section 3.2):
                                the weight across the face is dropped and
                                SSAMG_PB_ONE (default): the opposite weight is set to 1;
                                SSAMG_PB_LUMP: the dropped weight, the collapse of the
                                row's couplings U (-sum_j u_fj over the collapse
                                denominator), is added to the opposite weight.  Both
                                interpolate constants exactly on rows of zero sum; they
                                differ on rows next to a Dirichlet face */
  int hybrid_level;          /* 0 (default): off.  k >= 1: the hybrid coarse tail of
                                Section 3.5 - the hierarchy ends at level k (or earlier,
                                if it is shorter) and that level is solved exactly, in
                                FP64, with its dense inverse formed at setup_numeric
                                (blocked Gauss-Jordan on the device).  The level may
                                have at most 16384 unknowns (SSAMG_ERR_UNSUPPORTED from
                                setup_symbolic otherwise); SSAMG_ERR_NUMERIC when its
                                operator is not positive definite.  Overrides coarse */
  int coarse_op;             /* coarse stencils (Section 3.3; Section 5 plans the
                                second for isotropic problems):
                                SSAMG_COARSE_OP_GALERKIN (default): P^T S P;
                                SSAMG_COARSE_OP_NONGALERKIN: on parts whose stencil is a
                                star (every offset has at most one nonzero component,
                                e.g. 7-point) the coarse stencil keeps that pattern:
                                each Galerkin entry with components both across and
                                along d* is replaced by the four star entries along
                                the sides of the rectangle it spans, at half its
                                value, the diagonals keeping every row sum.  For the
                                constant-coefficient Laplacian this is the
                                finite-volume stencil of the coarsened cells.  Other
                                parts and the couplings P^T U P stay Galerkin */
} ssamg_params;

typedef struct {
  int nrhs;
  int iters[32];             /* per right-hand side */
  double relres[32];         /* ||r_k||/||b|| of the recursive residual at exit */
  double true_relres[32];    /* ||b - A x||/||b|| recomputed at exit */
  int converged[32];
  double t_setup;            /* seconds, host wall clock of the last setup_symbolic +
                                setup_numeric of this solver */
  double t_solve;            /* seconds, host wall clock around the solve */
} ssamg_info;

typedef struct {
  int dims[3];               /* box extents at this level */
  int64_t offset;            /* first cell of the part in the level vector */
  int dstar;                 /* semicoarsening direction 0,1,2; -1: not coarsened */
  double omega;              /* relaxation weight of the part at this level */
  int nent;                  /* stencil entries */
  int pattern[27][3];        /* stencil offsets (level 0: as given; coarser: sorted
                                by (dz, dy, dx)) */
  int fdims[3];              /* F-box (cells odd along dstar) extents */
  int skip;                  /* 1: the part does not relax at this level (skip option) */
} ssamg_level_desc;

ssamg_status ssamg_params_default(ssamg_params *params);

/* Create a solver for `prob` (which must outlive it) on `hip_stream`. */
ssamg_status ssamg_solver_create(ssamg_problem prob, const ssamg_params *params,
                                 void *hip_stream, ssamg_solver *out);
ssamg_status ssamg_solver_destroy(ssamg_solver s);

/* Symbolic setup: the metric reduction (device, one small copy back), W,
 * Algorithm 1, omega_p, symbolic coarse stencils and Galerkin tables, and the
 * structure of every coarse coupling matrix U_c (host, integer work). */
ssamg_status ssamg_setup_symbolic(ssamg_solver s);

/* Device bytes the numeric setup needs (hierarchy + work vectors). */
ssamg_status ssamg_workspace_bytes(ssamg_solver s, size_t *bytes);

/* Numeric setup (device kernels only): interpolation weights, structured and
 * unstructured Galerkin products per level, FP32 copies when cycle_precision =
 * SSAMG_FP32.  ws: caller-owned device buffer of at least workspace_bytes
 * (kept until the solver is destroyed), or NULL to let the library allocate. */
ssamg_status ssamg_setup_numeric(ssamg_solver s, void *ws, size_t bytes);

/* Replace the stencil coefficients of one part of the solver's problem (same
 * pattern; vals and where as in ssamg_problem_set_coeffs with constant = 0).
 * The hierarchy depends on the values (Section 3.1 metric, Algorithm 1), so
 * the solver returns to the created state: setup_symbolic and setup_numeric
 * must run again before the next solve (SSAMG_ERR_STATE otherwise). */
ssamg_status ssamg_update_coeffs(ssamg_solver s, int part, const double *vals, int where);

/* Solve A X = B for nrhs right-hand sides (1 <= nrhs <= max_nrhs, power of two)
 * by PCG with one V(1,1) cycle as preconditioner (Section 4 protocol).
 * b, x: device, N * nrhs doubles each, laid out as `layout` says:
 *   SSAMG_LAYOUT_CELL_MAJOR  [N][nrhs], right-hand side index fastest (the
 *                            library's own layout);
 *   SSAMG_LAYOUT_RHS_MAJOR   [nrhs][N], one contiguous vector per right-hand
 *                            side (transposed into the library's layout and
 *                            back, through two device buffers of N * nrhs
 *                            doubles that the solver allocates on first use).
 * For nrhs = 1 both layouts are the same plain vector.  x0 = 0.  Returns
 * SSAMG_NOT_CONVERGED when some right-hand side did not meet tol within
 * max_iter.  info may be NULL. */
ssamg_status ssamg_solve(ssamg_solver s, int nrhs, const double *b, double *x, int layout,
                         ssamg_info *info);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ssamg_solve with the
 * same arguments and results (bit for bit), except that the PCG work vectors
 * r, z, p, q, the reduction partials and scalars, and for
 * SSAMG_LAYOUT_RHS_MAJOR with nrhs > 1 the layout staging, come from one fixed
 * device array of SSAMG_NOALLOC_SCRATCH_BYTES per GPU (held until the process
 * ends) instead of the solver's workspace or buffers allocated on first use.
 * It calls no allocating routine: a V-cycle graph not yet instantiated for
 * this width is not built (the coarse levels are launched directly), and
 * autotune = 1 needs the width tuned beforehand (SSAMG_ERR_STATE otherwise).
 * Needs (4 N nrhs + 2 N nrhs if staged) doubles plus about 1 MiB of partials:
 * larger solves return SSAMG_ERR_ARG with the size in the message.  The
 * solver's device must be current.  Every call on one GPU shares its array:
 * calls that overlap on one GPU (two streams or threads) race and must be
 * serialised by the caller. */
#define SSAMG_NOALLOC_SCRATCH_BYTES (64u << 20)
ssamg_status ssamg_solve_noalloc(ssamg_solver s, int nrhs, const double *b, double *x, int layout,
                                 ssamg_info *info);

/* Launch options of the batched V-cycle (batch widths of 4 or more right-hand
 * sides), per level and width.  They choose how the kernels cover a level, not
 * what they compute: every choice gives bit-identical results.  The record is
 * int[5]:
 *   [0] strips    block order of the four-columns-per-thread stencil sweeps: each
 *                 z-plane of a part is cut into this many strips and a GPU die
 *                 sweeps one strip through its planes before the next, so the
 *                 planes above and below stay in its cache (1: plain order)
 *   [1] cols4     stencil sweeps with four columns per thread (1), one (0), or
 *                 the default (-1: four for widths >= 4 except FP64 27-point)
 *   [2] split     first sweep from zero as its own kernel before the residual
 *                 (1), fused with it (0), or the default rule (-1)
 *   [3] strips_mv, [4] cols4_mv   the same for the FP64 product of PCG on level 0
 *                 when cycle_precision = SSAMG_FP32 (it then has its own part
 *                 descriptors; in an FP64 cycle the product follows [0] and [1])
 * Records are kept per level shape (cycle precision, boxes, stencil sizes,
 * coarsening directions) and width, so they survive a new setup of the same
 * shapes. */

/* Time the candidate options of every level of width nrhs that has at least
 * 2^16 (cell, right-hand side) elements and runs grid kernels, and keep the
 * fastest (a candidate must beat the current choice by 2 %).  Needs the numeric
 * setup; overwrites the work vectors (not x or b of any solve).  cache_path:
 * NULL, or a JSON file of records (read first: levels found there are not
 * timed; written back with every record the solver holds, records of other
 * shapes in the file kept).  Widths below 4 have nothing to tune (SSAMG_OK).
 * SSAMG_ERR_ARG: nrhs not a power of two <= max_nrhs; SSAMG_ERR_STATE: no
 * numeric setup; SSAMG_ERR_ARG with a message when the file cannot be read or
 * written. */
ssamg_status ssamg_autotune(ssamg_solver s, int nrhs, const char *cache_path);

/* rec[0..4] = the options level `level` uses for width nrhs (stored or
 * defaults), rec[5] = 1 when a record is stored.  Needs the symbolic setup. */
ssamg_status ssamg_tune_get(ssamg_solver s, int level, int nrhs, int rec[6]);

/* Store a record (values as above; SSAMG_ERR_ARG for values out of range or
 * four columns per thread where not available). */
ssamg_status ssamg_tune_set(ssamg_solver s, int level, int nrhs, const int rec[5]);

/* y = A_l x at level `level` in FP64 (device vectors of that level's size). */
ssamg_status ssamg_apply_A(ssamg_solver s, int level, const double *x, double *y);

/* z = B r: one V(1,1) cycle in the configured precision (device, N doubles). */
ssamg_status ssamg_apply_precond(ssamg_solver s, const double *r, double *z);

ssamg_status ssamg_num_levels(ssamg_solver s, int *nlevels);
/* Cells N_l of level `level` (all parts). */
ssamg_status ssamg_level_cells(ssamg_solver s, int level, int64_t *ncell);
ssamg_status ssamg_level_info(ssamg_solver s, int level, int part, ssamg_level_desc *info);

/* c[p][d] of Section 3.1 as reduced on the device (host out, nparts*3). */
ssamg_status ssamg_direction_sums(ssamg_solver s, double *c_out);

/* Copies to host memory, for inspection and tests (after numeric setup). */
ssamg_status ssamg_copy_stencil(ssamg_solver s, int level, int part, double *vals /*[nent][ncell]*/);
ssamg_status ssamg_copy_interp(ssamg_solver s, int level, int part, double *wm, double *wp /*F-box*/);
ssamg_status ssamg_coupling_nnz(ssamg_solver s, int level, int64_t *nnz);
/* CSR over all cells of the level: rowptr[N_l+1], col[nnz], val[nnz] (columns
 * ascending in each row; structure is symbolic, numeric zeros kept). */
ssamg_status ssamg_copy_coupling(ssamg_solver s, int level, int64_t *rowptr, int64_t *col,
                                 double *val);

/* Measurement hooks: bracket every launch of one finest-level kernel kind with
 * HIP events on the solver's stream (inside solves and preconditioner
 * applications) and accumulate its algorithmic bytes (each array element
 * counted once: coefficients, inputs, outputs).  kind = SSAMG_PROBE_NONE turns
 * it off.  probe_read synchronizes, returns the launches, summed event time
 * (ms) and summed algorithmic bytes since the last set/read, and resets them.
 * At most 2048 launches are recorded between reads. */
enum {
  SSAMG_PROBE_NONE = -1,
  SSAMG_PROBE_MATVEC = 0,     /* PCG product q = A p (FP64) */
  SSAMG_PROBE_SMOOTH0 = 1,    /* reserved: the first sweep is fused into RESID0 */
  SSAMG_PROBE_RESID0 = 2,     /* first sweep from zero fused with the residual
                                 b - A x, finest level */
  SSAMG_PROBE_RESTRICT0 = 3,  /* restriction P^T r from the finest level */
  SSAMG_PROBE_INTERP0 = 4,    /* x += P x_c on the finest level */
  SSAMG_PROBE_JACOBI0 = 5     /* post-smoothing sweep, finest level */
};
ssamg_status ssamg_probe_set(ssamg_solver s, int kind);
ssamg_status ssamg_probe_read(ssamg_solver s, int64_t *launches, double *total_ms, double *alg_bytes);

const char *ssamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSAMG_H */
