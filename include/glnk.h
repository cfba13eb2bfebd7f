/*
 * glnk -- Jacobian solves for the discretised extreme type-II Ginzburg-Landau
 * problem on one AMD MI355X (gfx950).
 *
 * Method: N. Schloemer, W. Vanroose, "An optimal linear solver for the
 * Jacobian system of the extreme type-II Ginzburg-Landau problem".
 *   - discretisation (Sec. 3): Voronoi volumes |V_i| (D = diag|V_i|), edge
 *     coefficients alpha_jk, link variables U_jk, Hermitian K-hat with
 *     K = D^-1 K-hat (Remark on K = D^-1 K-hat);
 *   - GL_i(psi) = (K psi)_i - psi_i (1 - |psi_i|^2)          (eq. discr ginla)
 *   - (J(psi) phi)_i = (K phi)_i + (2|psi_i|^2 - 1) phi_i + psi_i^2 conj(phi_i)
 *                                               (discrete Jacobian, Sec. 3)
 *   - Newton: J(psi) dpsi = -GL(psi)                      (eq. Newton system)
 *   - MINRES in <u,v>_R = Re sum |V_i| conj(u_i) v_i       (Sec. 4, eq. disc inner2)
 *   - preconditioner R_k = AMG_k(K-hat + 2 D |psi|^2, D .) (eq. prec2),
 *     smoothed aggregation, 1 pre + 1 post symmetric Gauss-Seidel (Sec. 4.1).
 *
 * Conventions shared by every call:
 *   - Vectors are DEVICE pointers to n complex numbers stored as interleaved
 *     (re, im) doubles (the layout of torch.complex128 / std::complex<double>),
 *     node order x fastest, then y, then z.  The caller owns them; they must be
 *     8-byte aligned and must not alias unless a call says so.
 *   - Handles (gl_mesh, gl_precond) are owned by the library and freed by the
 *     matching *_destroy call.  Only *_create / *_setup calls allocate device
 *     memory; apply and solve calls allocate nothing.
 *   - stream is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *     on it; calls that return host scalars (norms, solve info) synchronise it.
 *   - Every call returns a gl_status; arguments are validated before any work
 *     is enqueued; gl_last_error() returns a description of the last failure
 *     of the calling thread.
 */
#ifndef GLNK_H
#define GLNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GL_OK = 0,
    GL_ERR_INVALID_ARGUMENT = 1,
    GL_ERR_HIP = 2,
    GL_ERR_OUT_OF_MEMORY = 3,
    GL_ERR_NOT_CONVERGED = 4,  /* iteration limit reached; outputs still written */
    GL_ERR_BREAKDOWN = 5,      /* MINRES: <v, M^-1 v> < 0 or NaN */
    GL_ERR_NONFINITE = 6,      /* NaN / Inf in an input or a residual */
    GL_ERR_SINGULAR = 7,       /* preconditioner matrix not positive definite */
    GL_ERR_UNSUPPORTED = 8
} gl_status;

/* Storage and arithmetic of the V-cycle (the Krylov iteration, the GL residual
 * and the Newton update are FP64 in every case):
 *   GL_FP64   every level in FP64;
 *   GL_FP32   every level and the coarsest solve in FP32;
 *   GL_MIXED  level 0 (the fine-grid sweeps and transfers, nearly all of the
 *             V-cycle's memory traffic) in FP32, levels >= 1 and the
 *             coarsest solve in FP64. */
typedef enum { GL_FP64 = 0, GL_FP32 = 1, GL_MIXED = 2 } gl_precision;

typedef struct gl_mesh gl_mesh;
typedef struct gl_precond gl_precond;
typedef struct gl_batch gl_batch;
typedef struct gl_unet gl_unet;
typedef void *gl_stream;

/* --------------------------------------------------------------- mesh --
 * Tensor grid of n_axis[0] x n_axis[1] (x n_axis[2]) nodes on the box
 * [-side/2, side/2]^dim, i.e. a Voronoi tessellation whose Delaunay dual is a
 * structured simplicial mesh (Sec. 3).  |V_i| is the Voronoi cell clipped to
 * the box; alpha_jk follows the Corollary on simplex edge coefficients
 * (2D: 1/2 cot of the opposite angle summed over both triangles; 3D: dual
 * facet area over edge length).  The vector potential is linear:
 *   potential == 0:  A(r) = mu/2 (b_dir x r)        (uniform field mu b_dir)
 *   potential == 1:  A(r) = a_matrix r               (3x3 row-major)
 * and U_jk = exp(-i (x_j - x_k) . A((x_j + x_k)/2)), the link variable of
 * Sec. 3 (exact for linear A), or
 *   potential == 2:  A(r) = mu m x (r - x0) / |r - x0|^3
 *                    (the dipole potential A_d of Sec. 4.1, moment
 *                    dipole_m at dipole_x0; the paper's experiments use
 *                    m = e_z and x0 = (0,0,6) in 3D, (0,0,1) in 2D)
 * with U_jk = exp(-i int e . A) along the straight edge in closed form; its
 * links are stored per edge (dim complex numbers per node, FP64 and FP32).
 * In 2D, r = (x, y, 0). */
typedef struct {
    int dim;            /* 2 or 3 */
    int64_t n_axis[3];  /* nodes per axis, >= 2 each (n_axis[2] ignored in 2D) */
    double side[3];     /* side lengths, > 0 */
    int potential;      /* 0, 1 or 2, see above */
    double mu;          /* field strength (potential 0 and 2) */
    double b_dir[3];    /* field direction (potential == 0), need not be unit */
    double a_matrix[9]; /* potential == 1 */
    double dipole_m[3]; /* potential == 2: dipole moment (nonzero) */
    double dipole_x0[3];/* potential == 2: dipole position, off every grid edge's line
                           segment */
} gl_grid_desc;

/* Build the grid and its link variables on the device.  Errors:
 * INVALID_ARGUMENT (dim, sizes, sides, more than 2^31 - 2 nodes),
 * OUT_OF_MEMORY, HIP. */
gl_status gl_mesh_create_grid(const gl_grid_desc *desc, gl_stream stream, gl_mesh **out);

/* Simplicial mesh given by its nodes and cells: triangles in the plane or
 * tetrahedra in space (Sec. 3: a Delaunay triangulation dual to the Voronoi
 * tessellation of the nodes; the paper's test domains of Sec. 4.1 beyond the
 * square and the cube, e.g. the triangle, the disc and the tetrahedron).  On
 * the device: alpha_jk = sum over the cells at edge jk of the cell's
 * coefficient of that edge, 1/2 cot of the opposite angle of a triangle (the
 * Remark on the Corollary's simplex coefficients) or |e'| cot(theta') / 6 for
 * a tetrahedron (e' the opposite edge, theta' the dihedral angle there: the
 * solution of the Corollary's system for that cell); |V_j| = sum over the
 * cells T at j of 1/(2 dim) sum_{edges e of T at j} alpha_e^T |e|^2, the part
 * of the Voronoi region V_j inside T when T holds its circumcentre (the
 * shares of a cell add up to its volume for any mesh); link variables of
 * every edge from the exact line integral (linear potentials: the midpoint
 * value; the dipole: closed form).  alpha_jk = alpha_kj and
 * U_kj = conj(U_jk) hold exactly.  The fields potential, mu, b_dir,
 * a_matrix, dipole_m and dipole_x0 mean what they mean in gl_grid_desc (2D
 * points r = (x, y, 0)).  x and cells are host arrays read during the call
 * and not kept.  Every node must lie in a cell.  Meshes of this kind support
 * the residual, the Jacobian, gl_precond_* (level 0 coloured like the coarse
 * levels), gl_jacobian_solve, gl_newton_solve, batches and the continuation
 * calls; not gl_mesh_export_links, the LDS-tiled level 0, or the U-Net.
 * Errors: INVALID_ARGUMENT (dim not 2 or 3, fewer than dim + 1 nodes or
 * more than 2^31 - 2, more than (2^31 - 1) / (dim (dim + 1)) cells, an index
 * out of range, a degenerate cell, a face (triangles: an edge) in more than
 * two cells, a node in no cell), OUT_OF_MEMORY, HIP. */
typedef struct {
    int dim;                   /* 2: triangles, 3: tetrahedra */
    int64_t n_nodes;
    const double *x;           /* host, n_nodes x dim coordinates, row-major */
    int64_t n_cells;
    const int64_t *cells;      /* host, n_cells x (dim + 1) node indices */
    int potential;             /* 0, 1 or 2, as in gl_grid_desc */
    double mu;
    double b_dir[3];
    double a_matrix[9];
    double dipole_m[3];
    double dipole_x0[3];       /* off every edge's line segment */
} gl_simplicial_desc;

gl_status gl_mesh_create_simplicial(const gl_simplicial_desc *desc, gl_stream stream, gl_mesh **out);

/* Replace mu (potential 0 or 2) and recompute the link variables: the
 * continuation parameter of Sec. 4 (numerical parameter continuation). */
gl_status gl_mesh_set_field(gl_mesh *mesh, double mu, gl_stream stream);

/* Number of nodes n. */
gl_status gl_mesh_num_nodes(const gl_mesh *mesh, int64_t *n);

/* Copy the forward-edge link variables of one axis to host memory: entry i
 * (n complex doubles) is U_jk for k = i, j = i + stride(axis); entries of
 * nodes on the upper face of that axis are 0.  Synchronous. */
gl_status gl_mesh_export_links(const gl_mesh *mesh, int axis, void *host_out);

void gl_mesh_destroy(gl_mesh *mesh);

/* ------------------------------------------------------- operators ----- */

/* out = GL(psi) (eq. discr ginla).  out may be NULL (norm only).  If norm_D
 * (host pointer) is non-NULL it receives ||GL(psi)||_D = sqrt(<GL, GL>_R) and
 * the stream is synchronised.  psi and out must not alias. */
gl_status gl_residual(const gl_mesh *mesh, const void *psi, void *out, double *norm_D,
                      gl_stream stream);

/* gl_residual without any device allocation or library-held reduction
 * buffer, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as gl_residual (bitwise the same
 * output and norm).  Its block partial sums and its result live in one
 * static device array per GPU (513 KiB, held until the process ends), so
 * meshes of at most 2^24 = 16,777,216 nodes are accepted (INVALID_ARGUMENT
 * beyond).  Calls that overlap on one GPU, on any streams or threads, share
 * that array and race; serialise them.  Nothing in the array needs clearing
 * between calls. */
gl_status gl_residual_noalloc(const gl_mesh *mesh, const void *psi, void *out, double *norm_D,
                              gl_stream stream);

/* out = J(psi) phi (discrete Jacobian, Sec. 3).  out aliases neither input. */
gl_status gl_jacobian_apply(const gl_mesh *mesh, const void *psi, const void *phi, void *out,
                            gl_stream stream);

/* Secant predictor of natural-parameter continuation in mu (Sec. 4,
 * numerical parameter continuation):
 *   out = psi_m + ratio (psi_m - e^{i chi} psi_prev),  chi = arg <psi_prev, psi_m>
 * with <u, v> = sum |V_i| conj(u_i) v_i.  The phase factor aligns the gauge of
 * the previous solution with psi_m (solutions are orbits e^{i chi} psi, Sec. 2);
 * ratio = (mu_{m+1} - mu_m) / (mu_m - mu_{m-1}).  If <psi_prev, psi_m> = 0 the
 * factor is 1.  out aliases neither input. */
gl_status gl_secant_predict(const gl_mesh *mesh, const void *psi_m, const void *psi_prev, double ratio,
                            void *out, gl_stream stream);

/* out = d GL(psi; mu) / d mu at the mesh's current mu (potential == 0,
 * A = mu A_1): GL_mu = D^-1 (dK-hat/dmu) psi with dU_jk/dmu = -i phi_jk U_jk,
 * phi_jk = (x_j - x_k) . A_1(edge midpoint).  The parameter derivative of the
 * bordered Newton system of pseudo-arclength continuation (Sec. 4, numerical
 * parameter continuation).  UNSUPPORTED for a matrix potential.  out does
 * not alias psi.  Stream-ordered. */
gl_status gl_residual_dmu(const gl_mesh *mesh, const void *psi, void *out, gl_stream stream);

/* *out = <u, v>_R = Re sum_i |V_i| conj(u_i) v_i (eq. disc inner2).  Host
 * scalar; the stream is synchronised. */
gl_status gl_inner(const gl_mesh *mesh, const void *u, const void *v, double *out, gl_stream stream);

/* out = a x + b y with real a, b (out may alias x or y).  Stream-ordered. */
gl_status gl_axpby(const gl_mesh *mesh, double a, const void *x, double b, const void *y, void *out,
                   gl_stream stream);

/* --------------------------------------------------- preconditioner ---- */
typedef struct {
    gl_precision precision; /* storage and arithmetic of the V-cycle */
    int cycles;             /* k in R_k (>= 1; 1 is the paper's choice);
                               0: R_inf = H^-1 D (eq. prec1) to about 1e-12:
                               conjugate gradients on H x = D r from 0 with one
                               V-cycle per step as preconditioner, for a fixed
                               number m of steps chosen at each setup as the
                               steps that take a seeded right-hand side's
                               residual below 1e-12, plus 2 (at most 64;
                               gl_precond_inner_steps); GL_FP64 only */
    int max_coarse;         /* coarsening stops at <= max_coarse rows (default 64) */
    int max_levels;         /* <= 16 */
} gl_amg_opts;

/* Set up R_k(psi) = AMG_k(H, D .), H = K-hat + 2 D |psi|^2 (eq. prec2).
 * *inout == NULL: build the hierarchy (aggregation, colours, sparsity patterns:
 * they depend only on the grid) and its values.  *inout != NULL (a handle from
 * an earlier call on the same mesh): recompute only the values for the new psi
 * (opts may then be NULL; a different precision or cycle count is applied).
 * Errors: SINGULAR (coarsest operator not positive definite, e.g. psi = 0 and
 * A = 0), UNSUPPORTED (a coarse row longer than the setup kernels handle),
 * OUT_OF_MEMORY, HIP. */
gl_status gl_precond_setup(const gl_mesh *mesh, const void *psi, const gl_amg_opts *opts,
                           gl_precond **inout, gl_stream stream);

/* z = R_k r = AMG_k(H, D r): k V-cycles from zero on H x = D r.  r and z are
 * length-n complex vectors and must not alias. */
gl_status gl_precond_apply(const gl_precond *pre, const void *r, void *z, gl_stream stream);

/* Hierarchy summary.  sizes[l], nnz[l], ncolors[l] for l < *nlev
 * (arrays of at least 16 entries; any may be NULL). */
gl_status gl_precond_info(const gl_precond *pre, int *nlev, int64_t *sizes, int64_t *nnz,
                          int *ncolors);

/* Export one array of level l to host memory (synchronous), for bit-exact
 * comparisons.  what: 0 aggregate of each node (int32, n_l), 1 roots (int32,
 * n_{l+1}), 2 colours (int32, n_l), 3 A row pointers (int32, n_l + 1),
 * 4 A columns (int32, nnz), 5 A values (complex double, nnz), 6 P row
 * pointers, 7 P columns, 8 P values, 9 R row pointers, 10 R columns,
 * 11 R values.  Level 0's A is the stencil H and is exported in CSR form with
 * ascending columns.  *bytes: in = capacity, out = size needed; a NULL
 * host_buf only queries the size.  Values are exported in double precision
 * whatever the storage precision. */
gl_status gl_precond_export(const gl_precond *pre, int level, int what, void *host_buf,
                            size_t *bytes);

/* V-cycles per application of the preconditioner: k for R_k, m for R_inf
 * (cycles == 0). */
gl_status gl_precond_inner_steps(const gl_precond *pre, int *steps);

void gl_precond_destroy(gl_precond *pre);

/* Launch-shape choices of the V-cycle (no effect on what is computed beyond
 * the order of rounding in row sums):
 *   lane_shift: lanes that share one row in the sparse kernels of levels >= 1
 *     = the built-in rule (about one lane per 2.5 stored entries of the row)
 *     times 2^lane_shift, clamped to 1 .. 32; -2 .. 2, default 0;
 *   bottom_rows: levels >= 1 with at most this many rows (and at most 64
 *     colours), and all coarser ones, run inside one work-group; 0 = default
 *     512, at most 65536;
 *   dense_rows: the first level >= 1 with at most this many rows has the
 *     V-cycle below it (its smoothing sweeps, residual, transfers and every
 *     coarser level: a linear map of its right-hand side) formed as an
 *     explicit matrix at every setup, in FP64 by the bottom kernel's
 *     arithmetic applied to the unit vectors, and applied as one dense
 *     product; the same operator up to rounding, one dispatch in place of a
 *     few dozen latency-bound ones.  0 = off (default), else 1 .. 8192; the
 *     matrix takes 24 n^2 bytes (FP64 and FP32 copies) and its formation a
 *     workspace of at most 1.5 GB (per-column vectors of every level from
 *     that one down), all held by the handle.
 * Chosen by the autotuner per grid shape; cached iteration graphs of the
 * handle are rebuilt on their next use. */
typedef struct {
    int lane_shift;
    int bottom_rows;
    int dense_rows;
    int l0_tiled;       /* 2D grids: 1, 2, 3 run level 0's passes of a
                           V-cycle as two LDS-tiled kernels (down: the three
                           sweep passes and the residual; up: the coarse
                           correction, the three passes and the output) on
                           tiles of 32 x 32 (1024 threads), 32 x 16 (512) or
                           16 x 16 nodes (256); 0 (default) one dispatch per
                           pass; the same operator up to rounding.  3D grids
                           always use one dispatch per pass */
} gl_tiles;

gl_status gl_precond_set_tiles(gl_precond *pre, const gl_tiles *tiles);
gl_status gl_precond_get_tiles(const gl_precond *pre, gl_tiles *tiles);

/* ----------------------------------------------------- Jacobian solve -- */
typedef struct {
    double rtol;       /* stop when ||b - J x||_{M^-1} <= rtol ||b||_{M^-1} */
    int max_iter;      /* total MINRES iterations */
    int poll_every;    /* iterations between host convergence checks (>= 1) */
    double inner_rtol; /* > 0: the solve is an FP64 iterative refinement whose
                          inner MINRES solves each reduce the residual by this
                          factor, stopped on the true residual; 0 = a single
                          MINRES run stopped on its recurrence estimate with an
                          FP64 preconditioner (or none), refinement with 1e-5
                          with an FP32 one */
    double relax_rtol; /* GL_FP32 / GL_MIXED preconditioner only, > 0: one
                          MINRES recurrence applies the FP64 V-cycle until
                          |eta_j| <= relax_rtol eta_0 and the reduced-precision
                          V-cycle after that (an inexact Krylov method whose
                          operator error may grow as the residual falls), run
                          to rtol and stopped on the true residual (restarted
                          by refinement if that misses rtol); 0 = the reduced
                          precision from the first iteration */
    int deflate;       /* 1: solve on the <.,.>_R-orthogonal complement of the
                          gauge mode u = i psi, which spans the kernel of J at a
                          solution (eq. jacobian nullspace) and makes J nearly
                          singular near one (Sec. 3 names deflation for such
                          systems): MINRES on Pi J Pi x = Pi b, preconditioner
                          Pi R_k Pi, Pi x = x - u <u, x>_R / <u, u>_R.  x is
                          orthogonal to u; for b = -GL(psi) (itself orthogonal
                          to u) this is the Newton step under the phase
                          condition <i psi, dpsi>_R = 0.  res_true is then
                          ||Pi (b - J x)||_D / ||Pi b||_D.  psi = 0: plain solve.
                          0: plain */
    int reorth;        /* > 0: store the Krylov basis (at most reorth vectors)
                          and fully reorthogonalise every new vector against
                          it (Sec. 4: the iteration peaks of the continuation
                          runs come from the loss of orthogonality of the
                          MINRES basis, which this alleviates, as in GMRES).
                          Each MINRES step is followed by one classical
                          Gram-Schmidt pass against every stored vector in
                          the preconditioned product; the coefficients join
                          the projected matrix, whose least-squares problem
                          is solved by Givens rotations (the GMRES form: with
                          an FP32 V-cycle, which is self-adjoint only up to
                          rounding, the basis stays orthogonal and the
                          iteration count stays that of the FP64 one); x =
                          Z y from the stored preconditioned vectors.  A
                          full basis restarts from the true residual (a
                          restart slows these indefinite solves down: size
                          reorth to the expected iteration count); each
                          start measures the true residual, and the solve
                          ends unconverged when a restart has not halved it
                          (the attainable accuracy is above rtol) or after
                          64 starts.  With a reduced-precision V-cycle the
                          passes read a BF16 copy of Z for the coefficients
                          and an FP32 copy of V for the update (the Lanczos
                          coefficients and x stay FP64).  The mesh keeps
                          the basis, with an FP64 V-cycle Z and V in FP64
                          (32 (reorth + 1) n bytes), with a reduced-precision
                          one Z in FP64 plus the two copies (28 (reorth + 1)
                          n bytes), allocated by the first such solve and
                          grown when a larger one comes.  Not with
                          inner_rtol or relax_rtol > 0 (INVALID_ARGUMENT).
                          Batches keep each mesh's basis the same way.
                          0: plain MINRES */
} gl_krylov_opts;

typedef struct {
    int iterations;
    int converged;
    double eta0;     /* ||b||_{M^-1} */
    double res_est;  /* |eta| / eta0 at exit */
    double res_true; /* ||b - J x||_D / ||b||_D at exit */
} gl_krylov_info;

/* Solve J(psi) x = b by preconditioned MINRES in <.,.>_R with x0 = 0
 * (Sec. 4).  With an FP32 preconditioner, or inner_rtol > 0, the solve is an
 * FP64 iterative refinement: r = b - J x in FP64, MINRES on J d = r to
 * inner_rtol, x += d, until the true ||r||_{M^-1} <= rtol ||b||_{M^-1}
 * (info->iterations sums the inner MINRES iterations).  pre == NULL: no preconditioner; otherwise a handle set up for
 * the same psi.  x is written even when the iteration limit is reached
 * (returns NOT_CONVERGED).  BREAKDOWN if <v, M^-1 v> becomes negative or NaN.
 * The stream is synchronised; info may be NULL. */
gl_status gl_jacobian_solve(const gl_mesh *mesh, const void *psi, const gl_precond *pre,
                            const void *b, void *x, const gl_krylov_opts *opts,
                            gl_krylov_info *info, gl_stream stream);

/* ------------------------------------------------------------- Newton -- */
typedef struct {
    double tol;       /* stop when ||GL(psi)||_D < tol */
    int max_steps;    /* <= 63 */
    int fixed_steps;  /* > 0: exactly this many steps, tol ignored */
    int use_precond;  /* 0: unpreconditioned MINRES */
    gl_krylov_opts krylov;
    gl_amg_opts amg;
    int linesearch;   /* 0: the full Newton step (the method as stated in
                         Sec. 4); k in 1..30: backtracking, the step length
                         alpha = 1, 1/2, ... (at most k halvings) until
                         ||GL(psi + alpha dpsi)||_D <= (1 - 1e-4 alpha)
                         ||GL(psi)||_D, else the last one tried.  A
                         globalisation this library adds: plain Newton from
                         a poor start (past a fold of the tracked branch) can
                         cycle or diverge */
} gl_newton_opts;

typedef struct {
    int steps;
    int converged;
    double res[64];         /* ||GL(psi_k)||_D, k = 0 .. steps */
    int krylov_iters[64];   /* MINRES iterations of step k */
    double alpha[64];       /* step length taken at step k (1 without linesearch) */
} gl_newton_info;

/* Newton for GL(psi) = 0 starting from psi_inout (eq. Newton system):
 * per step, set up R_k(psi), solve J(psi) dpsi = -GL(psi), psi += alpha
 * dpsi (alpha = 1 unless opts->linesearch > 0).
 * psi_inout is overwritten with the last iterate.  pre_inout (nullable):
 * a preconditioner handle of this mesh to reuse (only its values are
 * recomputed), or a pointer to NULL that receives the handle built on the
 * first step (then owned by the caller); with pre_inout == NULL the hierarchy
 * is built and freed inside the call.  NOT_CONVERGED if tol is not reached
 * within max_steps (fixed_steps == 0); NONFINITE if a residual becomes
 * NaN/Inf.  Synchronous. */
gl_status gl_newton_solve(const gl_mesh *mesh, void *psi_inout, const gl_newton_opts *opts,
                          gl_precond **pre_inout, gl_newton_info *info, gl_stream stream);

/* -------------------------------------------------------------- batch -- */
/* Many independent instances (each a mesh with its own grid and field, e.g.
 * the members of a continuation sweep) solved together.  The batch holds one
 * preconditioner per instance.  Instances whose launch sequences have the
 * same shape (same grid size and options) run every kernel of a MINRES
 * iteration as ONE dispatch for all of them (grid: work-groups x instances);
 * the iterations of all instances between two convergence checks are one
 * captured HIP graph, replayed with a single launch.  Instances that have
 * converged are skipped by device-side flags.  meshes: count distinct mesh
 * handles that must outlive the batch; 1 <= count <= 4096. */
gl_status gl_batch_create(int count, gl_mesh *const *meshes, gl_batch **out);

/* Newton (as gl_newton_solve) on every instance at once: psi_inout[i] is the
 * start and receives the result of instance i; infos (nullable) receives
 * count gl_newton_info records.  The preconditioner options and tile choices
 * apply to all instances.  Steps run in lock-step: the residuals, the
 * numeric preconditioner setups (once an instance's preconditioner exists;
 * it is built at the instance's first step, the hierarchy limits then fixed:
 * INVALID_ARGUMENT if a later call changes max_coarse or max_levels), the
 * Jacobian solves and the updates of all unconverged instances, each batched
 * per shape group (one dispatch per kernel).  Returns NOT_CONVERGED if any
 * instance missed tol (fixed_steps == 0), else the first failing status.
 * Synchronous. */
gl_status gl_batch_newton_solve(gl_batch *batch, void *const *psi_inout, const gl_newton_opts *opts,
                                gl_newton_info *infos, gl_stream stream);

/* Tile choices for instance `index` (-1: all); applied to its preconditioner
 * now if it exists, and at its creation otherwise. */
gl_status gl_batch_set_tiles(gl_batch *batch, int index, const gl_tiles *tiles);

/* Statistics of the last gl_batch_newton_solve: graph launches, the most
 * batched kernel dispatches per iteration pair (summed over the groups that
 * ran together), the most instance groups that ran together, and host wall
 * seconds (seconds[3], nullable) spent in residuals, preconditioner setups and
 * Krylov solves.  Any output may be NULL. */
gl_status gl_batch_stats(const gl_batch *batch, int64_t *graph_launches, int64_t *dispatches_per_graph,
                         int *groups, double *seconds);

void gl_batch_destroy(gl_batch *batch);

/* --------------------------------------------------- learned predictor -- */
/* A convolutional U-Net that corrects the continuation's start for
 * psi(mu + dmu) on a square 2D grid (a learned refinement of the secant step
 * of the continuation in Sec. 4).  psi_base is the base start (the secant
 * step, or psi itself without history); with s = (psi_base - psi) / dmu the
 * input planes are (Re psi, Im psi, Re s, Im s, mu, 50 dmu); `levels` levels
 * of two 3x3 convolutions + SiLU with base_channels * 2^l channels, vertex
 * subsampling down, linear vertex interpolation up with skip concatenation,
 * a 1x1 head to (o_re, o_im); psi_pred = psi_base + dmu (o_re + i o_im), so a
 * zero network is the base start.  BF16 weights and activations, FP32
 * accumulation on the matrix cores.  The grid needs 2^(levels-1) k + 1 nodes
 * per axis.  levels 1..6; base_channels a multiple of 32. */
gl_status gl_unet_create(int levels, int base_channels, gl_unet **out);
gl_status gl_unet_num_params(const gl_unet *unet, int64_t *n);

/* Parameters: one FP32 vector (host memory), per convolution the weights
 * W[c_out][ky][kx][c_in] (ky, kx = 0..2 for the offsets -1..1) then the bias
 * b[c_out], layers in execution order (encoder levels, decoder levels from
 * the coarsest, head W[2][c] then b[2]).  set_params also resets the Adam
 * moments and step count.  Both synchronise the device. */
gl_status gl_unet_set_params(gl_unet *unet, const float *host_params);
gl_status gl_unet_get_params(const gl_unet *unet, float *host_params);

/* psi_out = network prediction of psi at mu + dmu (device vectors of the
 * mesh's n nodes; psi_out must not alias an input; dmu != 0).
 * Stream-ordered. */
gl_status gl_unet_predict(gl_unet *unet, const gl_mesh *mesh, const void *psi, const void *psi_base, double mu,
                          double dmu, void *psi_out, gl_stream stream);

/* Loss of one sample and (host_grad != NULL) the parameter gradient:
 * with w = (t - psi_base) / dmu,
 * L = sum_i d_i |o_i - w_i|^2 / sum_i d_i (|w_i|^2 + 1e-4) (the squared error
 * of the prediction relative to that of the base start, floored),
 * the target already aligned to psi in phase (gl_secant_predict(mesh, psi,
 * target, -1, out) aligns it).  Synchronous. */
gl_status gl_unet_loss_grad(gl_unet *unet, const gl_mesh *mesh, const void *psi, const void *psi_base, double mu,
                            double dmu, const void *target, double *loss, float *host_grad, gl_stream stream);

typedef struct {
    double lr, beta1, beta2, eps;
} gl_adam_opts;

/* One Adam step (Kingma-Ba, bias-corrected) on the mean loss of `count`
 * aligned samples; *loss (nullable) receives that mean.  Synchronous. */
gl_status gl_unet_train_step(gl_unet *unet, const gl_mesh *mesh, int count, const void *const *psi,
                             const void *const *psi_base, const double *mu, const double *dmu,
                             const void *const *target, const gl_adam_opts *opts, double *loss,
                             gl_stream stream);

void gl_unet_destroy(gl_unet *unet);

/* -------------------------------------------------------- diagnostics -- */
/* Per-kernel timing for roofline reports.  Between gl_profile_start(id) and
 * gl_profile_stop, every launch of the selected internal kernel is bracketed
 * by HIP events on its stream; stop synchronises the device and returns the
 * summed kernel time (ms), the summed algorithmic bytes of those launches
 * (each array the kernel must touch counted once) and the launch count.
 * id: 1 MINRES Jacobian apply (+ fused dot), 2 level-0 Gauss-Seidel colour
 * sweep, 3 level-0 residual, 4 level-0 restriction / prolongation, 5 MINRES
 * v update, 6 MINRES w/x update, 7 GL residual, 8 Gauss-Seidel colour
 * sweep of a level >= 1.  Not thread-safe; for
 * benchmarking only (the events add a small gap between kernels). */
gl_status gl_profile_start(int kernel_id);
gl_status gl_profile_stop(double *ms_total, double *bytes_total, int64_t *launches);

/* ---------------------------------------------------------- allocator -- */
/* Device memory for the handles' workspaces (meshes, preconditioners,
 * batches, U-Nets) from the caller's allocator, e.g. PyTorch's caching
 * allocator: alloc(bytes, stream, ctx) returns device memory of the current
 * device, aligned to 256 bytes, or NULL (the creating call then returns
 * OUT_OF_MEMORY); release(ptr, stream, ctx) takes it back.  stream is NULL
 * (the memory is used on the library's streams, and the device is
 * synchronised before a buffer is released).  The allocator applies to
 * buffers allocated after the call; each buffer is released through the
 * allocator that gave it its memory, so release and ctx must stay valid
 * until every handle created meanwhile is destroyed.  alloc == NULL and
 * release == NULL restore hipMalloc / hipFree; setting only one of them is
 * INVALID_ARGUMENT.  Not thread-safe: set it before creating handles.  Host
 * (pinned) staging memory is not affected. */
typedef void *(*gl_alloc_fn)(size_t bytes, gl_stream stream, void *ctx);
typedef void (*gl_free_fn)(void *ptr, gl_stream stream, void *ctx);
gl_status gl_set_allocator(gl_alloc_fn alloc, gl_free_fn release, void *ctx);

/* ------------------------------------------------------------- errors -- */
const char *gl_status_string(gl_status s);
const char *gl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
