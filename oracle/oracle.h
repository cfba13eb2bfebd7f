/*
 * Plain FP64 CPU oracle for the discretised extreme type-II Ginzburg-Landau
 * problem of Schloemer & Vanroose, "An optimal linear solver for the Jacobian
 * system of the extreme type-II Ginzburg-Landau problem".
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the GPU path.  It is
 * written to be read against the paper: serial loops, general CSR matrices,
 * no blocking or fusion, double precision throughout.
 *
 * Parity pins (what fixes each function independently of itself) are listed in
 * the docstrings of the Python wrapper and exercised by tests/test_oracle_*.py.
 */
#ifndef GL_ORACLE_H
#define GL_ORACLE_H

#include <complex.h>
#include <stdint.h>

typedef double complex cplx;

/* ---------------------------------------------------------------- mesh --- */

/* Tensor-product grid on the box [-L/2, L/2]^dim (Sec. 3, Voronoi regions and
 * their Delaunay dual; experiments of Sec. 4 centre every domain at 0).
 * A(r) = amat * r is a linear vector potential (3x3 row-major, r = (x,y,z),
 * z = 0 in 2D). */
typedef struct {
    int dim;
    int64_t N[3];
    double L[3], h[3];
    double amat[9];
    int64_t n;
    double *x;        /* n*3 node coordinates */
    double *vol;      /* |V_i|, Voronoi region clipped to the domain */
    int64_t ne;       /* number of edges with nonzero coefficient */
    int64_t *ej, *ek; /* edge (j,k), e_jk = x_j - x_k, j > k */
    double *alpha;    /* edge coefficient alpha_jk */
    cplx *U;          /* link variable U_jk */
    /* Hermitian K-hat (Remark on K = D^-1 K-hat) in canonical CSR:
       rows ascending, columns ascending, diagonal included. */
    int64_t *rp, *ci;
    cplx *kv;
    int grid;         /* 1: tensor grid (dim, N, L, h describe it); 0: simplicial mesh */
} orc_mesh;

int  orc_mesh_build(int dim, const int64_t *N, const double *L, const double *amat,
                    orc_mesh **out);
/* the same grid in the dipole potential mu A_d(x) = mu m x (x - x0) / |x - x0|^3
 * (Sec. 4.1; 2D points are (x, y, 0)), link integrals in closed form */
int  orc_mesh_build_dipole(int dim, const int64_t *N, const double *L, double mu, const double *m,
                           const double *x0, orc_mesh **out);
/* 2D simplicial mesh: nodes xy (n x 2), triangles tri (ntri x 3, node
 * indices).  Edge coefficients by the Corollary's system M alpha = b per
 * triangle (M_ij = <e_i, e_j>^2, b_i = |T| |e_i|^2), summed over the
 * triangles at each edge; |V_j| = sum over triangles T at j of
 * 1/4 sum_{edges e of T at j} alpha_e^T |e|^2, the area of V_j within T when
 * the triangle holds its circumcentre, and sum_j |V_j| = sum_T |T| for any
 * triangulation.  Potential: A = amat r, or mu A_d with dip = (m, x0). */
int  orc_mesh_build_tri(int64_t n, const double *xy, int64_t ntri, const int64_t *tri, const double *amat,
                        orc_mesh **out);
int  orc_mesh_build_tri_dipole(int64_t n, const double *xy, int64_t ntri, const int64_t *tri, double mu,
                               const double *m, const double *x0, orc_mesh **out);
/* 3D: nodes xyz (n x 3), tetrahedra (ntet x 4); the same rules with six
 * edges per simplex and shares 1/6 alpha_e |e|^2. */
int  orc_mesh_build_tet(int64_t n, const double *xyz, int64_t ntet, const int64_t *tet, const double *amat,
                        orc_mesh **out);
int  orc_mesh_build_tet_dipole(int64_t n, const double *xyz, int64_t ntet, const int64_t *tet, double mu,
                               const double *m, const double *x0, orc_mesh **out);
void orc_mesh_free(orc_mesh *m);

/* --------------------------------------------------------- operators --- */
void   orc_khat_apply(const orc_mesh *m, const cplx *x, cplx *y);
void   orc_gl(const orc_mesh *m, const cplx *psi, cplx *out);
void   orc_jac(const orc_mesh *m, const cplx *psi, const cplx *phi, cplx *out);
double orc_inner(const orc_mesh *m, const cplx *u, const cplx *v);
double orc_energy(const orc_mesh *m, const cplx *psi);

/* ---------------------------------------------------------------- AMG --- */
#define ORC_MAX_LEVELS 16

typedef struct {
    int64_t n, nnz;
    int64_t *rp, *ci;
    cplx *v;              /* A_l */
    int64_t nc;           /* number of aggregates (next level size) */
    int64_t *agg;         /* aggregate of each node */
    int64_t *root;        /* root node of each aggregate (ascending) */
    int64_t *prp, *pci;   /* P: n x nc */
    cplx *pv;
    int64_t *rrp, *rci;   /* R = P^H: nc x n */
    cplx *rv;
    int32_t *color;
    int ncolors;
    double omega;
} orc_level;

typedef struct {
    int nlev;
    orc_level lev[ORC_MAX_LEVELS];
    cplx *chol;           /* lower Cholesky factor of the coarsest operator */
    int64_t grid_N[3];    /* level-0 grid dims for parity colouring, or 0 */
    int grid_dim;
} orc_amg;

/* status codes shared by the AMG / Krylov / Newton functions */
#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_SINGULAR 2
#define ORC_ERR_BREAKDOWN 3
#define ORC_ERR_NOT_CONVERGED 4
#define ORC_ERR_AGGREGATION 5

/* Build the hierarchy from A_0 in CSR (copied).  grid_dim/grid_N describe a
 * tensor grid for red-black level-0 colouring (grid_dim == 0: greedy). */
int  orc_amg_build(int64_t n, const int64_t *rp, const int64_t *ci, const cplx *v,
                   int grid_dim, const int64_t *grid_N, int max_coarse, int max_levels,
                   orc_amg **out);
void orc_amg_free(orc_amg *a);
/* x = AMG_k(A_0, b): k V-cycles from x = 0 */
void orc_amg_solve(const orc_amg *a, const cplx *b, cplx *x, int cycles);
/* one symmetric Gauss-Seidel sweep on level l, in place */
void orc_sgs(const orc_level *L, cplx *x, const cplx *b);

/* preconditioner matrix H = K-hat + 2 D |psi|^2 in CSR (same pattern as K-hat) */
void orc_hmat_values(const orc_mesh *m, const cplx *psi, cplx *hv);

/* ------------------------------------------------------------- MINRES --- */
typedef struct {
    int iterations;
    int converged;
    double eta0;        /* ||b||_{M^-1} */
    double eta;         /* final |eta| */
    double res_true;    /* ||b - J x||_D / ||b||_D */
} orc_krylov_info;

/* Solve J(psi) x = b by MINRES in the D-weighted real inner product with
 * preconditioner R_k = AMG_k(H, D .) (amg == NULL: none).  x0 = 0.
 * reorth > 0: the Krylov basis (at most reorth vectors, then a restart) is
 * stored and reorthogonalised in every step (orc_minres_reorth_generic).
 * hist (may be NULL) receives |eta_j|/eta0 for j = 0..iterations. */
int orc_minres(const orc_mesh *m, const cplx *psi, const orc_amg *amg, int cycles,
               const cplx *b, cplx *x, double rtol, int max_iter, int reorth,
               double *hist, orc_krylov_info *info);

/* Generic preconditioned MINRES on an operator that is self-adjoint in
 * <u,v> = Re sum_i w_i conj(u_i) v_i, with an SPD preconditioner minv. */
typedef void (*orc_op)(void *ctx, const cplx *x, cplx *y);
int orc_minres_generic(int64_t n, const double *w, orc_op A, void *actx, orc_op minv,
                       void *mctx, const cplx *b, cplx *x, double rtol, int max_iter,
                       double *hist, orc_krylov_info *info);

/* The same system with the Krylov basis stored: each MINRES step is followed
 * by one classical Gram-Schmidt pass against every stored vector in the
 * preconditioned product, the coefficients join the projected matrix (GMRES
 * form), and x = Z y from the stored preconditioned vectors (Sec. 4, the
 * remedy for the loss of orthogonality).  At most `basis` vectors, then a
 * restart from the true residual. */
int orc_minres_reorth_generic(int64_t n, const double *w, orc_op A, void *actx, orc_op minv,
                              void *mctx, const cplx *b, cplx *x, double rtol, int max_iter,
                              int basis, double *hist, orc_krylov_info *info);

/* Solve J(psi) x = b on the <.,.>_R-orthogonal complement of the gauge mode
 * u = i psi: MINRES (as orc_minres) on Pi J Pi x = Pi b with the orthogonal
 * projector Pi x = x - u <u, x>_R / <u, u>_R and the preconditioner
 * Pi R_k Pi.  x is orthogonal to u.  res_true = ||Pi (b - J x)||_D /
 * ||Pi b||_D.  psi = 0 (u = 0) is the plain solve. */
int orc_minres_deflated(const orc_mesh *m, const cplx *psi, const orc_amg *amg, int cycles,
                        const cplx *b, cplx *x, double rtol, int max_iter, int reorth,
                        double *hist, orc_krylov_info *info);

/* ------------------------------------------------------------- Newton --- */
typedef struct {
    int steps;
    int converged;
    double res[64];       /* ||GL(psi_k)||_D, k = 0..steps */
    int krylov_iters[64];
    double alpha[64];     /* step length of step k */
} orc_newton_info;

/* deflate != 0: every Newton step is solved on the complement of i psi
 * (orc_minres_deflated).  linesearch > 0 (not part of the paper's method, a
 * standard globalisation of Newton): the step psi_k + alpha dpsi takes the
 * first alpha in 1, 1/2, ..., 2^-linesearch with ||GL||_D <= (1 - 1e-4 alpha)
 * ||GL(psi_k)||_D, else the last one.  reorth > 0: the solves store and
 * reorthogonalise their Krylov basis (orc_minres). */
int orc_newton(const orc_mesh *m, cplx *psi, double tol, int max_steps, int fixed_steps,
               double krylov_rtol, int krylov_max_iter, int use_amg, int cycles,
               int max_coarse, int deflate, int linesearch, int reorth, orc_newton_info *info);

#endif
