// Smoothed-aggregation hierarchy for the preconditioner matrix
// H = K-hat + 2 D |psi|^2 (Sec. 4.1, eq. prec2).  Level 0 is applied as a
// stencil; its CSR copy exists for setup and export.  Coarser levels are CSR
// with int32 indices, values stored in FP64 and FP32.  The smallest levels and
// the dense coarsest solve run inside one work-group ("bottom" kernel), or the
// cycle below a chosen level is applied as an explicit dense matrix.
#pragma once

#include "common.h"
#include "launch.h"

namespace glk {

constexpr int kMaxLevels = 16;
constexpr int kMaxDense = 2048;   // largest coarsest level handled by the dense solve
constexpr int kMaxRow = 512;      // longest row handled by the setup kernels
constexpr int kMaxColors = 64;    // colours per level handled by the bottom kernel
constexpr int kBottomRows = 512;  // levels up to this size go to the bottom kernel
constexpr int kBottomDenseRows = 512;  // largest explicit sub-cycle the bottom kernel applies
constexpr int kMaxTail = 8192;    // largest level whose sub-cycle is formed as a dense matrix
constexpr size_t kTailWorkspace = size_t(1536) << 20;  // bytes of per-column vectors while forming it

struct Csr {
    int n = 0, m = 0, nnz = 0;  // rows, columns, entries
    DevBuf<int> rp, ci;
    DevBuf<double2> v64;
    DevBuf<float2> v32;
};

struct Level {
    int n = 0;
    Csr A;
    DevBuf<double> diag64;
    DevBuf<float> diag32;
    DevBuf<int> color;
    int ncolors = 0;
    DevBuf<int> cperm;          // rows grouped by colour, ascending inside a colour
    std::vector<int> coff;      // colour c occupies cperm[coff[c] .. coff[c+1])
    // transfer to level l + 1 (absent on the last level)
    int nc = 0;
    DevBuf<int> agg, root, aggsize;
    Csr P, R;
    DevBuf<int> rsrc;           // R entry q = conj(P entry rsrc[q])
    DevBuf<double> rho;         // estimate of rho(D^-1 A) (device scalar)
    DevBuf<int> rap_tp, rap_trip;  // products (p, q, s) of each entry of A_{l+1}, upper triangle
    // Copies used by the V-cycle: levels >= 1 renumbered so that every colour
    // is one contiguous row range (new index r' = position in cperm).
    DevBuf<int> perm, iperm;        // new -> old, old -> new (l >= 1)
    Csr Aa, Pa, Ra;                 // Aa (l >= 1); Pa, Ra: transfers to l + 1
    DevBuf<int> amap, pmap, rmap;   // value of entry q = value of entry map[q] of A, P, R
    Csr Rb;                         // level 0: Ra without the red columns (the residual is zero there),
                                    // columns numbered in the colour-split layout of the level-0 vectors
    Csr Pb;                         // level 0: Pa rows of the black nodes, row t = pair t
    DevBuf<int> pbmap;              // value of entry q of Pb = entry pbmap[q] of P
    DevBuf<double> hs64;            // level 0: the diagonal in that layout
    DevBuf<float> hs32;
    DevBuf<int> bmap;               // value of entry q of Rb = entry bmap[q] of R
    DevBuf<double> dg64;            // diagonal in the new order (l >= 1)
    DevBuf<float> dg32;
    // Aa once more, each colour as a padded row-major block (ELL): row r of
    // colour c has ewidth[c] entries at eoff[c] + (r - coff[c]) * ewidth[c];
    // padding entries point at the row itself with value 0
    std::vector<int> ewidth, eoff;
    DevBuf<int> eci, emap;          // emap: entry of Aa, or -1 for padding
    DevBuf<double2> ev64;
    DevBuf<float2> ev32;
    // V-cycle vectors (new order on levels >= 1; level 0: split by colour, the
    // node of colour c in red-black pair t at c * npair + t, 2 npair entries)
    DevBuf<double2> b64, x64, r64;
    DevBuf<float2> b32, x32, r32;
};

// One level as seen by the bottom kernel (device-resident descriptor).
template <class T>
struct BottomLevel {
    int n, nc, ncolors;
    const int *rp, *ci;
    const C<T> *v;
    const T *diag;
    int coff[kMaxColors + 1];  // colour c = rows coff[c] .. coff[c+1]-1
    const int *prp, *pci;
    const C<T> *pv;
    const int *rrp, *rci;
    const C<T> *rv;
    C<T> *b, *x, *r;
    // the operator once more as per-colour padded blocks (ELL): row r of
    // colour c holds ewidth[c] entries at eoff[c] + (r - coff[c]) ewidth[c]
    const int *eci;
    const C<T> *ev;
    int ewidth[kMaxColors], eoff[kMaxColors];
};

template <class T>
struct BottomDesc {
    int first, last;  // levels first .. last; last: the coarsest, or the level
                      // whose sub-cycle is an explicit matrix
    int lds_level;    // level whose x lives in LDS (-1: none)
    const C<T> *cinv; // dense row-major operator of level `last`
    BottomLevel<T> L[kMaxLevels];
};

// Krylov scalar state kept on the device (see krylov.hip).
// Deflation of the gauge mode u = i psi (the solve restricted to the
// <.,.>_R-orthogonal complement of u): defl_c = <u, u>_R, defl_sq the last
// projection coefficient of a residual-space vector, defl_sy that of the
// newest preconditioner output (0 when there is nothing to project), and
// defl_pending set by the recurrence whenever it has produced a new one.
struct KrylovScalars {
    double gamma, gamma_prev, c, c_prev, s, s_prev, eta, eta0, delta;
    double wx_inv_gamma, wx_a1, wx_a2, wx_a3, wx_coef;
    double rtol;
    double res_num, res_den;
    double defl_c, defl_sq, defl_sy, res_u_num, res_u_den;
    double rg2;  // reorthogonalised solves: <v, M^-1 v> of the newest vector
    int iter, max_iter, running, wx_valid, status, converged;
    int defl_pending;
};

// What a reduction's finalize kernel does with the total.
enum FinalizeMode {
    FIN_STORE = 0, FIN_MINRES_INIT = 1, FIN_MINRES_STEP = 2, FIN_DELTA = 3, FIN_RESNUM = 4,
    FIN_RESDEN = 5, FIN_DEFL_Y = 6, FIN_REORTH = 7
};

// Scalar part of preconditioned MINRES (Paige-Saunders Lanczos + Givens
// recurrence, x0 = 0), run by one thread once gamma^2 = <v, M^-1 v> of the new
// Lanczos vector is known.  INIT: first vector, gamma_1 = eta_0.  STEP: the
// Givens rotation of iteration j, the coefficients of the w / x update and the
// convergence test |eta| <= rtol eta_0.
__device__ __forceinline__ void minres_finalize(KrylovScalars *ks, int mode, double total)
{
    if (mode == FIN_DELTA) { ks->delta = total; return; }
    if (mode == FIN_RESNUM) { ks->res_num = total; return; }
    if (mode == FIN_RESDEN) { ks->res_den = total; return; }
    if (mode == FIN_REORTH) {
        // the rest of the step is the column of the projected matrix
        ks->rg2 = total;
        ks->defl_pending = 1;
        return;
    }
    if (mode == FIN_DEFL_Y) {
        // coefficient of the newest preconditioner output along u, or 0 when
        // the recurrence has produced none since the last projection
        ks->defl_sy = ks->defl_pending ? total : 0.0;
        ks->defl_pending = 0;
        return;
    }
    if (mode == FIN_MINRES_INIT) {
        ks->iter = 0;
        ks->converged = 0;
        ks->status = 0;
        ks->wx_valid = 0;
        if (!(total >= 0.0)) {
            ks->status = GL_ERR_BREAKDOWN;
            ks->running = 0;
            return;
        }
        const double g = sqrt(total);
        ks->gamma = g;
        ks->gamma_prev = 1.0;
        ks->eta = g;
        ks->eta0 = g;
        ks->c = ks->c_prev = 1.0;
        ks->s = ks->s_prev = 0.0;
        ks->converged = (g == 0.0);
        ks->running = (g > 0.0) && (ks->max_iter > 0);
        ks->defl_pending = 1;
        return;
    }
    // FIN_MINRES_STEP
    if (!(total >= 0.0)) {
        ks->status = GL_ERR_BREAKDOWN;
        ks->running = 0;
        ks->wx_valid = 0;
        return;
    }
    const double gnew = sqrt(total);
    const double g = ks->gamma, dl = ks->delta;
    const double a0 = ks->c * dl - ks->c_prev * ks->s * g;
    const double a1 = sqrt(a0 * a0 + gnew * gnew);
    const double a2 = ks->s * dl + ks->c_prev * ks->c * g;
    const double a3 = ks->s_prev * g;
    if (!(a1 > 0.0)) {
        ks->status = GL_ERR_BREAKDOWN;
        ks->running = 0;
        ks->wx_valid = 0;
        return;
    }
    const double cn = a0 / a1, sn = gnew / a1;
    ks->wx_inv_gamma = 1.0 / g;
    ks->wx_a1 = a1;
    ks->wx_a2 = a2;
    ks->wx_a3 = a3;
    ks->wx_coef = cn * ks->eta;
    ks->eta = -sn * ks->eta;
    ks->gamma_prev = g;
    ks->gamma = gnew;
    ks->c_prev = ks->c;
    ks->c = cn;
    ks->s_prev = ks->s;
    ks->s = sn;
    ks->iter += 1;
    ks->wx_valid = 1;
    ks->defl_pending = 1;
    if (fabs(ks->eta) <= ks->rtol * ks->eta0 || gnew == 0.0) {
        ks->converged = 1;
        ks->running = 0;
    } else if (ks->iter >= ks->max_iter) {
        ks->running = 0;
    }
}

// Sum nparts block partials in a fixed order (one work-group) and act on the
// total: store it to *out (FIN_STORE) or update the Krylov scalars.
void launch_finalize(const double *partials, int nparts, int mode, KrylovScalars *ks, double *out,
                     const int *gate, const Launch &L);
inline void launch_finalize(const double *partials, int nparts, int mode, KrylovScalars *ks, double *out,
                            const int *gate, hipStream_t s)
{
    launch_finalize(partials, nparts, mode, ks, out, gate, Launch{s});
}

}  // namespace glk

struct gl_precond {
    const gl_mesh *mesh = nullptr;
    uint64_t uid = 0;              // unique per handle (keys cached graphs)
    gl_amg_opts opts{};
    int nlev = 0;
    int bottom = 0;                // first level handled by the bottom kernel
    int tail = 0;                  // level whose sub-cycle is one dense product (the coarsest if none)
    int bottom_rows = glk::kBottomRows;  // tile choices (gl_precond_set_tiles)
    int lane_shift = 0;
    int dense_rows = 0;
    int l0_tiled = 0;              // 1: 2D level-0 passes in two LDS-tiled kernels
    bool has_values = false;       // a numeric setup has run
    glk::Level L[glk::kMaxLevels];
    glk::DevBuf<double2> cfac;     // Cholesky factor of the coarsest operator
    glk::DevBuf<double2> cinv64;   // its inverse, applied as a dense product
    glk::DevBuf<float2> cinv32;
    glk::DevBuf<int> status;       // device status word of the numeric setup
    glk::DevBuf<double> cdmax;     // largest diagonal entry of the coarsest operator
    glk::DevBuf<double2> cyc_r;    // k > 1 cycles: level-0 residual (and a setup scratch vector)
    // R_inf (cycles == 0): conjugate gradients on H x = v with the V-cycle as
    // preconditioner, a fixed number pcg_m of steps chosen at each setup
    glk::DevBuf<double2> pcg;      // x, r, p, q, z (5 n)
    glk::DevBuf<double> pcg_sc;    // <r_j, z_j> (j = 0 .. m) then <p_j, H p_j> (j = 0 .. m-1)
    int pcg_m = 0;
    glk::DevBuf<double2> vin;      // gl_precond_apply: D r (and a setup scratch vector)
    glk::DevBuf<double> pwn;       // setup: norms of the spectral-radius estimate
    glk::DevBuf<char> bdesc64, bdesc32;  // BottomDesc<double>, BottomDesc<float>
    // explicit sub-cycle of level `tail` (when above the coarsest): row-major
    // n_tail x n_tail in the V-cycle's row order, formed by TailColumns
    // from a descriptor of levels tail .. coarsest, a block of columns per
    // work-group
    glk::DevBuf<double2> tinv64;
    glk::DevBuf<float2> tinv32;
    glk::DevBuf<double2> tws;      // per-block vectors of that formation
    glk::DevBuf<char> tdesc64;
    size_t tws_col = 0;            // elements per block of columns in tws
    int tws_cols = 0;              // blocks of columns per launch
    int lds64 = 0, lds32 = 0;      // dynamic LDS bytes of the bottom kernel
};

namespace glk {
// V-cycle entry used by gl_precond_apply and by MINRES: z = AMG_k(H, v).
// gate (nullable): skip all work when *gate == 0.  When ks != nullptr the
// kernel that writes z also reduces Re<v, z> and the total is handed to
// minres_finalize(ks, mode, total).
// prec: the precision of this application (the handle holds both).
void vcycle_enqueue(const gl_precond *pre, const double2 *v, double2 *z, const int *gate,
                    KrylovScalars *ks, int mode, const Launch &L, gl_precision prec);
void vcycle_enqueue(const gl_precond *pre, const double2 *v, double2 *z, const int *gate,
                    KrylovScalars *ks, int mode, const Launch &L);  // in the handle's precision
void gl_residual_enqueue(const gl_mesh *m, const double2 *psi, double2 *out, double *dresult,
                         hipStream_t s);
// the same two dispatches (residual with block partials, fixed-order sum),
// launched or recorded; no profiling brackets
void gl_residual_enqueue(const gl_mesh *m, const double2 *psi, double2 *out, double *dresult,
                         const Launch &L);
void jacobian_enqueue(const gl_mesh *m, const double2 *psi, const double2 *phi, double2 *out,
                      hipStream_t s);
void precond_numeric(gl_precond *pre, const double2 *psi, hipStream_t s);
// A numeric setup in two halves, so that many instances can be recorded and
// run as batched dispatches: every kernel (launched or recorded; the coarsest
// factor's failure flag is left in pre->status), then, with that flag read,
// the error check, the explicit sub-cycle and R_inf's step count.
void precond_numeric_enqueue(gl_precond *pre, const double2 *psi, const Launch &L);
void precond_numeric_finish(gl_precond *pre, bool singular, hipStream_t s);
void check_amg_opts(const gl_amg_opts *opts, const char *who);
void pcg_calibrate(gl_precond *pre, hipStream_t s);  // R_inf: the CG step count of this setup
constexpr int kPcgMaxSteps = 64;
void scale_by_volume(const gl_mesh *m, const double2 *x, double2 *y, hipStream_t s);
void bottom_descriptors(gl_precond *pre, hipStream_t s);
void form_tail(gl_precond *pre, hipStream_t s);  // after a numeric setup
uint64_t new_precond_uid();
}  // namespace glk
