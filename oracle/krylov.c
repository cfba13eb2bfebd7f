/*
 * Oracle: preconditioned MINRES and Newton.  TEST INFRASTRUCTURE ONLY.
 *
 * Sec. 4: the Jacobian J(psi) is self-adjoint in <u,v>_R = Re <u,v> (discrete
 * weighted product with |V_i|), generally indefinite, so MINRES is the Krylov
 * method; it is preconditioned by R_k(psi) = AMG_k(H, D .), H = K-hat +
 * 2 D |psi|^2 (Sec. 4.1), which is self-adjoint in the same product.  Newton
 * solves J(psi) dpsi = -GL(psi) and updates psi += dpsi (Sec. 2, Newton system).
 *
 * MINRES is the preconditioned Lanczos + Givens recurrence of Paige and
 * Saunders (1975) in the form of Elman, Silvester and Wathen, with x0 = 0 and
 * no reorthogonalisation.  |eta_j| equals the preconditioned residual norm
 * ||b - A x_j||_{M^-1}; the iteration stops when |eta_j| <= rtol |eta_0|.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double wip(int64_t n, const double *w, const cplx *u, const cplx *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += w[i] * creal(conj(u[i]) * v[i]);
    return s;
}

int orc_minres_generic(int64_t n, const double *w, orc_op A, void *actx, orc_op minv,
                       void *mctx, const cplx *b, cplx *x, double rtol, int max_iter,
                       double *hist, orc_krylov_info *info)
{
    const size_t bytes = (size_t)n * sizeof(cplx);
    cplx *v_prev = calloc(1, bytes), *v = malloc(bytes), *v_new = malloc(bytes);
    cplx *z = malloc(bytes), *z_new = malloc(bytes), *q = malloc(bytes);
    cplx *w_prev = calloc(1, bytes), *w_cur = calloc(1, bytes), *w_new = malloc(bytes);
    int rc = ORC_OK;
    memset(info, 0, sizeof(*info));
    for (int64_t i = 0; i < n; ++i) x[i] = 0;

    memcpy(v, b, bytes);
    if (minv) minv(mctx, v, z); else memcpy(z, v, bytes);
    double g2 = wip(n, w, v, z);
    if (!(g2 >= 0.0)) { rc = ORC_ERR_BREAKDOWN; goto done; }
    double gamma = sqrt(g2), gamma_prev = 1.0;
    double eta = gamma, eta0 = gamma;
    double c_prev = 1.0, c = 1.0, s_prev = 0.0, s = 0.0;
    info->eta0 = eta0;
    if (hist) hist[0] = 1.0;
    if (gamma == 0.0) { info->converged = 1; goto done; }

    int j;
    for (j = 1; j <= max_iter; ++j) {
        for (int64_t i = 0; i < n; ++i) z[i] /= gamma;
        A(actx, z, q);
        double delta = wip(n, w, q, z);
        for (int64_t i = 0; i < n; ++i)
            v_new[i] = q[i] - (delta / gamma) * v[i] - (gamma / gamma_prev) * v_prev[i];
        if (minv) minv(mctx, v_new, z_new); else memcpy(z_new, v_new, bytes);
        g2 = wip(n, w, v_new, z_new);
        if (!(g2 >= 0.0)) { rc = ORC_ERR_BREAKDOWN; break; }
        double gamma_new = sqrt(g2);
        double a0 = c * delta - c_prev * s * gamma;
        double a1 = sqrt(a0 * a0 + gamma_new * gamma_new);
        double a2 = s * delta + c_prev * c * gamma;
        double a3 = s_prev * gamma;
        if (!(a1 > 0.0)) { rc = ORC_ERR_BREAKDOWN; break; }
        double c_new = a0 / a1, s_new = gamma_new / a1;
        for (int64_t i = 0; i < n; ++i) {
            w_new[i] = (z[i] - a3 * w_prev[i] - a2 * w_cur[i]) / a1;
            x[i] += c_new * eta * w_new[i];
        }
        eta = -s_new * eta;
        if (hist) hist[j] = fabs(eta) / eta0;
        /* shift the recurrence */
        cplx *t;
        t = v_prev; v_prev = v; v = v_new; v_new = t;
        t = z; z = z_new; z_new = t;
        t = w_prev; w_prev = w_cur; w_cur = w_new; w_new = t;
        gamma_prev = gamma; gamma = gamma_new;
        c_prev = c; c = c_new; s_prev = s; s = s_new;
        info->iterations = j;
        if (fabs(eta) <= rtol * eta0 || gamma == 0.0) { info->converged = 1; break; }
    }
    info->eta = fabs(eta);
    if (rc == ORC_OK && !info->converged) rc = ORC_ERR_NOT_CONVERGED;
done:
    free(v_prev); free(v); free(v_new); free(z); free(z_new); free(q);
    free(w_prev); free(w_cur); free(w_new);
    return rc;
}

/* ------------------------------------------------- Jacobian solve --- */
typedef struct { const orc_mesh *m; const cplx *psi; } jac_ctx;
typedef struct { const orc_mesh *m; const orc_amg *amg; int cycles; cplx *tmp; } pre_ctx;

static void jac_op(void *ctx, const cplx *x, cplx *y)
{
    jac_ctx *c = ctx;
    orc_jac(c->m, c->psi, x, y);
}

/* R_k r = AMG_k(H, D r) */
static void pre_op(void *ctx, const cplx *r, cplx *z)
{
    pre_ctx *c = ctx;
    for (int64_t i = 0; i < c->m->n; ++i) c->tmp[i] = c->m->vol[i] * r[i];
    orc_amg_solve(c->amg, c->tmp, z, c->cycles);
}

int orc_minres(const orc_mesh *m, const cplx *psi, const orc_amg *amg, int cycles,
               const cplx *b, cplx *x, double rtol, int max_iter,
               double *hist, orc_krylov_info *info)
{
    jac_ctx jc = {m, psi};
    pre_ctx pc = {m, amg, cycles < 1 ? 1 : cycles, NULL};
    if (amg) pc.tmp = malloc((size_t)m->n * sizeof(cplx));
    int rc = orc_minres_generic(m->n, m->vol, jac_op, &jc, amg ? pre_op : NULL, &pc, b, x,
                                rtol, max_iter, hist, info);
    free(pc.tmp);
    /* true residual in the D-norm */
    cplx *r = malloc((size_t)m->n * sizeof(cplx));
    orc_jac(m, psi, x, r);
    for (int64_t i = 0; i < m->n; ++i) r[i] = b[i] - r[i];
    double nb = sqrt(orc_inner(m, b, b));
    info->res_true = nb > 0 ? sqrt(orc_inner(m, r, r)) / nb : 0.0;
    free(r);
    return rc;
}

/* ------------------------------------ solve on the complement of i psi --- */
/* Near a solution J(psi) is nearly singular along the gauge mode i psi
 * (eq. jacobian nullspace: exactly singular at a solution); Sec. 3 names
 * deflation among the remedies for such systems.  Reading: MINRES restricted
 * to the <.,.>_R-orthogonal complement of u = i psi, i.e. applied to the
 * self-adjoint operator Pi J Pi, the right-hand side Pi b and the
 * preconditioner Pi R_k Pi, with Pi x = x - u <u, x>_R / <u, u>_R the
 * orthogonal projector.  x0 = 0 lies in the complement and so does every
 * iterate (each is a combination of preconditioner outputs). */
typedef struct {
    const orc_mesh *m;
    const cplx *u;
    double uu;
    orc_op op;
    void *ctx;
    cplx *tmp;
} defl_ctx;

static void project(const orc_mesh *m, const cplx *u, double uu, cplx *x)
{
    if (!(uu > 0.0)) return;
    const double s = orc_inner(m, u, x) / uu;
    for (int64_t i = 0; i < m->n; ++i) x[i] -= s * u[i];
}

/* y = Pi op(Pi x) */
static void projected_op(void *ctx, const cplx *x, cplx *y)
{
    defl_ctx *c = ctx;
    memcpy(c->tmp, x, (size_t)c->m->n * sizeof(cplx));
    project(c->m, c->u, c->uu, c->tmp);
    c->op(c->ctx, c->tmp, y);
    project(c->m, c->u, c->uu, y);
}

int orc_minres_deflated(const orc_mesh *m, const cplx *psi, const orc_amg *amg, int cycles,
                        const cplx *b, cplx *x, double rtol, int max_iter,
                        double *hist, orc_krylov_info *info)
{
    const int64_t n = m->n;
    const size_t bytes = (size_t)n * sizeof(cplx);
    cplx *u = malloc(bytes), *pb = malloc(bytes), *r = malloc(bytes);
    for (int64_t i = 0; i < n; ++i) u[i] = I * psi[i];
    const double uu = orc_inner(m, u, u);
    memcpy(pb, b, bytes);
    project(m, u, uu, pb);
    jac_ctx jc = {m, psi};
    pre_ctx pc = {m, amg, cycles < 1 ? 1 : cycles, NULL};
    if (amg) pc.tmp = malloc(bytes);
    defl_ctx dj = {m, u, uu, jac_op, &jc, malloc(bytes)};
    defl_ctx dm = {m, u, uu, pre_op, &pc, malloc(bytes)};
    int rc = orc_minres_generic(n, m->vol, projected_op, &dj, amg ? projected_op : NULL, &dm, pb, x,
                                rtol, max_iter, hist, info);
    /* without a preconditioner the iterates are combinations of Pi-images
     * already; project once more so that x is in the complement to rounding */
    project(m, u, uu, x);
    orc_jac(m, psi, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    project(m, u, uu, r);
    double nb = sqrt(orc_inner(m, pb, pb));
    info->res_true = nb > 0 ? sqrt(orc_inner(m, r, r)) / nb : 0.0;
    free(pc.tmp); free(dj.tmp); free(dm.tmp);
    free(u); free(pb); free(r);
    return rc;
}

/* ----------------------------------------------------------- Newton --- */
int orc_newton(const orc_mesh *m, cplx *psi, double tol, int max_steps, int fixed_steps,
               double krylov_rtol, int krylov_max_iter, int use_amg, int cycles,
               int max_coarse, int deflate, int linesearch, orc_newton_info *info)
{
    const int64_t n = m->n;
    cplx *r = malloc((size_t)n * sizeof(cplx)), *b = malloc((size_t)n * sizeof(cplx));
    cplx *dx = malloc((size_t)n * sizeof(cplx)), *psik = malloc((size_t)n * sizeof(cplx));
    cplx *hv = malloc((size_t)m->rp[n] * sizeof(cplx));
    int rc = ORC_OK;
    memset(info, 0, sizeof(*info));
    if (max_steps > 63) max_steps = 63;
    if (fixed_steps > 63) fixed_steps = 63;
    orc_gl(m, psi, r);
    double res = sqrt(orc_inner(m, r, r));
    info->res[0] = res;
    int k = 0;
    for (;;) {
        if (fixed_steps > 0) { if (k == fixed_steps) break; }
        else if (res < tol || k == max_steps) break;
        orc_amg *amg = NULL;
        if (use_amg) {
            orc_hmat_values(m, psi, hv);
            /* level 0 of a tensor grid is coloured red-black, of a simplicial mesh greedily */
            rc = orc_amg_build(n, m->rp, m->ci, hv, m->grid ? m->dim : 0, m->N, max_coarse, 16, &amg);
            if (rc != ORC_OK) break;
        }
        for (int64_t i = 0; i < n; ++i) b[i] = -r[i];
        orc_krylov_info ki;
        int krc = deflate ? orc_minres_deflated(m, psi, amg, cycles, b, dx, krylov_rtol, krylov_max_iter, NULL, &ki)
                          : orc_minres(m, psi, amg, cycles, b, dx, krylov_rtol, krylov_max_iter, NULL, &ki);
        orc_amg_free(amg);
        if (krc != ORC_OK && krc != ORC_ERR_NOT_CONVERGED) { rc = krc; break; }
        /* psi_{k+1} = psi_k + alpha dx: alpha = 1, halved while the residual
         * norm does not fall by the factor 1 - 1e-4 alpha (at most linesearch
         * times) */
        memcpy(psik, psi, (size_t)n * sizeof(cplx));
        double alpha = 1.0, res_new;
        for (int h = 0;; ++h) {
            for (int64_t i = 0; i < n; ++i) psi[i] = psik[i] + alpha * dx[i];
            orc_gl(m, psi, r);
            res_new = sqrt(orc_inner(m, r, r));
            if (h == linesearch || res_new <= (1.0 - 1e-4 * alpha) * res) break;
            alpha *= 0.5;
        }
        res = res_new;
        info->krylov_iters[k] = ki.iterations;
        info->alpha[k] = alpha;
        ++k;
        info->res[k] = res;
        if (!isfinite(res)) { rc = ORC_ERR_NOT_CONVERGED; break; }
    }
    info->steps = k;
    info->converged = res < tol;
    if (rc == ORC_OK && fixed_steps <= 0 && !info->converged) rc = ORC_ERR_NOT_CONVERGED;
    free(r); free(b); free(dx); free(psik); free(hv);
    return rc;
}
