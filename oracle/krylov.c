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
 * no reorthogonalisation; orc_minres_reorth_generic stores the basis and
 * reorthogonalises it (the paper's remedy for the loss of orthogonality).  |eta_j| equals the preconditioned residual norm
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

/* ------------------------------------ MINRES with reorthogonalisation --- */
/* Sec. 4 (remark on the iteration peaks of the continuation runs): they come
 * from the loss of orthogonality of the MINRES Krylov basis, which storing
 * the basis and fully reorthogonalising it in every step, as GMRES does,
 * alleviates.  Reading: each step is the MINRES (preconditioned Lanczos)
 * step -- q = A z_j minus its components alpha v_j and gamma_j v_{j-1} --
 * followed by one classical Gram-Schmidt pass of q against every stored
 * v_i in the preconditioned product, h_i = <z_i, q>; the coefficients join
 * the column of the projected matrix (GMRES form), whose least-squares
 * problem min || eta_0 e_1 - H y || is solved by Givens rotations, and
 * x = x_0 + Z y with the stored preconditioned vectors z_i.  With an exactly
 * self-adjoint preconditioner the h_i vanish in exact arithmetic and the
 * iterates are those of MINRES.  When `basis` vectors are stored without
 * convergence the solve restarts from the true residual.  |g_j| is the
 * preconditioned residual norm; the iteration stops when |g_j| <= rtol eta_0,
 * eta_0 the norm of b. */
int orc_minres_reorth_generic(int64_t n, const double *w, orc_op A, void *actx, orc_op minv,
                              void *mctx, const cplx *b, cplx *x, double rtol, int max_iter,
                              int basis, double *hist, orc_krylov_info *info)
{
    if (basis < 2) basis = 2;
    const size_t bytes = (size_t)n * sizeof(cplx);
    cplx *V = malloc(bytes * (size_t)(basis + 1)), *Z = malloc(bytes * (size_t)(basis + 1));
    cplx *q = malloc(bytes), *r = malloc(bytes), *t = malloc(bytes);
    double *H = calloc((size_t)(basis + 1) * basis, sizeof(double));   /* column-major, basis+1 rows */
    double *cs = malloc((size_t)basis * sizeof(double)), *sn = malloc((size_t)basis * sizeof(double));
    double *g = malloc((size_t)(basis + 1) * sizeof(double)), *y = malloc((size_t)basis * sizeof(double));
    double *h = malloc((size_t)(basis + 1) * sizeof(double));
    int rc = ORC_OK, total = 0;
    double eta0 = 0.0, eta = 0.0;
    memset(info, 0, sizeof(*info));
    for (int64_t i = 0; i < n; ++i) x[i] = 0;
    memcpy(r, b, bytes);
    if (hist) hist[0] = 1.0;
    for (int start = 0;; ++start) {
        /* v_0 = r / beta, z_0 = M r / beta */
        memcpy(V, r, bytes);
        if (minv) minv(mctx, V, Z); else memcpy(Z, V, bytes);
        double b2 = wip(n, w, V, Z);
        if (!(b2 >= 0.0)) { rc = ORC_ERR_BREAKDOWN; break; }
        const double beta = sqrt(b2);
        if (start == 0) { eta0 = beta; info->eta0 = eta0; }
        eta = beta;
        if (beta <= rtol * eta0 || beta == 0.0) { info->converged = 1; break; }
        if (total >= max_iter) break;
        for (int64_t i = 0; i < n; ++i) { V[i] /= beta; Z[i] /= beta; }
        g[0] = beta;
        int k = 0, done = 0;
        for (int j = 0; j < basis && total < max_iter; ++j) {
            cplx *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            double *col = H + (size_t)j * (basis + 1);
            A(actx, zj, q);
            /* the MINRES (Lanczos) step */
            const double alpha = wip(n, w, zj, q);
            const double gam = j > 0 ? H[(size_t)(j - 1) * (basis + 1) + j] : 0.0;
            for (int64_t i = 0; i < n; ++i) q[i] -= alpha * vj[i];
            if (j > 0)
                for (int64_t i = 0; i < n; ++i) q[i] -= gam * V[(size_t)(j - 1) * n + i];
            /* full reorthogonalisation: every h_i from the same q */
            for (int i = 0; i <= j; ++i) h[i] = wip(n, w, Z + (size_t)i * n, q);
            for (int i = 0; i <= j; ++i) {
                const cplx *vi = V + (size_t)i * n;
                for (int64_t e = 0; e < n; ++e) q[e] -= h[i] * vi[e];
            }
            for (int i = 0; i <= j; ++i) col[i] = h[i];
            col[j] += alpha;
            if (j > 0) col[j - 1] += gam;
            cplx *zn = Z + (size_t)(j + 1) * n;
            if (minv) minv(mctx, q, zn); else memcpy(zn, q, bytes);
            double g2 = wip(n, w, q, zn);
            if (!(g2 >= 0.0)) { rc = ORC_ERR_BREAKDOWN; done = 1; break; }
            const double gnew = sqrt(g2);
            col[j + 1] = gnew;
            /* the rotations of the previous columns, then this column's own */
            for (int i = 0; i < j; ++i) {
                const double a0 = col[i], a1 = col[i + 1];
                col[i] = cs[i] * a0 + sn[i] * a1;
                col[i + 1] = -sn[i] * a0 + cs[i] * a1;
            }
            const double rr = hypot(col[j], col[j + 1]);
            if (!(rr > 0.0)) { rc = ORC_ERR_BREAKDOWN; done = 1; break; }
            cs[j] = col[j] / rr;
            sn[j] = col[j + 1] / rr;
            col[j] = rr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            ++total;
            eta = fabs(g[j + 1]);
            if (hist) hist[total] = eta / eta0;
            if (eta <= rtol * eta0 || gnew == 0.0) { info->converged = 1; done = 1; break; }
            cplx *vn = V + (size_t)(j + 1) * n;
            for (int64_t i = 0; i < n; ++i) { vn[i] = q[i] / gnew; zn[i] /= gnew; }
        }
        /* x += Z y, R y = g (R: the rotated columns) */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int c = i + 1; c < k; ++c) s -= H[(size_t)c * (basis + 1) + i] * y[c];
            y[i] = s / H[(size_t)i * (basis + 1) + i];
        }
        for (int i = 0; i < k; ++i) {
            const cplx *zi = Z + (size_t)i * n;
            for (int64_t e = 0; e < n; ++e) x[e] += y[i] * zi[e];
        }
        if (done || total >= max_iter) break;
        /* restart from the true residual */
        A(actx, x, t);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    }
    info->iterations = total;
    info->eta = eta;
    if (rc == ORC_OK && !info->converged) rc = ORC_ERR_NOT_CONVERGED;
    free(V); free(Z); free(q); free(r); free(t); free(H); free(cs); free(sn); free(g); free(y); free(h);
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
               const cplx *b, cplx *x, double rtol, int max_iter, int reorth,
               double *hist, orc_krylov_info *info)
{
    jac_ctx jc = {m, psi};
    pre_ctx pc = {m, amg, cycles < 1 ? 1 : cycles, NULL};
    if (amg) pc.tmp = malloc((size_t)m->n * sizeof(cplx));
    int rc = reorth > 0
        ? orc_minres_reorth_generic(m->n, m->vol, jac_op, &jc, amg ? pre_op : NULL, &pc, b, x, rtol, max_iter,
                                    reorth, hist, info)
        : orc_minres_generic(m->n, m->vol, jac_op, &jc, amg ? pre_op : NULL, &pc, b, x, rtol, max_iter, hist,
                             info);
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
                        const cplx *b, cplx *x, double rtol, int max_iter, int reorth,
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
    int rc = reorth > 0
        ? orc_minres_reorth_generic(n, m->vol, projected_op, &dj, amg ? projected_op : NULL, &dm, pb, x, rtol,
                                    max_iter, reorth, hist, info)
        : orc_minres_generic(n, m->vol, projected_op, &dj, amg ? projected_op : NULL, &dm, pb, x, rtol,
                             max_iter, hist, info);
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
               int max_coarse, int deflate, int linesearch, int reorth, orc_newton_info *info)
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
        int krc = deflate ? orc_minres_deflated(m, psi, amg, cycles, b, dx, krylov_rtol, krylov_max_iter, reorth,
                                                NULL, &ki)
                          : orc_minres(m, psi, amg, cycles, b, dx, krylov_rtol, krylov_max_iter, reorth, NULL, &ki);
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
