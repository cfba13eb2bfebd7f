// Preconditioned MINRES for the Jacobian system and the Newton iteration.
//
// Sec. 4: J(psi) is self-adjoint in <u,v>_R = Re sum |V_i| conj(u_i) v_i and
// generally indefinite, so the Krylov method is MINRES, preconditioned by
// R_k(psi) = AMG_k(H, D .) (eq. prec2).  Internally the system is scaled by D:
// A = D J(psi), b_hat = D b, M^-1 = AMG_k(H, .), with the Euclidean real inner
// product; the iterates equal those of MINRES on J in <.,.>_R with M^-1 = R_k,
// because <D r, z>_E = <r, z>_R.  Without a preconditioner M^-1 = D^-1.
//
// Iteration j, gated by device flags so that the host can enqueue (or replay
// a graph of) several iterations between convergence checks:
//   1. the w / x update of iteration j-1 (w_j = (z_{j-1}/gamma_{j-1} - a3 w_{j-2}
//      - a2 w_{j-1}) / a1, x += c eta w_j), fused with q = D J(psi)(z_j / gamma_j)
//      and the partial sums of delta = Re<q, z_j / gamma_j>
//   2. finalize: delta
//   3. v_{j+1} = q - (delta / gamma) v_j - (gamma / gamma_prev) v_{j-1}
//   4. z_{j+1} = M^-1 v_{j+1} (V-cycle) with partial sums of gamma_{j+1}^2
//   5. finalize: the Givens recurrence (minres_finalize)
// The w / x update of the last iteration is applied after the loop.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "amg.h"
#include "stencil.h"

namespace glk {

__global__ void k_ks_init_running(KrylovScalars *ks)
{
    ks->running = (ks->eta0 > 0.0) && (ks->max_iter > 0) && (ks->status == 0);
    ks->iter = 0;
    ks->wx_valid = 0;
}

__global__ void k_ks_init(KrylovScalars *ks, double rtol, int max_iter)
{
    ks->rtol = rtol;
    ks->max_iter = max_iter;
    ks->running = 1;
    ks->wx_valid = 0;
    ks->iter = 0;
    ks->status = 0;
    ks->converged = 0;
    ks->delta = 0.0;
}

// v = D b, v_prev = w = w_prev = x = 0
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_minres_init(GeomT<double> g, const double2 *__restrict__ b,
                                                        double2 *__restrict__ v, double2 *__restrict__ vp,
                                                        double2 *__restrict__ w, double2 *__restrict__ wp,
                                                        double2 *__restrict__ x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    double sf[3];
    const double d = node_volume<DIM, double>(g, c, sf);
    const double2 zero = make_double2(0.0, 0.0);
    v[i] = cscale(b[i], d);
    vp[i] = zero;
    w[i] = zero;
    wp[i] = zero;
    x[i] = zero;
}

// no preconditioner: M^-1 = I in <.,.>_R, i.e. z = D^-1 v in the scaled form,
// with the partial sums of gamma^2 = Re<v, z>
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_unprec(GeomT<double> g, const double2 *__restrict__ v,
                                                   double2 *__restrict__ z, const int *gate, RedSlot slot)
{
    if (gate && *gate == 0) return;
    __shared__ double sm[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double part = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        double sf[3];
        const double d = node_volume<DIM, double>(g, c, sf);
        const double2 vi = v[i];
        const double2 zi = cscale(vi, 1.0 / d);
        z[i] = zi;
        part = redot(vi, zi);
    }
    block_reduce_store(part, slot, sm);
}

// w / x update of the previous iteration (when iter >= 1) and q = D J (z / gamma)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_minres_japply(GeomT<double> g, const double2 *__restrict__ psi,
                                                          const double2 *__restrict__ z,
                                                          const double2 *__restrict__ U,
                                                          double2 *__restrict__ q,
                                                          const double2 *__restrict__ zprev,
                                                          const double2 *__restrict__ w,
                                                          double2 *__restrict__ wp, double2 *__restrict__ x,
                                                          const KrylovScalars *ks, RedSlot slot)
{
    if (ks->running == 0) return;
    __shared__ double sm[kBlock / 64];
    const double ig = 1.0 / ks->gamma;
    const bool upd = ks->iter >= 1;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    double part = 0.0;
    if (i < g.n) {
        if (upd) {
            const double2 zp = cscale(zprev[i], ks->wx_inv_gamma);
            const double2 wn = cscale(csub(csub(zp, cscale(wp[i], ks->wx_a3)), cscale(w[i], ks->wx_a2)),
                                      1.0 / ks->wx_a1);
            wp[i] = wn;
            x[i] = cadd(x[i], cscale(wn, ks->wx_coef));
        }
        int c[3];
        node_coords<DIM>(g.N, i, c);
        const double2 zi = z[i];
        double d, asum;
        const double2 kz = khat_node<DIM, double>(g, i, c, z, U, zi, d, asum);
        const double2 zn = cscale(zi, ig);
        const double2 p = psi[i];
        const double2 react = cadd(cscale(zn, 2.0 * cabs2(p) - 1.0), cmul(cmul(p, p), cconj(zn)));
        const double2 qi = cadd(cscale(kz, ig), cscale(react, d));
        q[i] = qi;
        part = redot(qi, zn);
    }
    block_reduce_store(part, slot, sm);
}

__global__ __launch_bounds__(kBlock) void k_minres_vupdate(int n, const double2 *__restrict__ q,
                                                           const double2 *__restrict__ v,
                                                           double2 *__restrict__ vp, const KrylovScalars *ks)
{
    if (ks->running == 0) return;
    const double a = ks->delta / ks->gamma, b = ks->gamma / ks->gamma_prev;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    vp[i] = csub(csub(q[i], cscale(v[i], a)), cscale(vp[i], b));
}

// the pending w / x update after the last iteration
__global__ __launch_bounds__(kBlock) void k_minres_wx(int n, const double2 *__restrict__ z,
                                                      const double2 *__restrict__ w, double2 *__restrict__ wp,
                                                      double2 *__restrict__ x, const KrylovScalars *ks)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double2 zn = cscale(z[i], ks->wx_inv_gamma);
    const double2 wn = cscale(csub(csub(zn, cscale(wp[i], ks->wx_a3)), cscale(w[i], ks->wx_a2)), 1.0 / ks->wx_a1);
    wp[i] = wn;
    x[i] = cadd(x[i], cscale(wn, ks->wx_coef));
}

// partial sums of ||b - J x||_D^2 and ||b||_D^2
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_true_residual(GeomT<double> g, const double2 *__restrict__ psi,
                                                          const double2 *__restrict__ x,
                                                          const double2 *__restrict__ b,
                                                          const double2 *__restrict__ U, RedSlot s1, RedSlot s2)
{
    __shared__ double sm[kBlock / 64];
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    double pr = 0.0, pb = 0.0;
    if (i < g.n) {
        int c[3];
        node_coords<DIM>(g.N, i, c);
        const double2 xi = x[i];
        double d, asum;
        const double2 kx = khat_node<DIM, double>(g, i, c, x, U, xi, d, asum);
        const double2 p = psi[i];
        const double2 jx = cadd(cadd(cscale(kx, 1.0 / d), cscale(xi, 2.0 * cabs2(p) - 1.0)),
                                cmul(cmul(p, p), cconj(xi)));
        const double2 bi = b[i];
        pr = d * cabs2(csub(bi, jx));
        pb = d * cabs2(bi);
    }
    block_reduce_store(pr, s1, sm);
    block_reduce_store(pb, s2, sm);
}

// psi -= dx
__global__ void k_sub(int n, double2 *psi, const double2 *dx)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) psi[i] = csub(psi[i], dx[i]);
}

// x += d
__global__ void k_add(int n, double2 *x, const double2 *d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = cadd(x[i], d[i]);
}

// r = b - J(psi) x
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_vec(GeomT<double> g, const double2 *__restrict__ psi,
                                                         const double2 *__restrict__ x,
                                                         const double2 *__restrict__ b,
                                                         const double2 *__restrict__ U, double2 *__restrict__ r)
{
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int c[3];
    node_coords<DIM>(g.N, i, c);
    const double2 xi = x[i];
    double d, asum;
    const double2 kx = khat_node<DIM, double>(g, i, c, x, U, xi, d, asum);
    const double2 p = psi[i];
    const double2 jx = cadd(cadd(cscale(kx, 1.0 / d), cscale(xi, 2.0 * cabs2(p) - 1.0)),
                            cmul(cmul(p, p), cconj(xi)));
    r[i] = csub(b[i], jx);
}

__global__ void k_ks_set(KrylovScalars *ks, double rtol, int max_iter)
{
    ks->rtol = rtol;
    ks->max_iter = max_iter;
}

__global__ void k_zero(int n, double2 *x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = make_double2(0.0, 0.0);
}

__global__ void k_copy(int n, double2 *dst, const double2 *src)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

static void read_scalars(const gl_mesh *m, KrylovScalars *h, hipStream_t s)
{
    GLK_HIP(hipMemcpyAsync(m->hscal, m->kscal.get(), sizeof(KrylovScalars), hipMemcpyDeviceToHost, s));
    GLK_HIP(hipStreamSynchronize(s));
    std::memcpy(h, m->hscal, sizeof(KrylovScalars));
}

// Buffers of one MINRES solve.  Two iterations rotate (v, vp), (z, zn), (w, wp)
// back to their starting roles, so a captured pair of iterations can be
// replayed any number of times.
struct Ksolve {
    const gl_mesh *m;
    const double2 *psi;
    const gl_precond *pre;
    const double2 *rhs;
    double2 *x;
    double2 *v, *vp, *z, *zn, *q, *w, *wp;
};

static Ksolve make_ksolve(const gl_mesh *m, const double2 *psi, const gl_precond *pre, const double2 *rhs,
                          double2 *x)
{
    const size_t n = (size_t)m->g.n;
    double2 *W = m->work.get();
    return Ksolve{m, psi, pre, rhs, x, W, W + n, W + 2 * n, W + 3 * n, W + 4 * n, W + 5 * n, W + 6 * n};
}

// x = 0, v = D rhs, z = M^-1 v, gamma_1, eta_0
template <int DIM>
static void ksolve_init(const Ksolve &k, double rtol, int max_iter, hipStream_t s)
{
    const gl_mesh *m = k.m;
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    k_ks_init<<<1, 1, 0, s>>>(ks, rtol, max_iter);
    k_minres_init<DIM><<<nb, kBlock, 0, s>>>(g, k.rhs, k.v, k.vp, k.w, k.wp, k.x);
    GLK_CHECK_LAUNCH();
    if (k.pre) {
        vcycle_enqueue(k.pre, k.v, k.z, nullptr, ks, FIN_MINRES_INIT, s);
    } else {
        k_unprec<DIM><<<nb, kBlock, 0, s>>>(g, k.v, k.z, nullptr, red_slot(m, 1));
        launch_finalize(red_slot(m, 1).partials, nb, FIN_MINRES_INIT, ks, nullptr, nullptr, s);
    }
    GLK_CHECK_LAUNCH();
}

template <int DIM>
static void enqueue_iteration(Ksolve &k, hipStream_t s)
{
    const gl_mesh *m = k.m;
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    const int *gate = &ks->running;
    prof_launch(PROF_MINRES_JAPPLY, (48.0 * n + 16.0 * grid_edges(m->g)) + 96.0 * n, s, [&] {
        k_minres_japply<DIM><<<nb, kBlock, 0, s>>>(g, k.psi, k.z, m->U64.get(), k.q, k.zn, k.w, k.wp, k.x, ks,
                                                   red_slot(m, 0));
    });
    launch_finalize(red_slot(m, 0).partials, nb, FIN_DELTA, ks, nullptr, gate, s);
    prof_launch(PROF_VUPDATE, 64.0 * n, s, [&] { k_minres_vupdate<<<nb, kBlock, 0, s>>>(n, k.q, k.v, k.vp, ks); });
    if (k.pre) {
        vcycle_enqueue(k.pre, k.vp, k.zn, gate, ks, FIN_MINRES_STEP, s);
    } else {
        k_unprec<DIM><<<nb, kBlock, 0, s>>>(g, k.vp, k.zn, gate, red_slot(m, 1));
        launch_finalize(red_slot(m, 1).partials, nb, FIN_MINRES_STEP, ks, nullptr, gate, s);
    }
    GLK_CHECK_LAUNCH();
    std::swap(k.v, k.vp);
    std::swap(k.z, k.zn);
    std::swap(k.w, k.wp);
}

// The graph of two iterations for this (psi, rhs, x, preconditioner) set.
template <int DIM>
static hipGraphExec_t iteration_graph(Ksolve k, hipStream_t s)
{
    gl_mesh *m = const_cast<gl_mesh *>(k.m);
    const uint64_t key[6] = {(uint64_t)(uintptr_t)k.psi, (uint64_t)(uintptr_t)k.rhs, (uint64_t)(uintptr_t)k.x,
                             k.pre ? k.pre->uid : 0,
                             k.pre ? (uint64_t)(k.pre->opts.precision * 4096 + k.pre->opts.cycles) : 0, 0};
    for (auto &e : m->graphs)
        if (std::memcmp(e.key, key, sizeof(key)) == 0) return e.exec;
    hipGraph_t graph = nullptr;
    GLK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_iteration<DIM>(k, s);
        enqueue_iteration<DIM>(k, s);
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(s, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    GLK_HIP(hipStreamEndCapture(s, &graph));
    hipGraphExec_t exec;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GLK_HIP(e);
    if (m->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(m->graphs.front().exec);
        m->graphs.erase(m->graphs.begin());
    }
    GraphEntry ge;
    std::memcpy(ge.key, key, sizeof(key));
    ge.exec = exec;
    m->graphs.push_back(ge);
    return exec;
}

// Iterate until the device flags stop (convergence, breakdown or max_iter),
// then apply the pending w / x update of the last iteration.
template <int DIM>
static void ksolve_iterate(Ksolve k, int max_iter, int poll, hipStream_t s, KrylovScalars &h)
{
    const bool graphs = profiler().kernel == 0;
    hipGraphExec_t exec = graphs ? iteration_graph<DIM>(k, s) : nullptr;
    const Ksolve k0 = k;
    int launched = 0;
    for (;;) {
        read_scalars(k.m, &h, s);
        if (!h.running || launched >= max_iter) break;
        if (graphs) {
            for (int t = 0; t < std::max(1, poll / 2) && launched < max_iter; ++t, launched += 2)
                GLK_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int t = 0; t < poll && launched < max_iter; ++t, ++launched) enqueue_iteration<DIM>(k, s);
        }
    }
    if (h.wx_valid && h.iter >= 1) {
        // roles after h.iter iterations: swapped when h.iter is odd
        Ksolve kk = k0;
        if (h.iter & 1) {
            std::swap(kk.v, kk.vp);
            std::swap(kk.z, kk.zn);
            std::swap(kk.w, kk.wp);
        }
        const int n = k.m->g.n;
        k_minres_wx<<<blocks_for(n), kBlock, 0, s>>>(n, kk.zn, kk.w, kk.wp, kk.x,
                                                    reinterpret_cast<const KrylovScalars *>(k.m->kscal.get()));
        GLK_CHECK_LAUNCH();
    }
}

template <int DIM>
static void true_residual(const gl_mesh *m, const double2 *psi, const double2 *x, const double2 *b, hipStream_t s)
{
    const int nb = blocks_for(m->g.n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    k_true_residual<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, m->U64.get(), red_slot(m, 2), red_slot(m, 3));
    GLK_CHECK_LAUNCH();
    launch_finalize(red_slot(m, 2).partials, nb, FIN_RESNUM, ks, nullptr, nullptr, s);
    launch_finalize(red_slot(m, 3).partials, nb, FIN_RESDEN, ks, nullptr, nullptr, s);
}

template <int DIM>
static gl_status minres_run(const gl_mesh *m, const double2 *psi, const gl_precond *pre,
                            const double2 *b, double2 *x, const gl_krylov_opts &o,
                            gl_krylov_info *info, hipStream_t s)
{
    const int n = m->g.n, nb = blocks_for(n);
    const GeomT<double> g = geom_t<double>(m->g);
    KrylovScalars *ks = reinterpret_cast<KrylovScalars *>(m->kscal.get());
    const int poll = std::max(1, o.poll_every);
    KrylovScalars h;
    gl_status st = GL_OK;
    int iters = 0;
    bool converged = false;
    double eta0 = 0.0, res_est = 0.0;
    const bool fp64 = !pre || pre->opts.precision == GL_FP64;
    if (fp64 && o.inner_rtol <= 0.0) {
        Ksolve k = make_ksolve(m, psi, pre, b, x);
        ksolve_init<DIM>(k, o.rtol, o.max_iter, s);
        ksolve_iterate<DIM>(k, o.max_iter, poll, s, h);
        iters = h.iter;
        converged = h.converged;
        eta0 = h.eta0;
        res_est = h.eta0 > 0 ? std::fabs(h.eta) / h.eta0 : 0.0;
        if (h.status) st = (gl_status)h.status;
    } else {
        // iterative refinement in FP64 around MINRES solves, each to the inner
        // tolerance (FP32 V-cycle: a fixed rounded preconditioner, whose
        // rounding caps what one MINRES run attains), stopped on the true
        // residual in the preconditioner norm
        const double inner = o.inner_rtol > 0.0 ? o.inner_rtol : 1e-5;
        double2 *d = m->work.get() + 9 * (size_t)n, *r = m->work.get() + 10 * (size_t)n;
        k_copy<<<nb, kBlock, 0, s>>>(n, r, b);
        k_zero<<<nb, kBlock, 0, s>>>(n, x);
        Ksolve k = make_ksolve(m, psi, pre, r, d);
        double eta_first = 0.0;
        for (int outer = 0; outer < 64; ++outer) {
            ksolve_init<DIM>(k, inner, 0, s);
            read_scalars(m, &h, s);
            if (h.status) { st = (gl_status)h.status; break; }
            if (outer == 0) eta_first = h.eta0;
            res_est = eta_first > 0 ? h.eta0 / eta_first : 0.0;
            if (h.eta0 <= o.rtol * eta_first || h.eta0 == 0.0) { converged = true; break; }
            if (iters >= o.max_iter) break;
            const double rt = std::max(inner, o.rtol * eta_first / h.eta0);
            k_ks_set<<<1, 1, 0, s>>>(ks, rt, o.max_iter - iters);
            // re-open the gate: max_iter was 0 during the norm-only start
            k_ks_init_running<<<1, 1, 0, s>>>(ks);
            ksolve_iterate<DIM>(k, o.max_iter - iters, poll, s, h);
            iters += h.iter;
            if (h.status) { st = (gl_status)h.status; break; }
            k_add<<<nb, kBlock, 0, s>>>(n, x, d);
            k_residual_vec<DIM><<<nb, kBlock, 0, s>>>(g, psi, x, b, m->U64.get(), r);
            GLK_CHECK_LAUNCH();
        }
        eta0 = eta_first;
    }
    true_residual<DIM>(m, psi, x, b, s);
    read_scalars(m, &h, s);
    if (info) {
        info->iterations = iters;
        info->converged = converged;
        info->eta0 = eta0;
        info->res_est = res_est;
        info->res_true = h.res_den > 0 ? std::sqrt(h.res_num / h.res_den) : 0.0;
    }
    if (st != GL_OK) return st;
    if (!std::isfinite(res_est) || !std::isfinite(h.res_num)) return GL_ERR_NONFINITE;
    return converged ? GL_OK : GL_ERR_NOT_CONVERGED;
}

// All Krylov work runs on the mesh's own stream (graph capture needs a
// non-default stream); it is ordered after, and before, the caller's stream.
gl_status minres_solve(const gl_mesh *m, const double2 *psi, const gl_precond *pre, const double2 *b,
                       double2 *x, const gl_krylov_opts &o, gl_krylov_info *info, hipStream_t s)
{
    GLK_HIP(hipEventRecord(m->ev_in, s));
    GLK_HIP(hipStreamWaitEvent(m->ws, m->ev_in, 0));
    gl_status st = m->g.dim == 2 ? minres_run<2>(m, psi, pre, b, x, o, info, m->ws)
                                 : minres_run<3>(m, psi, pre, b, x, o, info, m->ws);
    GLK_HIP(hipEventRecord(m->ev_out, m->ws));
    GLK_HIP(hipStreamWaitEvent(s, m->ev_out, 0));
    return st;
}

static void check_krylov_opts(const gl_krylov_opts *o, const char *who)
{
    if (!o) fail(GL_ERR_INVALID_ARGUMENT, std::string(who) + ": NULL options");
    if (!(o->rtol >= 0.0) || o->max_iter < 0 || o->max_iter > 100000000 || o->poll_every < 1 ||
        !(o->inner_rtol >= 0.0 && o->inner_rtol < 1.0))
        fail(GL_ERR_INVALID_ARGUMENT, std::string(who) + ": invalid Krylov options");
}

}  // namespace glk

using namespace glk;

extern "C" {

gl_status gl_jacobian_solve(const gl_mesh *mesh, const void *psi, const gl_precond *pre, const void *b,
                            void *x, const gl_krylov_opts *opts, gl_krylov_info *info, gl_stream stream)
{
    gl_status rc = GL_OK;
    gl_status g = guarded([&] {
        if (!mesh || !psi || !b || !x) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: NULL argument");
        if (x == b || x == psi) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: x aliases an input");
        if (pre && pre->mesh != mesh) fail(GL_ERR_INVALID_ARGUMENT, "gl_jacobian_solve: preconditioner of another mesh");
        check_krylov_opts(opts, "gl_jacobian_solve");
        rc = minres_solve(mesh, (const double2 *)psi, pre, (const double2 *)b, (double2 *)x, *opts, info,
                          as_stream(stream));
        if (rc != GL_OK) set_last_error(std::string("gl_jacobian_solve: ") + gl_status_string(rc));
    });
    return g != GL_OK ? g : rc;
}

gl_status gl_newton_solve(const gl_mesh *mesh, void *psi_inout, const gl_newton_opts *opts,
                          gl_precond **pre_inout, gl_newton_info *info, gl_stream stream)
{
    gl_status rc = GL_OK;
    gl_precond *pre = pre_inout ? *pre_inout : nullptr;
    gl_status g = guarded([&] {
        if (!mesh || !psi_inout || !opts) fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: NULL argument");
        if (pre && pre->mesh != mesh) fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: preconditioner of another mesh");
        check_krylov_opts(&opts->krylov, "gl_newton_solve");
        if (opts->max_steps < 0 || opts->max_steps > 63 || opts->fixed_steps < 0 || opts->fixed_steps > 63)
            fail(GL_ERR_INVALID_ARGUMENT, "gl_newton_solve: steps must be in 0..63");
        hipStream_t s = as_stream(stream);
        const int n = mesh->g.n;
        double2 *psi = (double2 *)psi_inout;
        double2 *r = mesh->work.get() + 7 * (size_t)n;
        double2 *dx = mesh->work.get() + 8 * (size_t)n;
        gl_newton_info ni;
        std::memset(&ni, 0, sizeof(ni));
        auto residual = [&]() {
            gl_residual_enqueue(mesh, psi, r, mesh->dscal.get(), s);
            GLK_HIP(hipMemcpyAsync(mesh->hscal, mesh->dscal.get(), sizeof(double), hipMemcpyDeviceToHost, s));
            GLK_HIP(hipStreamSynchronize(s));
            return std::sqrt(mesh->hscal[0]);
        };
        double res = residual();
        ni.res[0] = res;
        int k = 0;
        for (;;) {
            if (!std::isfinite(res)) { rc = GL_ERR_NONFINITE; break; }
            if (opts->fixed_steps > 0) { if (k == opts->fixed_steps) break; }
            else if (res < opts->tol || k == opts->max_steps) break;
            if (opts->use_precond) {
                gl_status ps = gl_precond_setup(mesh, psi, &opts->amg, &pre, stream);
                if (ps != GL_OK) fail(ps, gl_last_error());
                if (pre_inout) *pre_inout = pre;
            }
            gl_krylov_info ki;
            gl_status ks = minres_solve(mesh, psi, opts->use_precond ? pre : nullptr, r, dx, opts->krylov, &ki, s);
            if (ks != GL_OK && ks != GL_ERR_NOT_CONVERGED) { rc = ks; break; }
            k_sub<<<blocks_for(n), kBlock, 0, s>>>(n, psi, dx);
            GLK_CHECK_LAUNCH();
            ni.krylov_iters[k] = ki.iterations;
            ++k;
            res = residual();
            ni.res[k] = res;
        }
        ni.steps = k;
        ni.converged = std::isfinite(res) && res < opts->tol;
        if (rc == GL_OK && opts->fixed_steps == 0 && !ni.converged) rc = GL_ERR_NOT_CONVERGED;
        if (rc != GL_OK) set_last_error(std::string("gl_newton_solve: ") + gl_status_string(rc));
        if (info) *info = ni;
    });
    if (!pre_inout) gl_precond_destroy(pre);
    return g != GL_OK ? g : rc;
}

}  // extern "C"
