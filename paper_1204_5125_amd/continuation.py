"""Continuation in the field strength mu (Sec. 4, numerical parameter
continuation): natural continuation, which steps mu directly, and the
paper's pseudo-arclength continuation, which follows the solution curve in
(psi, mu) round folds.

Host orchestration only: every state update, residual, inner product and
solve runs in libglnk kernels (gl_mesh_set_field, gl_secant_predict,
gl_newton_solve, gl_residual, gl_residual_dmu, gl_inner, gl_axpby,
gl_jacobian_solve).
"""
from . import glnk


def continuation_path(mesh, psi0, mus, tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=4000, max_newton=30,
                      precision=glnk.GL_FP64, max_coarse=64, max_halvings=3, predictor=None, keep=False,
                      callback=None, poll_every=8, deflate=False, reorth=0):
    """Continue from psi0 (corrected by Newton at mus[0]) through the field
    values mus.  Each step predicts psi at the next mu -- secant
    psi_m + r (psi_m - e^{i chi} psi_{m-1}) with r the ratio of the steps, or
    `predictor(psi_m, psi_prev, mu_prev, mu_m, mu_next)` when given (a tensor,
    or None for the secant; psi_prev and mu_prev are None at the first step) -- and corrects it by Newton.
    When Newton fails from the predictor's start, the same step is solved
    once more from the secant start (its fallback; the record's predictor
    reads "custom->secant" and failed_newton_steps / failed_krylov_iters hold
    the cost of the failed attempt).  A failed Newton halves the step (at
    most max_halvings times; the halved points are extra steps).
    Returns (records, psi, states): states lists (mu, tensor) of every
    converged point when keep is set.  deflate: every Newton step under the
    phase condition <i psi, dpsi>_R = 0 (Jacobian solves on the complement
    of the gauge mode); reorth > 0: the Jacobian solves store and
    reorthogonalise their Krylov basis (at most reorth vectors)."""
    import torch
    handle = glnk.PrecondHandle(mesh)
    opts = dict(tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol, krylov_max_iter=krylov_max_iter,
                precision=precision, max_coarse=max_coarse, precond=handle, raise_on_fail=False,
                poll_every=poll_every, deflate=deflate, reorth=reorth)
    psi = psi0.clone()
    mesh.set_field(mus[0])
    rc, info = glnk.gl_newton_solve(mesh, psi, **opts)
    records = [{"mu": mus[0], "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
                "res": info["res"][-1], "status": rc, "predictor": "start"}]
    states = [(mus[0], psi.clone())] if keep and rc == 0 else []
    prev, mu, dmu_prev = None, mus[0], None
    pred = torch.empty_like(psi)
    for target_mu in mus[1:]:
        while mu < target_mu - 1e-12:
            h = target_mu - mu
            failed_steps, failed_krylov = 0, 0
            for attempt in range(max_halvings + 1):
                mu_next = mu + h
                mesh.set_field(mu_next)

                def plain():
                    if prev is not None:
                        glnk.gl_secant_predict(mesh, psi, prev, h / dmu_prev, pred)
                        return "secant"
                    pred.copy_(psi)
                    return "constant"

                mu_prev = mu - dmu_prev if prev is not None else None
                custom = predictor(psi, prev, mu_prev, mu, mu_next) if predictor is not None else None
                if custom is not None:
                    pred.copy_(custom)
                    used = "custom"
                else:
                    used = plain()
                rc, info = glnk.gl_newton_solve(mesh, pred, **opts)
                if rc != 0 and used == "custom":
                    failed_steps += info["steps"]
                    failed_krylov += sum(info["krylov_iters"])
                    used = "custom->" + plain()
                    rc, info = glnk.gl_newton_solve(mesh, pred, **opts)
                if rc == 0:
                    break
                h *= 0.5
            rec = {"mu": mu_next, "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
                   "res": info["res"][-1], "status": rc, "predictor": used, "dmu": h}
            if used.startswith("custom->"):
                rec["failed_newton_steps"] = failed_steps
                rec["failed_krylov_iters"] = failed_krylov
            records.append(rec)
            if callback is not None:
                callback(rec, pred)
            if rc != 0:
                return records, psi, states
            prev, psi = psi, pred.clone()
            mu, dmu_prev = mu_next, h
            if keep:
                states.append((mu, psi.clone()))
    return records, psi, states


def continuation(mesh, psi0, mu0, dmu, steps, **kw):
    """Equally spaced continuation: mu0, mu0 + dmu, ..., mu0 + steps dmu.
    Returns (records, psi)."""
    mus = [mu0 + k * dmu for k in range(steps + 1)]
    records, psi, _ = continuation_path(mesh, psi0, mus, **kw)
    return records, psi


def arclength_path(mesh, psi0, mu0, ds, steps, tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=4000,
                   max_newton=20, precision=glnk.GL_FP64, max_coarse=64, max_halvings=3, poll_every=8,
                   callback=None, reorth=0):
    """Pseudo-arclength continuation from psi0 (corrected by Newton at mu0)
    for `steps` steps of arclength ds, in the product
    <(u, a), (v, b)> = <u, v>_R / |Omega| + a b.

    Predictor: (psi, mu) + h t, t the unit tangent (at the first point from
    J z = -GL_mu, t ~ (z, 1) towards growing mu; later the gauge-aligned
    secant of the last two points).  Corrector: Newton on GL(psi; mu) = 0
    and N = <t_psi, psi - psi_p>_R / |Omega| + t_mu (mu - mu_p) = 0, each
    step by the two Jacobian solves J z1 = -GL, J z2 = -GL_mu on the
    complement of i psi (deflate): dmu = -(N + <t_psi, z1>/|Omega|) /
    (<t_psi, z2>/|Omega| + t_mu), dpsi = z1 + dmu z2.  A corrector that does
    not converge within max_newton steps is retried with h halved (at most
    max_halvings times).  reorth > 0: the Jacobian solves store and
    reorthogonalise their Krylov basis (at most reorth vectors).  Returns
    (records, states) with states the (mu, tensor) of every point."""
    import torch
    area = 1.0
    for v in mesh.side:
        area *= v
    kw = dict(rtol=krylov_rtol, max_iter=krylov_max_iter, poll_every=poll_every, deflate=True,
              raise_on_fail=False, reorth=reorth)
    psi = psi0.clone()
    mesh.set_field(mu0)
    handle = glnk.PrecondHandle(mesh)
    rc, info = glnk.gl_newton_solve(mesh, psi, tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol,
                                    krylov_max_iter=krylov_max_iter, precision=precision, max_coarse=max_coarse,
                                    precond=handle, poll_every=poll_every, deflate=True, raise_on_fail=False,
                                    reorth=reorth)
    handle.close()
    mu = mu0
    records = [{"mu": mu, "newton_steps": info["steps"], "res": info["res"][-1], "converged": rc == 0,
                "ds": 0.0, "krylov_iters": [(k, 0) for k in info["krylov_iters"]]}]
    states = [(mu, psi.clone())]
    if rc != 0:
        return records, states
    g, gm, rhs = torch.empty_like(psi), torch.empty_like(psi), torch.empty_like(psi)
    z1, z2, diff = torch.empty_like(psi), torch.empty_like(psi), torch.empty_like(psi)
    psi_p, p, t_psi = torch.empty_like(psi), torch.empty_like(psi), torch.empty_like(psi)
    pre = glnk.Precond(mesh, psi, precision=precision, max_coarse=max_coarse)

    def solve(state, b, x):
        glnk.gl_axpby(mesh, -1.0, b, 0.0, b, rhs)
        rc_, ki = glnk.gl_jacobian_solve(mesh, state, pre, rhs, x, **kw)
        return rc_, ki["iterations"]

    # unit tangent at the first point
    glnk.gl_residual_dmu(mesh, psi, gm)
    rc1, _ = solve(psi, gm, z2)
    nrm = (glnk.gl_inner(mesh, z2, z2) / area + 1.0) ** 0.5
    glnk.gl_axpby(mesh, 1.0 / nrm, z2, 0.0, z2, t_psi)
    t_mu = 1.0 / nrm
    for _ in range(steps):
        h = ds
        for _attempt in range(max_halvings + 1):
            glnk.gl_axpby(mesh, 1.0, psi, h, t_psi, psi_p)
            mu_p = mu + h * t_mu
            p.copy_(psi_p)
            m_ = mu_p
            nsteps, iters, res, ok = 0, [], [], False
            while True:
                mesh.set_field(m_)
                r = glnk.gl_residual(mesh, p, g)
                res.append(r)
                if r < tol:
                    ok = True
                    break
                if nsteps == max_newton or not (r == r) or r == float("inf"):
                    break
                pre.update(p)
                rca, ia = solve(p, g, z1)
                glnk.gl_residual_dmu(mesh, p, gm)
                rcb, ib = solve(p, gm, z2)
                if rca not in (0, 4) or rcb not in (0, 4):
                    break
                glnk.gl_axpby(mesh, 1.0, p, -1.0, psi_p, diff)
                nres = glnk.gl_inner(mesh, t_psi, diff) / area + t_mu * (m_ - mu_p)
                a1 = glnk.gl_inner(mesh, t_psi, z1) / area
                a2 = glnk.gl_inner(mesh, t_psi, z2) / area
                dmu = -(nres + a1) / (a2 + t_mu)
                glnk.gl_axpby(mesh, 1.0, p, 1.0, z1, p)
                glnk.gl_axpby(mesh, 1.0, p, dmu, z2, p)
                m_ += dmu
                nsteps += 1
                iters.append((ia, ib))
            if ok:
                break
            h *= 0.5
        rec = {"mu": m_, "ds": h, "newton_steps": nsteps, "krylov_iters": iters, "res": res[-1], "converged": ok}
        records.append(rec)
        if callback is not None:
            callback(rec, p)
        if not ok:
            break
        # gauge-aligned secant of the last two points: the next tangent
        glnk.gl_secant_predict(mesh, p, psi, -1.0, diff)   # diff = e^{i chi} psi aligned to p
        glnk.gl_axpby(mesh, 1.0, p, -1.0, diff, t_psi)
        d_mu = m_ - mu
        nrm = (glnk.gl_inner(mesh, t_psi, t_psi) / area + d_mu * d_mu) ** 0.5
        glnk.gl_axpby(mesh, 1.0 / nrm, t_psi, 0.0, t_psi, t_psi)
        t_mu = d_mu / nrm
        psi.copy_(p)
        mu = m_
        states.append((mu, psi.clone()))
    return records, states
