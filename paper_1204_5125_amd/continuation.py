"""Natural-parameter continuation in the field strength mu (Sec. 4; the
paper continues with pseudo-arclength, this driver steps mu directly).

Host orchestration only: every state update runs in libglnk kernels
(gl_mesh_set_field, gl_secant_predict, gl_newton_solve).
"""
from . import glnk


def continuation_path(mesh, psi0, mus, tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=4000, max_newton=30,
                      precision=glnk.GL_FP64, max_coarse=64, max_halvings=3, predictor=None, keep=False,
                      callback=None, poll_every=8):
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
    converged point when keep is set."""
    import torch
    handle = glnk.PrecondHandle(mesh)
    opts = dict(tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol, krylov_max_iter=krylov_max_iter,
                precision=precision, max_coarse=max_coarse, precond=handle, raise_on_fail=False,
                poll_every=poll_every)
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
