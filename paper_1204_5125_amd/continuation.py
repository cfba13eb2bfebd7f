"""Natural-parameter continuation in the field strength mu with the secant
predictor (Sec. 4, numerical parameter continuation; the paper uses
pseudo-arclength, this driver steps mu directly).

Host orchestration only: every state update runs in libglnk kernels
(gl_mesh_set_field, gl_secant_predict, gl_newton_solve).
"""
from . import glnk


def continuation(mesh, psi0, mu0, dmu, steps, tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=4000,
                 max_newton=30, precision=glnk.GL_FP64, max_coarse=64, max_halvings=3, callback=None,
                 predictor=None):
    """Start from psi0 at mu0 (corrected by Newton), then take `steps` steps of
    size dmu.  Each step predicts psi at the next mu (secant, or `predictor`
    if given: a function (psi_m, psi_prev, mu_m, mu_next) -> tensor or None),
    and corrects it by Newton.  A failed Newton halves the step (at most
    max_halvings times).  Returns the list of per-step records."""
    import torch
    handle = glnk.PrecondHandle(mesh)
    opts = dict(tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol, krylov_max_iter=krylov_max_iter,
                precision=precision, max_coarse=max_coarse, precond=handle, raise_on_fail=False)
    psi = psi0.clone()
    mesh.set_field(mu0)
    rc, info = glnk.gl_newton_solve(mesh, psi, **opts)
    records = [{"mu": mu0, "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
                "res": info["res"][-1], "status": rc, "predictor": "start"}]
    prev, mu, dmu_prev = None, mu0, None
    pred = torch.empty_like(psi)
    for _ in range(steps):
        h = dmu
        for attempt in range(max_halvings + 1):
            mu_next = mu + h
            mesh.set_field(mu_next)
            used = "constant"
            custom = predictor(psi, prev, mu, mu_next) if predictor is not None else None
            if custom is not None:
                pred.copy_(custom)
                used = "custom"
            elif prev is not None:
                glnk.gl_secant_predict(mesh, psi, prev, h / dmu_prev, pred)
                used = "secant"
            else:
                pred.copy_(psi)
            rc, info = glnk.gl_newton_solve(mesh, pred, **opts)
            if rc == 0:
                break
            h *= 0.5
        rec = {"mu": mu_next, "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
               "res": info["res"][-1], "status": rc, "predictor": used, "dmu": h}
        records.append(rec)
        if callback is not None:
            callback(rec, pred)
        if rc != 0:
            break
        prev, psi = psi, pred.clone()
        mu, dmu_prev = mu_next, h
    return records, psi
