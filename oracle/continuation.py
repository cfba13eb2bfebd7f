"""Oracle: natural continuation in mu with the secant predictor.
TEST INFRASTRUCTURE ONLY.

Sec. 4 (numerical parameter continuation): each step predicts the solution at
the next parameter value and corrects it by Newton.  Solutions are gauge
orbits (Sec. 2), so the previous solution is first rotated onto the current
one's global phase: chi = arg <psi_prev, psi_m> with the weighted product of
eq. (discr inner); then psi_pred = psi_m + ratio (psi_m - e^{i chi} psi_prev).
"""
import numpy as np

from . import Mesh, newton


def secant_predict(mesh, psi_m, psi_prev, ratio):
    ip = np.sum(mesh.vol * np.conj(psi_prev) * psi_m)
    ph = ip / abs(ip) if abs(ip) > 0 else 1.0
    return psi_m + ratio * (psi_m - ph * psi_prev)


def continuation(dim, N, L, bdir, psi0, mu0, dmu, steps, tol=1e-10, krylov_rtol=1e-10,
                 krylov_max_iter=4000, max_newton=30, max_coarse=64, max_halvings=3):
    """Same protocol as the GPU driver; returns (records, final psi)."""
    m = Mesh(dim, N, L, mu=mu0, bdir=bdir)
    psi, info = newton(m, psi0, tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol,
                       krylov_max_iter=krylov_max_iter, max_coarse=max_coarse)
    records = [{"mu": mu0, "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
                "res": info["res"][-1], "status": info["status"], "predictor": "start"}]
    prev, mu, dmu_prev = None, mu0, None
    for _ in range(steps):
        h = dmu
        for attempt in range(max_halvings + 1):
            mu_next = mu + h
            m = Mesh(dim, N, L, mu=mu_next, bdir=bdir)
            if prev is not None:
                pred, used = secant_predict(m, psi, prev, h / dmu_prev), "secant"
            else:
                pred, used = psi.copy(), "constant"
            out, info = newton(m, pred, tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol,
                               krylov_max_iter=krylov_max_iter, max_coarse=max_coarse)
            if info["status"] == 0:
                break
            h *= 0.5
        records.append({"mu": mu_next, "newton_steps": info["steps"], "krylov_iters": info["krylov_iters"],
                        "res": info["res"][-1], "status": info["status"], "predictor": used, "dmu": h})
        if info["status"] != 0:
            break
        prev, psi = psi, out
        mu, dmu_prev = mu_next, h
    return records, psi
