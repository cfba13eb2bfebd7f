"""Oracle: pseudo-arclength continuation in the field strength mu.
TEST INFRASTRUCTURE ONLY.

Sec. 4 (numerical parameter continuation): the solution curve in X x A is
traced by a predictor-corrector method; each step extrapolates along the
curve and corrects perpendicularly to that extrapolation by Newton.  This
module states that method for GL(psi; mu) = 0 on the oracle's meshes:

  parameter derivative  GL_mu(psi) = D^-1 (dK-hat/dmu) psi, with
                        A = mu A_1, U_jk = exp(-i mu phi_jk),
                        phi_jk = (x_j - x_k) . A_1(edge midpoint) (the link
                        integral, exact for linear A), dU/dmu = -i phi U;
  arclength product     <(u, a), (v, b)> = <u, v>_R / |Omega| + a b, so that
                        psi = 1 has unit length;
  predictor             (psi, mu) + ds t, with t the unit tangent: at the
                        first point from J z = -GL_mu (t ~ (z, 1)), later the
                        gauge-aligned secant (psi_m - e^{i chi} psi_{m-1},
                        mu_m - mu_{m-1}), chi = arg <psi_{m-1}, psi_m>;
  corrector             Newton on GL(psi; mu) = 0 and
                        N = <t_psi, psi - psi_p>_R / |Omega| + t_mu (mu - mu_p) = 0
                        (perpendicular to the predictor), the bordered system
                        solved by two Jacobian solves of the same J,
                        J z1 = -GL, J z2 = -GL_mu:
                        dmu = -(N + <t_psi, z1>/|Omega|) / (<t_psi, z2>/|Omega| + t_mu),
                        dpsi = z1 + dmu z2.
The Jacobian solves are restricted to the complement of the gauge mode
i psi (oracle.minres(deflate=True)): J is singular along it at every
solution (eq. jacobian nullspace), and both right-hand sides are orthogonal
to it (<i psi, GL(psi; mu)>_R = 0 for all psi and mu, hence also for GL_mu).
"""
import numpy as np

from . import Amg, Mesh, field_matrix, minres


def gl_dmu(mesh, psi, bdir):
    """d GL(psi; mu) / d mu for the uniform field A = mu/2 (b x r)."""
    psi = np.asarray(psi, dtype=np.complex128)
    a1 = field_matrix(1.0, bdir)
    xj, xk = mesh.x[mesh.ej], mesh.x[mesh.ek]
    mid = 0.5 * (xj + xk)
    phi1 = np.sum((xj - xk) * (mid @ a1.T), axis=1)
    dU = -1j * phi1 * mesh.U
    y = np.zeros(mesh.n, dtype=np.complex128)
    # K-hat(j, k) = -alpha U_jk, K-hat(k, j) = -alpha conj(U_jk); the diagonal
    # does not depend on mu
    np.add.at(y, mesh.ej, -mesh.alpha * dU * psi[mesh.ek])
    np.add.at(y, mesh.ek, -mesh.alpha * np.conj(dU) * psi[mesh.ej])
    return y / mesh.vol


def _solve(m, psi, b, amg, rtol, max_iter):
    x, info, _ = minres(m, psi, b, amg=amg, rtol=rtol, max_iter=max_iter, deflate=True)
    return x, info


def tangent_at(m, psi, bdir, area, krylov_rtol=1e-10, krylov_max_iter=4000, max_coarse=64):
    """Unit tangent (t_psi, t_mu) at a solution, oriented towards growing mu."""
    amg = Amg.for_state(m, psi, max_coarse=max_coarse)
    z, _ = _solve(m, psi, -gl_dmu(m, psi, bdir), amg, krylov_rtol, krylov_max_iter)
    nrm = np.sqrt(m.inner(z, z) / area + 1.0)
    return z / nrm, 1.0 / nrm


def corrector(dim, N, L, bdir, psi_p, mu_p, t_psi, t_mu, area, tol=1e-10, krylov_rtol=1e-10,
              krylov_max_iter=4000, max_newton=20, max_coarse=64):
    """Newton on (GL = 0, N = 0) from the predicted point; returns
    (psi, mu, info)."""
    psi, mu = psi_p.copy(), mu_p
    steps, iters, res = 0, [], []
    while True:
        m = Mesh(dim, N, L, mu=mu, bdir=bdir)
        g = m.gl(psi)
        r = m.norm(g)
        res.append(r)
        if r < tol or steps == max_newton or not np.isfinite(r):
            break
        amg = Amg.for_state(m, psi, max_coarse=max_coarse)
        z1, i1 = _solve(m, psi, -g, amg, krylov_rtol, krylov_max_iter)
        z2, i2 = _solve(m, psi, -gl_dmu(m, psi, bdir), amg, krylov_rtol, krylov_max_iter)
        nres = m.inner(t_psi, psi - psi_p) / area + t_mu * (mu - mu_p)
        dmu = -(nres + m.inner(t_psi, z1) / area) / (m.inner(t_psi, z2) / area + t_mu)
        psi = psi + z1 + dmu * z2
        mu = mu + dmu
        steps += 1
        iters.append((i1["iterations"], i2["iterations"]))
    info = {"newton_steps": steps, "krylov_iters": iters, "res": res,
            "converged": bool(res[-1] < tol)}
    return psi, mu, info


def arclength(dim, N, L, bdir, psi0, mu0, ds, steps, tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=4000,
              max_newton=20, max_coarse=64, max_halvings=3):
    """Trace the branch through (psi0 corrected at mu0) for `steps` steps of
    arclength ds (halved on a failed corrector, at most max_halvings times).
    Returns (records, states): records per point (mu, Newton steps, Krylov
    counts, residual, ds used); states the (mu, psi) of every point."""
    area = float(np.prod(L[:dim]))
    m = Mesh(dim, N, L, mu=mu0, bdir=bdir)
    from . import newton
    psi, info = newton(m, psi0, tol=tol, max_steps=max_newton, krylov_rtol=krylov_rtol,
                       krylov_max_iter=krylov_max_iter, max_coarse=max_coarse, deflate=True)
    mu = mu0
    records = [{"mu": mu, "newton_steps": info["steps"], "res": info["res"][-1], "converged": info["converged"],
                "ds": 0.0}]
    states = [(mu, psi.copy())]
    t_psi, t_mu = tangent_at(m, psi, bdir, area, krylov_rtol, krylov_max_iter, max_coarse)
    for _ in range(steps):
        h = ds
        for _attempt in range(max_halvings + 1):
            psi_p, mu_p = psi + h * t_psi, mu + h * t_mu
            pn, mn, ci = corrector(dim, N, L, bdir, psi_p, mu_p, t_psi, t_mu, area, tol, krylov_rtol,
                                   krylov_max_iter, max_newton, max_coarse)
            if ci["converged"]:
                break
            h *= 0.5
        rec = {"mu": mn, "ds": h, "newton_steps": ci["newton_steps"], "krylov_iters": ci["krylov_iters"],
               "res": ci["res"][-1], "converged": ci["converged"]}
        records.append(rec)
        if not ci["converged"]:
            break
        # gauge-aligned secant: the new tangent
        mm = Mesh(dim, N, L, mu=mn, bdir=bdir)
        ip = np.sum(mm.vol * np.conj(psi) * pn)
        ph = ip / abs(ip) if abs(ip) > 0 else 1.0
        d_psi, d_mu = pn - ph * psi, mn - mu
        nrm = np.sqrt(mm.inner(d_psi, d_psi) / area + d_mu * d_mu)
        t_psi, t_mu = d_psi / nrm, d_mu / nrm
        psi, mu = pn, mn
        states.append((mu, psi.copy()))
    return records, states
