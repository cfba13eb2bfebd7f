"""Pins of the oracle's solve on the complement of the gauge mode i psi.

J(psi)(i psi) = i GL(psi) for every psi, so at a solution i psi spans a
kernel of J (eq. jacobian nullspace) and near one J is nearly singular along
it; Sec. 3 names deflation among the remedies.  The oracle's deflated solve
is MINRES on Pi J Pi x = Pi b (Pi the <.,.>_R-orthogonal projector onto the
complement of i psi) with the preconditioner Pi R_1 Pi.  Pinned against a
dense solve of the same restricted system in the real 2n-dimensional form
(Remark on the isometry of C^n over R with R^2n)."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs


def real_matrix(m, psi):
    """J(psi) as a real 2n x 2n matrix acting on (Re x, Im x)."""
    n = m.n
    Jr = np.zeros((2 * n, 2 * n))
    for k in range(n):
        for part, val in ((0, 1.0), (1, 1j)):
            e = np.zeros(n, complex)
            e[k] = val
            y = m.jac(psi, e)
            Jr[:n, k + part * n] = y.real
            Jr[n:, k + part * n] = y.imag
    return Jr


def dense_complement_solve(m, psi, b):
    """x in the complement of u = i psi with Pi (J x - b) = 0, by a basis of
    the complement (orthonormal in the weighted product) and a dense solve."""
    n = m.n
    W = np.concatenate([m.vol, m.vol])
    ur = np.concatenate([(1j * psi).real, (1j * psi).imag])
    # orthonormal basis of {y : sum W u y = 0} in the scaled coordinates s = sqrt(W) y
    su = np.sqrt(W) * ur
    Qs = np.linalg.svd(su[None, :])[2][1:].T          # columns orthogonal to su
    Q = Qs / np.sqrt(W)[:, None]                        # back to y coordinates
    Jr = real_matrix(m, psi)
    br = np.concatenate([b.real, b.imag])
    A = Q.T @ (W[:, None] * Jr) @ Q
    y = np.linalg.solve(A, Q.T @ (W * br))
    xr = Q @ y
    return xr[:n] + 1j * xr[n:]


@pytest.mark.parametrize("precond", [True, False], ids=["R1", "none"])
def test_deflated_solve_equals_dense_complement_solve(precond):
    m = oracle.Mesh(2, (6, 5), (4.0, 3.0), mu=0.7)
    psi = inputs.random_complex(m.n, seed=31)
    b = inputs.random_complex(m.n, seed=32)
    amg = oracle.Amg.for_state(m, psi, max_coarse=8) if precond else None
    x, info, hist = oracle.minres(m, psi, b, amg=amg, rtol=1e-14, max_iter=400, deflate=True)
    ref = dense_complement_solve(m, psi, b)
    assert info["converged"] and info["res_true"] < 1e-12
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()
    # the solution lies in the complement of i psi
    assert abs(m.inner(1j * psi, x)) < 1e-13 * m.norm(x) * m.norm(psi)
    # the residual estimate is non-increasing (MINRES on the restricted operator)
    assert np.all(np.diff(hist) <= 1e-12)


def test_deflated_solve_at_a_solution_where_j_is_singular():
    """At a converged solution J(psi) (i psi) = 0: the plain system is
    singular along the gauge mode, the restricted one is not, and the
    deflated solve equals its dense solution."""
    m = oracle.Mesh(2, (9, 9), (4.0, 4.0), mu=0.4)
    psi, info = oracle.newton(m, np.ones(m.n, complex), tol=1e-13, max_steps=30, krylov_rtol=1e-13)
    assert info["converged"] and np.abs(psi).min() > 0.5
    assert m.norm(m.jac(psi, 1j * psi)) < 1e-11 * m.norm(psi)
    Jr = real_matrix(m, psi)
    sv = np.linalg.svd(Jr, compute_uv=False)
    assert sv[-1] < 1e-10 * sv[0] and sv[-2] > 1e-3 * sv[0]
    b = inputs.random_complex(m.n, seed=33)
    amg = oracle.Amg.for_state(m, psi, max_coarse=16)
    x, ki, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-14, max_iter=400, deflate=True)
    ref = dense_complement_solve(m, psi, b)
    assert ki["converged"]
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()


def test_deflation_is_the_plain_solve_for_psi_zero():
    """u = i psi = 0 leaves nothing to deflate: the plain solve."""
    m = oracle.Mesh(2, (7, 7), (4.0, 4.0), mu=0.6)
    psi = np.zeros(m.n, complex)
    b = inputs.random_complex(m.n, seed=34)
    amg = oracle.Amg.for_state(m, psi, max_coarse=16)
    x0, i0, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-12, max_iter=400)
    x1, i1, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-12, max_iter=400, deflate=True)
    assert i0["iterations"] == i1["iterations"]
    assert np.array_equal(x0, x1)


def test_deflated_newton_step_is_the_phase_condition_step():
    """The deflated Newton step is the Newton step under the phase condition
    <i psi, dpsi>_R = 0, i.e. the bordered system J dpsi + lam (i psi) = -GL
    (Sec. 3 names phase conditions and deflation side by side): dpsi is
    orthogonal to i psi, the residual -GL - J dpsi is a multiple lam i psi of
    the gauge mode, and, J being self-adjoint with J (i psi) = i GL(psi),
    lam = -<i GL(psi), dpsi>_R / <i psi, i psi>_R.  The right-hand side is
    itself orthogonal to i psi (<i psi, GL(psi)>_R = 0 for every psi)."""
    m = oracle.Mesh(2, (11, 11), (5.0, 5.0), mu=0.5)
    psi = 0.9 * np.ones(m.n, complex) + 0.05 * inputs.random_complex(m.n, seed=35)
    g = m.gl(psi)
    b = -g
    u = 1j * psi
    assert abs(m.inner(u, b)) < 1e-13 * m.norm(b) * m.norm(psi)
    amg = oracle.Amg.for_state(m, psi, max_coarse=16)
    x, ki, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-13, max_iter=400, deflate=True)
    assert ki["converged"]
    assert abs(m.inner(u, x)) < 1e-12 * m.norm(x) * m.norm(psi)
    r = b - m.jac(psi, x)
    lam = m.inner(u, r) / m.inner(u, u)
    assert m.norm(r - lam * u) < 1e-11 * m.norm(b)
    lam_closed = -m.inner(1j * g, x) / m.inner(u, u)
    assert lam == pytest.approx(lam_closed, rel=1e-8, abs=1e-14)
    assert abs(lam) > 1e-6  # away from a solution the multiplier is not zero


def test_deflated_newton_is_insensitive_to_rounding():
    """A continuation step (129^2, side 10, mu 0.2 -> 0.22 from the converged
    state): started from the same state rotated by global phases (the same
    mathematical path, rounded differently), deflated Newton takes identical
    steps and Krylov counts, while plain Newton's tail changes (its steps
    pick up a rounding-sized component along the near-kernel i psi)."""
    N, side = (129, 129), (10.0, 10.0)
    m0 = oracle.Mesh(2, N, side, mu=0.2)
    p0, i0 = oracle.newton(m0, np.ones(m0.n, complex), tol=1e-10, max_steps=40, krylov_max_iter=4000,
                           deflate=True)
    assert i0["converged"]
    m1 = oracle.Mesh(2, N, side, mu=0.22)
    defl, plain = [], []
    for rot in (0.0, 0.7):
        _, io = oracle.newton(m1, p0 * np.exp(1j * rot), tol=1e-10, max_steps=40, krylov_max_iter=4000,
                              deflate=True)
        assert io["converged"]
        defl.append(io["krylov_iters"])
        _, ip = oracle.newton(m1, p0 * np.exp(1j * rot), tol=1e-10, max_steps=40, krylov_max_iter=4000)
        assert ip["converged"]
        plain.append(ip["krylov_iters"])
    assert defl[0] == defl[1]
    assert plain[0] != plain[1]
    # and the deflated steps need fewer MINRES iterations
    assert sum(defl[0]) < sum(plain[0])
