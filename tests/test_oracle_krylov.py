"""Pins of the oracle's MINRES and Newton (Sec. 2 Newton system, Sec. 4 MINRES
with the R_k preconditioner)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def real_matrix(op, n):
    """2n x 2n real matrix of a real-linear map on C^n (Remark on the isometry
    of C^n over R with R^2n)."""
    cols = []
    for unit in (1.0, 1j):
        for k in range(n):
            e = np.zeros(n, complex)
            e[k] = unit
            y = op(e)
            cols.append(np.concatenate([y.real, y.imag]))
    return np.array(cols).T


def to_r(v):
    return np.concatenate([v.real, v.imag])


@pytest.fixture(scope="module")
def small_system():
    m = oracle.Mesh(2, (6, 5), (5.0, 4.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=21)
    amg = oracle.Amg.for_state(m, psi, max_coarse=8)
    assert amg.nlev >= 2
    b = inputs.random_complex(m.n, seed=22)
    Jr = real_matrix(lambda e: m.jac(psi, e), m.n)
    Mr = real_matrix(lambda e: amg.precond(m, e), m.n)
    W = np.diag(np.concatenate([m.vol, m.vol]))
    return m, psi, amg, b, Jr, Mr, W


def test_minres_iterates_minimise_preconditioned_residual(small_system):
    """x_k minimises ||b - J x||_{M^-1} over the Krylov space K_k(M^-1 J, M^-1 b)
    (MINRES optimality), and |eta_k| equals that minimum."""
    m, psi, amg, b, Jr, Mr, W = small_system
    G = W @ Mr
    G = 0.5 * (G + G.T)
    Lg = np.linalg.cholesky(G)
    br = to_r(b)
    Q = []
    v = Mr @ br
    for k in range(1, 9):
        for q in Q:
            v = v - (q @ v) * q
        for q in Q:
            v = v - (q @ v) * q
        Q.append(v / np.linalg.norm(v))
        V = np.array(Q).T
        c, *_ = np.linalg.lstsq(Lg.T @ (Jr @ V), Lg.T @ br, rcond=None)
        x_ref = V @ c
        x, info, hist = oracle.minres(m, psi, b, amg=amg, rtol=0.0, max_iter=k)
        assert info["iterations"] == k
        np.testing.assert_allclose(to_r(x), x_ref, rtol=1e-8, atol=1e-9 * np.abs(x_ref).max())
        r = br - Jr @ x_ref
        assert hist[k] * info["eta0"] == pytest.approx(np.sqrt(r @ G @ r), rel=1e-7)
        v = Mr @ (Jr @ Q[-1])


def test_minres_residual_estimate_monotone(small_system):
    m, psi, amg, b, *_ = small_system
    x, info, hist = oracle.minres(m, psi, b, amg=amg, rtol=1e-12, max_iter=200)
    assert info["converged"]
    assert np.all(np.diff(hist) <= 1e-15)


def test_jacobian_solve_matches_dense_solve(small_system):
    """The Newton-system solve equals the dense solution of the 2n x 2n real
    system (Sec. 4: brute force on a tiny grid), with and without R_1."""
    m, psi, amg, b, Jr, Mr, W = small_system
    ref = np.linalg.solve(Jr, to_r(b))
    for a in (amg, None):
        x, info, _ = oracle.minres(m, psi, b, amg=a, rtol=1e-13, max_iter=500)
        assert info["converged"]
        np.testing.assert_allclose(to_r(x), ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
        assert info["res_true"] < 1e-11


def test_minres_three_distinct_eigenvalues():
    """An operator with three distinct eigenvalues is solved in three steps."""
    n = 40
    rng = np.random.default_rng(3)
    lam = rng.choice([-1.5, 0.5, 3.0], n)
    w = rng.uniform(0.5, 2.0, n)
    b = inputs.random_complex(n, seed=4)
    x, info, hist = oracle.minres_generic(w, lambda v: lam * v, b, rtol=1e-12, max_iter=10)
    assert info["converged"] and info["iterations"] == 3
    np.testing.assert_allclose(x, b / lam, rtol=1e-10)


def test_minres_failure_paths(small_system):
    """max_iter reached -> not converged with outputs written; an indefinite
    preconditioner -> breakdown."""
    m, psi, amg, b, *_ = small_system
    x, info, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-14, max_iter=1)
    assert info["status"] == oracle.ORC_ERR_NOT_CONVERGED and info["iterations"] == 1
    assert np.all(np.isfinite(x))
    w = np.ones(10)
    x, info, _ = oracle.minres_generic(w, lambda v: v, inputs.random_complex(10, 1),
                                       minv=lambda v: -v)
    assert info["status"] == oracle.ORC_ERR_BREAKDOWN


def test_newton_fixed_points():
    """psi = 1 at A = 0 and psi = 0 for any A solve GL = 0: no Newton step."""
    m0 = oracle.Mesh(2, (9, 9), (5.0, 5.0), mu=0.0)
    psi, info = oracle.newton(m0, np.ones(m0.n), tol=1e-12)
    assert info["steps"] == 0 and info["converged"]
    m1 = oracle.Mesh(2, (9, 9), (5.0, 5.0), mu=0.8)
    psi, info = oracle.newton(m1, np.zeros(m1.n), tol=1e-12)
    assert info["steps"] == 0 and info["converged"]


@pytest.fixture(scope="module")
def superconducting_state():
    m = oracle.Mesh(2, (17, 17), (5.0, 5.0), mu=0.8)
    psi, info = oracle.newton(m, np.ones(m.n), tol=1e-11, max_steps=30, krylov_rtol=1e-13)
    return m, psi, info


def test_newton_quadratic_convergence(superconducting_state):
    """Near the solution ||GL||_D contracts quadratically until the rounding
    floor of the near-singular Jacobian (gauge direction) is reached."""
    m, psi, info = superconducting_state
    assert info["converged"]
    assert np.mean(np.abs(psi) ** 2) > 0.3  # not the normal state
    res = info["res"]
    pairs = [(a, b) for a, b in zip(res[:-1], res[1:]) if 1e-9 < a < 0.2]
    assert len(pairs) >= 3
    for a, b in pairs:
        assert b <= 2.0 * a * a


def test_solution_identities(superconducting_state):
    """At a solution <psi, GL(psi)>_R = 0 gives sum_e alpha |psi_j - U psi_k|^2
    = sum_i |V_i| |psi_i|^2 (1 - |psi_i|^2), and i psi spans the gauge kernel of
    J (eq. jacobian nullspace)."""
    m, psi, info = superconducting_state
    kin = (m.alpha * np.abs(psi[m.ej] - m.U * psi[m.ek]) ** 2).sum()
    rhs = (m.vol * np.abs(psi) ** 2 * (1 - np.abs(psi) ** 2)).sum()
    assert kin == pytest.approx(rhs, rel=1e-9)
    assert m.norm(m.jac(psi, 1j * psi)) < 1e-9 * m.norm(psi)


def test_cube_iteration_counts_bounded():
    """Mesh independence on the cube in A_z (Fig. 3 protocol: psi = b = 1,
    x0 = 0, relative residual 1e-11).  The paper's counts come from PyAMG on its
    meshes, so the comparison is a trend band, not parity."""
    with open(os.path.join(GOLDEN, "paper_fig3_cube_az.json")) as f:
        ref = json.load(f)
    side = 10.0 / np.sqrt(3.0)
    counts = {}
    for N in (5, 10, 15):
        m = oracle.Mesh(3, (N, N, N), (side,) * 3, mu=1.0)
        psi = np.ones(m.n, complex)
        amg = oracle.Amg.for_state(m, psi)
        _, info, _ = oracle.minres(m, psi, np.ones(m.n, complex), amg=amg, rtol=1e-11, max_iter=300)
        _, info0, _ = oracle.minres(m, psi, np.ones(m.n, complex), amg=None, rtol=1e-11, max_iter=300)
        counts[N] = (info["iterations"], info0["iterations"])
    # preconditioned counts stay in a band while unpreconditioned ones grow
    assert counts[15][0] <= counts[10][0] + 4
    assert counts[15][1] > counts[10][1] > counts[5][1]
    assert max(c[0] for c in counts.values()) <= 2 * max(ref["R1"])
