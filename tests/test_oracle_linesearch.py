"""The oracle's backtracking Newton (option `linesearch`, a globalisation the
library adds to the paper's plain Newton), pinned against the plain oracle
Newton and the oracle's GL residual: full steps reproduce plain Newton
exactly; a shortened step is psi_k + alpha dpsi with the plain step's dpsi,
meets the sufficient-decrease test, and the doubled step fails it.  And the
fold that stops the batched continuation's instance 8 (129^2, side 10, mu
16/63 + 3 x 0.02): neither Newton form converges at mu = 0.314, the half
step does."""
import numpy as np
import pytest

import oracle
from oracle.continuation import secant_predict
from paper_1204_5125_amd import inputs


def dnorm(m, r):
    return float(np.sqrt(np.sum(m.vol * np.abs(r) ** 2)))


def test_full_steps_are_plain_newton():
    m = oracle.Mesh(2, (33, 33), (5.0, 5.0), mu=0.8)
    psi0 = inputs.random_phase_state(m.n, seed=0)
    pa, a = oracle.newton(m, psi0, max_steps=25, max_coarse=16)
    pb, b = oracle.newton(m, psi0, max_steps=25, max_coarse=16, linesearch=8)
    assert b["alpha"] == [1.0] * b["steps"]
    assert a["res"] == b["res"] and a["krylov_iters"] == b["krylov_iters"]
    assert np.array_equal(pa, pb)


def test_shortened_step_meets_the_decrease_test():
    m = oracle.Mesh(2, (33, 33), (5.0, 5.0), mu=1.5)
    psi0 = inputs.random_phase_state(m.n, seed=1, amplitude=0.3)
    _, info = oracle.newton(m, psi0, max_steps=25, max_coarse=16, linesearch=8)
    assert info["converged"]
    j = next(k for k, a in enumerate(info["alpha"]) if a < 1.0)
    # the state before step j, then that step with and without backtracking
    pj, _ = oracle.newton(m, psi0, fixed_steps=j, max_coarse=16, linesearch=8) if j else (psi0.copy(), None)
    p1, i1 = oracle.newton(m, pj, fixed_steps=1, max_coarse=16, linesearch=8)
    pfull, _ = oracle.newton(m, pj, fixed_steps=1, max_coarse=16)
    alpha = i1["alpha"][0]
    assert alpha == info["alpha"][j] and alpha < 1.0
    dpsi = pfull - pj
    assert np.abs(p1 - (pj + alpha * dpsi)).max() < 1e-12 * np.abs(pj).max()
    r0 = dnorm(m, m.gl(pj))
    assert dnorm(m, m.gl(pj + alpha * dpsi)) <= (1 - 1e-4 * alpha) * r0
    assert not dnorm(m, m.gl(pj + 2 * alpha * dpsi)) <= (1 - 2e-4 * alpha) * r0
    assert i1["res"][1] == pytest.approx(dnorm(m, m.gl(p1)), rel=1e-12)


def test_backtracking_shortens_a_slow_start():
    """From a small random start the full steps wander: 21 plain steps, 9
    with backtracking."""
    m = oracle.Mesh(2, (33, 33), (5.0, 5.0), mu=1.5)
    psi0 = inputs.random_phase_state(m.n, seed=1, amplitude=0.3)
    _, a = oracle.newton(m, psi0, max_steps=30, max_coarse=16)
    _, b = oracle.newton(m, psi0, max_steps=30, max_coarse=16, linesearch=8)
    assert a["converged"] and b["converged"]
    assert b["steps"] < a["steps"] - 5
    # the residual falls at every step whose search succeeded
    for k, al in enumerate(b["alpha"]):
        if al > 2.0 ** -8:
            assert b["res"][k + 1] <= (1 - 1e-4 * al) * b["res"][k]


def test_fold_of_batched_instance_8():
    N, side, mu = 129, 10.0, 2.0 * 8 / 63
    m = oracle.Mesh(2, (N, N), (side, side), mu=mu)
    psi, info = oracle.newton(m, np.ones(m.n, complex), max_steps=40, krylov_max_iter=4000, deflate=True)
    assert info["converged"]
    prev = None
    for _ in range(2):
        mu += 0.02
        m = oracle.Mesh(2, (N, N), (side, side), mu=mu)
        pred = psi.copy() if prev is None else secant_predict(m, psi, prev, 1.0)
        out, info = oracle.newton(m, pred, max_steps=15, krylov_max_iter=1000, deflate=True)
        assert info["converged"]
        prev, psi = psi, out
    m = oracle.Mesh(2, (N, N), (side, side), mu=mu + 0.02)
    pred = secant_predict(m, psi, prev, 1.0)
    _, plain = oracle.newton(m, pred, max_steps=15, krylov_max_iter=1000, deflate=True)
    _, ls = oracle.newton(m, pred, max_steps=15, krylov_max_iter=1000, deflate=True, linesearch=8)
    assert not plain["converged"] and not ls["converged"]
    assert min(ls["res"]) > 0.1   # backtracking stalls at a local minimum of ||GL||
    mh = oracle.Mesh(2, (N, N), (side, side), mu=mu + 0.01)
    _, half = oracle.newton(mh, secant_predict(mh, psi, prev, 0.5), max_steps=15, krylov_max_iter=1000,
                            deflate=True)
    assert half["converged"] and half["steps"] <= 6
