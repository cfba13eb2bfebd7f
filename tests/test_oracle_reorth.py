"""Pins of the oracle's MINRES with full reorthogonalisation (Sec. 4: the
iteration peaks of the continuation runs come from the loss of
orthogonality of the Krylov basis, which storing and reorthogonalising the
basis in every step, as GMRES does, alleviates).

The method minimises the preconditioned residual norm ||b - J x||_{M} over
x in the Krylov space K_k(M J, M b), M = R_1 the V-cycle (self-adjoint and
positive definite in the D-weighted real product): checked against that
least-squares problem solved densely on a small grid (the real-linear maps
as 2n x 2n matrices).  Its first iterates are MINRES's; it needs fewer
iterations than MINRES where MINRES loses orthogonality; it stays close to
its count when the preconditioner is perturbed by a non-self-adjoint term of
FP32 rounding size, where MINRES's count grows; restarts and the deflated
form converge."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs


def dense(f, n):
    """The real-linear map f on C^n as a 2n x 2n real matrix."""
    cols = []
    for k in range(2 * n):
        e = np.zeros(n, complex)
        e[k % n] = 1.0 if k < n else 1j
        y = f(e)
        cols.append(np.concatenate([y.real, y.imag]))
    return np.array(cols).T


def to_c(v, n):
    return v[:n] + 1j * v[n:]


def system(N, seed, max_coarse=16):
    """The second Newton system on an N x N grid (side 10, mu 1 along z)
    from a random-phase start, the experiments' workload."""
    mo = oracle.Mesh(2, (N, N), (10., 10.), mu=1.0)
    psi0 = inputs.random_phase_state(mo.n, seed=seed)
    psi1, _ = oracle.newton(mo, psi0, fixed_steps=1, krylov_rtol=1e-10, krylov_max_iter=2000,
                            max_coarse=max_coarse)
    amg = oracle.Amg.for_state(mo, psi1, max_coarse=max_coarse)
    return mo, psi1, amg, -mo.gl(psi1)


def test_iterates_minimise_over_the_krylov_space():
    mo, psi, amg, b = system(6, 3, max_coarse=4)
    n = mo.n
    Jm = dense(lambda x: mo.jac(psi, x), n)
    Mm = dense(lambda r: amg.precond(mo, r), n)
    W = np.diag(np.concatenate([mo.vol, mo.vol]))
    G = W @ Mm
    assert np.abs(G - G.T).max() < 1e-12 * np.abs(G).max()       # M self-adjoint in the product
    L = np.linalg.cholesky(0.5 * (G + G.T))
    bv = np.concatenate([b.real, b.imag])
    # an orthonormal basis of K_k(M J, M b) by dense Arnoldi in the
    # Euclidean product (two Gram-Schmidt passes per vector)
    Q = [Mm @ bv / np.linalg.norm(Mm @ bv)]
    for _ in range(29):
        u = Mm @ (Jm @ Q[-1])
        for _ in range(2):
            u = u - np.array(Q).T @ (np.array(Q) @ u)
        Q.append(u / np.linalg.norm(u))
    Q = np.array(Q).T
    for k in (1, 3, 8, 15, 30):
        Qk = Q[:, :k]
        c, *_ = np.linalg.lstsq(L.T @ (Jm @ Qk), L.T @ bv, rcond=None)
        want = to_c(Qk @ c, n)
        x, info, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k, reorth=64)
        assert info["iterations"] == k
        assert np.abs(x - want).max() < 1e-8 * np.abs(want).max(), k


def test_first_iterates_are_minres():
    mo, psi, amg, b = system(33, 0)
    for k in (1, 2, 5, 10):
        a, _, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k)
        c, _, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k, reorth=64)
        assert np.abs(a - c).max() < 1e-12 * np.abs(a).max(), k


@pytest.fixture(scope="module")
def sys65():
    return system(65, 0)


def test_fewer_iterations_and_the_same_solution(sys65):
    mo, psi, amg, b = sys65
    xp, ip, hp = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000)
    xr, ir, hr = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000, reorth=400)
    assert ip["converged"] and ir["converged"]
    assert ir["iterations"] < 0.8 * ip["iterations"]
    assert ir["res_true"] < 1e-9
    assert np.abs(xr - xp).max() < 1e-7 * np.abs(xp).max()
    # the preconditioned residual estimate never increases (a minimisation
    # over nested spaces)
    assert np.all(np.diff(hr) <= 1e-14)


def test_robust_to_a_non_self_adjoint_preconditioner(sys65):
    """A linear non-self-adjoint perturbation of relative size 1e-7 (the
    rounding of an FP32 V-cycle): MINRES's three-term recurrence takes many
    more iterations, the reorthogonalised form about as many as without it."""
    mo, psi, amg, b = sys65
    J = lambda x: mo.jac(psi, x)
    M = lambda r: amg.precond(mo, r)
    d = np.random.default_rng(1).uniform(-1, 1, mo.n)
    Mp = lambda r: (lambda z: z + 1e-7 * np.roll(z, 1) * d)(M(r))
    counts = {}
    for name, f in (("exact", M), ("perturbed", Mp)):
        for reorth in (0, 400):
            x, info, _ = oracle.minres_generic(mo.vol, J, b, minv=f, rtol=1e-10, max_iter=3000, reorth=reorth)
            r = b - J(x)
            assert info["converged"]
            assert np.sqrt(mo.inner(r, r) / mo.inner(b, b)) < 1e-8
            counts[name, reorth] = info["iterations"]
    assert counts["perturbed", 0] > 1.3 * counts["exact", 0]
    assert abs(counts["perturbed", 400] - counts["exact", 400]) <= 2


def test_restart_and_deflation(sys65):
    mo, psi, amg, b = sys65
    # the first Newton system (near-definite): a basis of 8 restarts twice or more
    mo1 = oracle.Mesh(2, (33, 33), (10., 10.), mu=1.0)
    psi0 = inputs.random_phase_state(mo1.n, seed=0)
    amg0 = oracle.Amg.for_state(mo1, psi0, max_coarse=16)
    b0 = -mo1.gl(psi0)
    xp, ip, _ = oracle.minres(mo1, psi0, b0, amg=amg0, rtol=1e-10, max_iter=500)
    xr, ir, _ = oracle.minres(mo1, psi0, b0, amg=amg0, rtol=1e-10, max_iter=500, reorth=8)
    assert ip["iterations"] > 16 and ir["converged"] and ir["res_true"] < 1e-9
    assert np.abs(xr - xp).max() < 1e-8 * np.abs(xp).max()
    # deflated: the solution orthogonal to i psi, fewer iterations than the
    # deflated MINRES
    xd, idf, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000, deflate=True)
    xq, iq, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000, deflate=True, reorth=400)
    assert idf["converged"] and iq["converged"] and iq["res_true"] < 1e-9
    assert abs(mo.inner(1j * psi, xq)) < 1e-10 * np.sqrt(mo.inner(xq, xq) * mo.inner(psi, psi))
    assert iq["iterations"] < idf["iterations"]
    assert np.abs(xq - xd).max() < 1e-7 * np.abs(xd).max()
