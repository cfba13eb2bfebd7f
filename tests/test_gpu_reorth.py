"""MINRES with the Krylov basis stored and reorthogonalised (Krylov option
`reorth`; Sec. 4, the remedy the paper names for the loss of orthogonality)
against the oracle's, through the C-ABI: fixed-k iterates within 1e-12 on
grids (2D, 3D, ragged) and a simplicial mesh, plain and deflated, with and
without a preconditioner; converged counts within 1 of the oracle's and the
solution within 1e-10 of the oracle's iterate after the same count; a small
basis that restarts; Newton; the FP32 V-cycle (with a BF16 copy of Z and
an FP32 copy of V for the reorthogonalisation: iterates within 1e-4, the
minimised residual norm within 1e-6), whose count stays
that of the FP64 one (where plain MINRES needs about twice as many); the graph replay
(poll interval) bitwise neutral; batches bitwise equal to single solves; and
the option errors."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs, meshes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("2d-33x33", lambda: ((2, (33, 33), (10.0, 10.0)), dict(mu=1.0))),
    ("2d-37x23", lambda: ((2, (37, 23), (6.0, 4.0)), dict(mu=1.1))),
    ("3d-9^3", lambda: ((3, (9, 9, 9), (5.0, 5.0, 5.0)), dict(mu=0.6, bdir=tuple(np.ones(3) / np.sqrt(3.0))))),
    ("disc-9", None),
]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def glnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5125_amd import glnk as g
    g.lib()
    return g


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def pair(glnk, name):
    """(GPU mesh, oracle mesh, psi, b): the second Newton system of the case
    from a random-phase start (the oracle's first step)."""
    case = dict(CASES)[name]
    if case is None:
        xy, tri = meshes.disc(9)
        mg, mo = glnk.Mesh.simplicial(xy, tri, mu=0.8), oracle.Mesh.simplices(xy, tri, mu=0.8)
    else:
        (dim, N, side), kw = case()
        bdir = kw.get("bdir", (0.0, 0.0, 1.0))
        mg = glnk.Mesh(dim, N, side, mu=kw["mu"], b_dir=bdir)
        mo = oracle.Mesh(dim, N, side, mu=kw["mu"], bdir=bdir)
    psi0 = inputs.random_phase_state(mo.n, seed=7)
    psi, _ = oracle.newton(mo, psi0, fixed_steps=1, krylov_rtol=1e-10, krylov_max_iter=2000, max_coarse=16)
    return mg, mo, psi, -mo.gl(psi)


@pytest.mark.parametrize("deflate", [False, True], ids=["plain", "deflated"])
@pytest.mark.parametrize("precond", [True, False], ids=["R1", "none"])
@pytest.mark.parametrize("name", IDS)
def test_reorth_iterates(glnk, name, precond, deflate):
    mg, mo, psi, b = pair(glnk, name)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16) if precond else None
    pre = glnk.Precond(mg, dev(psi), max_coarse=16) if precond else None
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    for k in (1, 2, 5, 20, 60):
        xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k, deflate=deflate, reorth=200)
        rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=0.0, max_iter=k, poll_every=4,
                                        deflate=deflate, reorth=200, raise_on_fail=False)
        assert ig["iterations"] == io["iterations"] == k
        assert relerr(host(x), xo) < 1e-12, (k, relerr(host(x), xo))


@pytest.mark.parametrize("name", IDS)
def test_reorth_converged(glnk, name):
    """Converged solves: counts within 1 of the oracle's, the solution within
    1e-10 of the oracle's iterate after the GPU's count, fewer iterations than
    plain MINRES."""
    mg, mo, psi, b = pair(glnk, name)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000, reorth=500)
    rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=2000, reorth=500)
    assert rc == 0 and io["converged"] and ig["converged"]
    assert abs(ig["iterations"] - io["iterations"]) <= 1
    assert ig["res_true"] < 1e-9
    xk, _, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=ig["iterations"], reorth=500)
    assert relerr(host(x), xk) < 1e-10
    rc, ip = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=2000)
    assert ig["iterations"] <= ip["iterations"]


def test_restart_small_basis(glnk):
    """A basis of 6 vectors on the first (near-definite) Newton system
    restarts several times; every restart matches the oracle's."""
    mg = glnk.Mesh(2, (33, 33), (10.0, 10.0), mu=1.0)
    mo = oracle.Mesh(2, (33, 33), (10.0, 10.0), mu=1.0)
    psi = inputs.random_phase_state(mo.n, seed=7)
    b = -mo.gl(psi)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    for k in (5, 6, 7, 13, 20):
        xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k, reorth=6)
        rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=0.0, max_iter=k, reorth=6,
                                        raise_on_fail=False)
        assert ig["iterations"] == k
        assert relerr(host(x), xo) < 1e-11, k
    xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=500, reorth=6)
    rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=500, reorth=6)
    assert rc == 0 and abs(ig["iterations"] - io["iterations"]) <= 1 and ig["res_true"] < 1e-9


def test_newton_with_reorth(glnk):
    mg = glnk.Mesh(2, (33, 33), (10.0, 10.0), mu=1.0)
    mo = oracle.Mesh(2, (33, 33), (10.0, 10.0), mu=1.0)
    psi0 = inputs.random_phase_state(mo.n, seed=7)
    po, io = oracle.newton(mo, psi0, fixed_steps=4, krylov_rtol=1e-10, krylov_max_iter=2000, max_coarse=16,
                           reorth=300)
    psi = dev(psi0)
    rc, ig = glnk.gl_newton_solve(mg, psi, fixed_steps=4, krylov_rtol=1e-10, krylov_max_iter=2000, max_coarse=16,
                                  reorth=300, raise_on_fail=False)
    # the first system is the same on both sides; the later ones differ by
    # the rounding of the two trajectories (their counts stay close)
    assert abs(ig["krylov_iters"][0] - io["krylov_iters"][0]) <= 1
    assert all(abs(a - c) <= 3 for a, c in zip(ig["krylov_iters"], io["krylov_iters"]))
    assert relerr(host(psi), po) < 1e-8


def test_fp32_vcycle_keeps_the_fp64_count(glnk):
    """With the FP32 V-cycle plain MINRES needs far more iterations than with
    the FP64 one (the rounding breaks the preconditioner's self-adjointness);
    the reorthogonalised solve needs about as many as the FP64 one and meets
    the tolerance on the true residual."""
    mg, mo, psi, b = pair(glnk, "2d-33x33")
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    counts = {}
    for prec in (glnk.GL_FP64, glnk.GL_FP32):
        pre = glnk.Precond(mg, dev(psi), precision=prec, max_coarse=16)
        for reorth in (0, 500):
            rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=3000,
                                              reorth=reorth)
            assert rc == 0 and info["res_true"] < 1e-9
            counts[prec, reorth] = info["iterations"]
    assert abs(counts[glnk.GL_FP32, 500] - counts[glnk.GL_FP64, 500]) <= 2
    assert counts[glnk.GL_FP64, 500] < counts[glnk.GL_FP64, 0]
    # the FP32 mode (FP32 V-cycle; the reorthogonalisation's coefficients
    # from a BF16 copy of Z, its update from an FP32 copy of V) against the
    # oracle's FP64 iterates.  The BF16 rounding (unit roundoff 2^-9) falls
    # on the correction coefficients only, which are of the size of the loss
    # of orthogonality (the Lanczos coefficients are FP64), so the basis
    # stays orthogonal to about 2^-9 of that: the iterate moves within the
    # Krylov space by about 1e-5 relative (bound 1e-4).  The minimised norm
    # moves only to second order, since the minimiser's residual is
    # M-orthogonal to J K_k: ||r||_M^2 = ||r*||_M^2 + ||J e||_M^2 for an
    # iterate x* + e; bound 1e-6 relative (the FP32 V-cycle's own rounding
    # moves it by about 1e-9).
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    pre = glnk.Precond(mg, dev(psi), precision=glnk.GL_FP32, max_coarse=16)

    def res_m(xv):
        r = b - mo.jac(psi, xv)
        return np.sqrt(mo.inner(r, amg.precond(mo, r)))

    for k in (5, 20, 60):
        xo, _, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k, reorth=500)
        rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=0.0, max_iter=k, reorth=500,
                                          raise_on_fail=False)
        assert relerr(host(x), xo) < 1e-4, k
        assert abs(res_m(host(x)) / res_m(xo) - 1.0) < 1e-6, k


def test_poll_interval_is_bitwise_neutral(glnk):
    mg, mo, psi, b = pair(glnk, "2d-37x23")
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    outs = []
    for poll in (1, 3, 16):
        x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
        rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=2000, poll_every=poll,
                                          reorth=400)
        outs.append((info["iterations"], host(x)))
    assert all(o[0] == outs[0][0] and np.array_equal(o[1], outs[0][1]) for o in outs)


def test_reorth_errors(glnk):
    mg = glnk.Mesh(2, (9, 9), (5.0, 5.0), mu=0.5)
    psi = torch.ones(mg.n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(psi)
    pre = glnk.Precond(mg, psi, precision=glnk.GL_FP32)
    with pytest.raises(RuntimeError, match="invalid Krylov options"):
        glnk.gl_jacobian_solve(mg, psi, pre, psi, x, inner_rtol=1e-5, reorth=50)
    with pytest.raises(RuntimeError, match="invalid Krylov options"):
        glnk.gl_jacobian_solve(mg, psi, pre, psi, x, relax_rtol=1e-4, reorth=50)
    with pytest.raises(RuntimeError, match="invalid Krylov options"):
        glnk.gl_jacobian_solve(mg, psi, pre, psi, x, reorth=-1)


@pytest.mark.parametrize("deflate", [False, True], ids=["plain", "deflated"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_batch_equals_single(glnk, fp32, deflate):
    """Reorthogonalised Newton in a batch of three shapes (2D grid, 3D grid,
    disc) bitwise equal to the single solves."""
    prec = glnk.GL_FP32 if fp32 else glnk.GL_FP64
    ms, p0 = [], []
    for name in ("2d-33x33", "3d-9^3", "disc-9"):
        mg, mo, psi, b = pair(glnk, name)
        ms.append(mg)
        p0.append(inputs.random_phase_state(mo.n, seed=9))
    kw = dict(fixed_steps=3, krylov_rtol=1e-10, krylov_max_iter=2000, max_coarse=16, precision=prec,
              deflate=deflate, reorth=300)
    singles = []
    for m, p in zip(ms, p0):
        psi = dev(p)
        rc, info = glnk.gl_newton_solve(m, psi, raise_on_fail=False, **kw)
        singles.append((info, host(psi)))
    batch = glnk.Batch(ms)
    psis = [dev(p) for p in p0]
    rc, infos = batch.newton_solve(psis, raise_on_fail=False, **kw)
    for (i1, ps1), i2, psi in zip(singles, infos, psis):
        assert i1["res"] == i2["res"] and i1["krylov_iters"] == i2["krylov_iters"]
        assert np.array_equal(ps1, host(psi))
    assert sum(infos[0]["krylov_iters"]) > 0


def test_unattainable_tolerance_stops(glnk):
    """Asked for a tolerance below the attainable accuracy, the
    reorthogonalised solve stops once a restart no longer halves the true
    residual (NOT_CONVERGED), far below its iteration limit, with the
    accuracy the system allows."""
    mg, mo, psi, b = pair(glnk, "2d-33x33")
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-17, max_iter=5000, reorth=500,
                                      raise_on_fail=False)
    assert rc == 4 and not info["converged"]
    assert info["iterations"] < 1000
    assert info["res_true"] < 1e-12
