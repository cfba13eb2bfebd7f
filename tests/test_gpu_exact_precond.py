"""R_inf = H^-1 D (eq. prec1; gl_amg_opts.cycles = 0: conjugate gradients
with the V-cycle as preconditioner, a step count fixed at setup) against
the oracle's sparse direct solve, and MINRES preconditioned by it against
the oracle's MINRES with the exact preconditioner."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [(2, (33, 33), (5.0, 5.0), 0.8, (0, 0, 1)), (2, (37, 23), (6.0, 4.0), 1.1, (0, 0, 1)),
         (3, (9, 9, 9), (5.0, 5.0, 5.0), 0.6, (1, 1, 1)), (2, (129, 129), (10.0, 10.0), 1.0, (0, 0, 1))]
IDS = ["2d-33", "2d-37x23", "3d-9", "2d-129"]


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


def pair(glnk, case):
    dim, N, side, mu, b = case
    b = np.asarray(b, float) / np.linalg.norm(b)
    return glnk.Mesh(dim, N, side, mu=mu, b_dir=b), oracle.Mesh(dim, N, side, mu=mu, bdir=b)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_exact_preconditioner_apply(glnk, case):
    mg, mo = pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=71)
    r = inputs.random_complex(mo.n, seed=72)
    pre = glnk.Precond(mg, dev(psi), cycles=0)
    m = pre.inner_steps()
    assert 1 <= m <= 64
    z = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    pre.apply(dev(r), z)
    e = relerr(host(z), oracle.precond_exact(mo, psi, r))
    assert e < 1e-10, (m, e)
    # a later setup recalibrates for the new state; R_k handles stay R_k
    psi2 = inputs.random_phase_state(mo.n, seed=73)
    pre.update(dev(psi2))
    pre.apply(dev(r), z)
    assert relerr(host(z), oracle.precond_exact(mo, psi2, r)) < 1e-10
    pre.update(dev(psi2), cycles=2)
    assert pre.inner_steps() == 2


@pytest.mark.parametrize("case", CASES[:3], ids=IDS[:3])
def test_minres_with_exact_preconditioner(glnk, case):
    """Iteration counts within 1 of the oracle's MINRES with the exact
    preconditioner; the solution within 1e-10 of the oracle's iterate after
    the same count; no more iterations than R_1 (as many on the 9^3 grid,
    whose two-level hierarchy makes R_1 nearly exact)."""
    mg, mo = pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=74)
    b = inputs.random_complex(mo.n, seed=75)
    xo, io, _ = oracle.minres_exact_precond(mo, psi, b, rtol=1e-10, max_iter=1000)
    pre = glnk.Precond(mg, dev(psi), cycles=0)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=1000)
    assert rc == 0 and io["converged"]
    assert abs(ig["iterations"] - io["iterations"]) <= 1
    xk = xo if ig["iterations"] == io["iterations"] else \
        oracle.minres_exact_precond(mo, psi, b, rtol=0.0, max_iter=ig["iterations"])[0]
    e = relerr(host(x), xk)
    assert e < 1e-10, e
    p1 = glnk.Precond(mg, dev(psi))
    rc, i1 = glnk.gl_jacobian_solve(mg, dev(psi), p1, dev(b), x, rtol=1e-10, max_iter=1000)
    assert ig["iterations"] <= i1["iterations"]


def test_exact_preconditioner_needs_fp64(glnk):
    mg, mo = pair(glnk, CASES[0])
    with pytest.raises(glnk.GlnkError):
        glnk.Precond(mg, torch.ones(mo.n, dtype=torch.complex128, device="cuda"), cycles=0,
                     precision=glnk.GL_FP32)
