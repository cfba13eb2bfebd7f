"""Pseudo-arclength continuation on the GPU against the oracle's (Sec. 4,
numerical parameter continuation), and the entry points it rests on:
gl_residual_dmu (d GL / d mu), gl_inner and gl_axpby.  The traced branch of
the 33 x 33, side-8 square passes the Meissner branch's fold near
mu = 0.707: every point's mu within 1e-8 of the oracle's, the same Newton
steps and step halvings, states within 1e-10 after phase alignment, and the
deflated Krylov counts within 1 wherever the oracle's own counts do not move
when its start is rotated by a global phase (the same path rounded
differently).  They do move at the first point past the fold, where an
eigenvalue of the restricted Jacobian has just crossed zero: there the
oracle alone takes (45, 46), (45, 43) or (46, 46) MINRES iterations for the
same corrector step."""
import numpy as np
import pytest

import oracle
from oracle import arclength as oal
from paper_1204_5125_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("case", [(2, (33, 33), (5.0, 5.0), 0.8, (0, 0, 1)),
                                  (2, (37, 23), (6.0, 4.0), 1.1, (0, 0, 1)),
                                  (3, (9, 9, 9), (5.0, 5.0, 5.0), 0.6, (1, 1, 1)),
                                  (3, (7, 5, 11), (3.0, 2.0, 4.0), 0.9, (0.3, -0.5, 1.0))],
                         ids=["2d-33", "2d-37x23", "3d-9", "3d-7x5x11"])
def test_parameter_derivative_inner_axpby(glnk, case):
    dim, N, side, mu, b = case
    b = np.asarray(b, float) / np.linalg.norm(b)
    mg = glnk.Mesh(dim, N, side, mu=mu, b_dir=b)
    mo = oracle.Mesh(dim, N, side, mu=mu, bdir=b)
    psi = inputs.random_complex(mo.n, seed=61)
    phi = inputs.random_complex(mo.n, seed=62)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    glnk.gl_residual_dmu(mg, dev(psi), out)
    ref = oal.gl_dmu(mo, psi, b)
    assert np.abs(host(out) - ref).max() < 1e-12 * np.abs(ref).max()
    assert glnk.gl_inner(mg, dev(psi), dev(phi)) == pytest.approx(mo.inner(psi, phi), rel=1e-12)
    x = dev(psi)
    glnk.gl_axpby(mg, 0.5, x, -2.0, dev(phi), x)
    assert np.abs(host(x) - (0.5 * psi - 2.0 * phi)).max() < 1e-15 * np.abs(psi).max() * 4


def test_parameter_derivative_needs_a_field_parameter(glnk):
    mg = glnk.Mesh(2, (9, 9), (4.0, 4.0), a_matrix=np.eye(3) * 0.1)
    x = torch.ones(81, dtype=torch.complex128, device="cuda")
    with pytest.raises(glnk.GlnkError) as e:
        glnk.gl_residual_dmu(mg, x, torch.empty_like(x))
    assert e.value.code == 8


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_arclength_passes_the_fold_like_the_oracle(glnk, precision):
    from paper_1204_5125_amd import continuation as gc
    N, L, B = (33, 33), (8.0, 8.0), (0, 0, 1)
    ro, so = oal.arclength(2, N, L, B, np.ones(33 * 33, complex), 0.0, 0.1, 19)
    rr, _ = oal.arclength(2, N, L, B, np.exp(0.3j) * np.ones(33 * 33, complex), 0.0, 0.1, 19)
    mg = glnk.Mesh(2, N, L, mu=0.0)
    rg, sg = gc.arclength_path(mg, torch.ones(33 * 33, dtype=torch.complex128, device="cuda"), 0.0, 0.1, 19,
                               precision=precision)
    assert len(rg) == len(ro) and all(r["converged"] for r in rg)
    mus = np.array([r["mu"] for r in rg])
    k = int(np.argmax(mus))
    assert 0.70 < mus[k] < 0.72 and k < len(mus) - 3
    compared = 0
    for a, b, c in zip(rg[1:], ro[1:], rr[1:]):
        assert a["mu"] == pytest.approx(b["mu"], abs=1e-8)
        assert a["ds"] == b["ds"] and a["newton_steps"] == b["newton_steps"], (a, b)
        if precision == 0 and b["krylov_iters"] == c["krylov_iters"]:
            compared += 1
            for (x1, y1), (x2, y2) in zip(a["krylov_iters"], b["krylov_iters"]):
                assert abs(x1 - x2) <= 1 and abs(y1 - y2) <= 1, (a["krylov_iters"], b["krylov_iters"])
    if precision == 0:
        assert compared >= len(ro) - 4
    for (mg_, pg), (mo_, po) in zip(sg, so):
        ps = host(pg)
        chi = np.angle(np.vdot(ps, po))
        e = np.abs(ps * np.exp(1j * chi) - po).max() / max(np.abs(po).max(), 1.0)
        assert e < 1e-10, (mo_, e)
