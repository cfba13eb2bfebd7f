"""GPU path vs the FP64 oracle, element by element, through the C-ABI.

Sizes: several tiles of 256 nodes with ragged tails, 2D and 3D, plus the
33 x 33 config-0 grid.  Tolerances: integer and index arrays bit-exact;
FP64 operators within 1e-12 and V-cycles within 1e-11 relative; MINRES
iterates after the same number of iterations within 1e-12 (a few) or 1e-10
(a converged solve, compared with the oracle run to the GPU's count);
Krylov counts within 1; Newton states within 1e-10 of max(|psi|, 1) after
phase alignment;
FP32 preconditioner outputs within 1e-5 relative to the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # dim, N, side, mu, bdir
    (2, (33, 33), (5.0, 5.0), 0.8, (0, 0, 1)),
    (2, (37, 23), (6.0, 4.0), 1.1, (0, 0, 1)),
    (3, (9, 9, 9), (5.0, 5.0, 5.0), 0.6, (1, 1, 1)),
    (3, (7, 5, 11), (3.0, 2.0, 4.0), 0.9, (0.3, -0.5, 1.0)),
    # even x-widths: every red-black pair of the level-0 layout holds two nodes
    (2, (24, 17), (5.0, 4.0), 0.9, (0, 0, 1)),
    (3, (8, 6, 5), (4.0, 3.0, 2.5), 0.7, (0.2, 0.4, 1.0)),
]
IDS = ["2d-33x33", "2d-37x23", "3d-9^3", "3d-7x5x11", "2d-24x17", "3d-8x6x5"]


@pytest.fixture(scope="module")
def glnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5125_amd import glnk as g
    g.lib()
    return g


def unit(b):
    b = np.asarray(b, float)
    return b / np.linalg.norm(b)


def make_pair(glnk, case):
    dim, N, side, mu, bdir = case
    b = unit(bdir)
    m_gpu = glnk.Mesh(dim, N, side, mu=mu, b_dir=b)
    m_orc = oracle.Mesh(dim, N, side, mu=mu, bdir=b)
    return m_gpu, m_orc


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_link_variables(glnk, case):
    mg, mo = make_pair(glnk, case)
    dim, N = case[0], case[1]
    off = 0
    for a in range(dim):
        u = mg.export_links(a)
        idx = np.stack(np.unravel_index(np.arange(mo.n), N[::-1])[::-1], axis=1)
        lower = np.nonzero(idx[:, a] < N[a] - 1)[0]
        ne_a = lower.size
        assert np.array_equal(mo.ek[off:off + ne_a], lower)
        assert np.abs(u[lower] - mo.U[off:off + ne_a]).max() < 1e-14
        assert np.all(u[idx[:, a] == N[a] - 1] == 0)
        off += ne_a


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_residual_and_jacobian(glnk, case):
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_complex(mo.n, seed=1) * 0.8
    phi = inputs.random_complex(mo.n, seed=2)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    nrm = glnk.gl_residual(mg, dev(psi), out)
    ref = mo.gl(psi)
    assert relerr(host(out), ref) < 1e-12
    assert nrm == pytest.approx(mo.norm(ref), rel=1e-12)
    jo = torch.empty_like(out)
    glnk.gl_jacobian_apply(mg, dev(psi), dev(phi), jo)
    assert relerr(host(jo), mo.jac(psi, phi)) < 1e-12


def test_residual_norm_only_and_errors(glnk):
    mg, mo = make_pair(glnk, CASES[0])
    psi = dev(inputs.random_phase_state(mo.n, seed=0))
    n1 = glnk.gl_residual(mg, psi, None)
    assert n1 == pytest.approx(mo.norm(mo.gl(host(psi))), rel=1e-12)
    with pytest.raises(glnk.GlnkError) as e:
        glnk.gl_residual(mg, psi, psi)
    assert e.value.code == 1
    with pytest.raises(glnk.GlnkError):
        glnk.Mesh(4, (3, 3, 3), (1.0, 1.0, 1.0))
    with pytest.raises(glnk.GlnkError):
        glnk.Mesh(2, (1, 5), (1.0, 1.0))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_hierarchy_bit_exact(glnk, case):
    """Aggregates, roots, colours and every sparsity pattern equal the oracle's
    bit for bit; values within 1e-12."""
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=3)
    pre = glnk.Precond(mg, dev(psi))
    amg = oracle.Amg.for_state(mo, psi)
    info = pre.info()
    assert info["nlev"] == amg.nlev
    for l, L in enumerate(amg.levels):
        assert info["sizes"][l] == L["n"]
        assert np.array_equal(pre.export(l, "color"), L["color"])
        assert np.array_equal(pre.export(l, "A_rp"), L["A"].indptr)
        assert np.array_equal(pre.export(l, "A_ci"), L["A"].indices)
        assert relerr(pre.export(l, "A_v"), L["A"].data) < 1e-12
        if l < amg.nlev - 1:
            assert np.array_equal(pre.export(l, "agg"), L["agg"])
            assert np.array_equal(pre.export(l, "root"), L["root"])
            for M in ("P", "R"):
                assert np.array_equal(pre.export(l, M + "_rp"), L[M].indptr)
                assert np.array_equal(pre.export(l, M + "_ci"), L[M].indices)
                assert relerr(pre.export(l, M + "_v"), L[M].data) < 1e-12


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_vcycle(glnk, case):
    """R_1 r = AMG_1(H, D r): FP64 within 1e-11, FP32 within 1e-5."""
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=4)
    r = inputs.random_complex(mo.n, seed=5)
    amg = oracle.Amg.for_state(mo, psi)
    ref = amg.precond(mo, r)
    z = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    pre = glnk.Precond(mg, dev(psi))
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-11
    pre.update(dev(psi), precision=glnk.GL_FP32)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-5
    # level 0 in FP32, coarser levels in FP64
    pre.update(dev(psi), precision=glnk.GL_MIXED)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-5
    # k = 3 cycles
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=3)
    pre.apply(dev(r), z)
    assert relerr(host(z), amg.precond(mo, r, cycles=3)) < 1e-11
    # the cycle below level 1 as an explicit matrix (where the hierarchy has
    # a level between level 1 and the coarsest), FP64, FP32 and k = 3 cycles
    glnk.gl_precond_set_tiles(pre, 0, 64, 8192)
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=1)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-11
    pre.update(dev(psi), precision=glnk.GL_FP32)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-5
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=3)
    pre.apply(dev(r), z)
    assert relerr(host(z), amg.precond(mo, r, cycles=3)) < 1e-11


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("precond", [True, False], ids=["R1", "none"])
def test_minres_iterates(glnk, case, precond):
    """Fixed-k iterates equal the oracle's (1e-12); to rtol 1e-10 the
    iteration count agrees within 1 and the solution equals the oracle's
    iterate after the same number of iterations within 1e-10."""
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=6)
    b = inputs.random_complex(mo.n, seed=7)
    amg = oracle.Amg.for_state(mo, psi) if precond else None
    pre = glnk.Precond(mg, dev(psi)) if precond else None
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    for k in (1, 2, 5):
        xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k)
        rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=0.0, max_iter=k, poll_every=2)
        assert ig["iterations"] == k == io["iterations"]
        e = relerr(host(x), xo)
        assert e < 1e-12, (k, e)
        assert ig["res_est"] == pytest.approx(io["eta"] / io["eta0"], rel=1e-10)
    xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000)
    rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=2000)
    assert io["converged"] and ig["converged"]
    assert abs(ig["iterations"] - io["iterations"]) <= 1
    # the same iterate: the oracle run to the GPU's count
    xk, ik, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=ig["iterations"])
    e = relerr(host(x), xk)
    assert e < 1e-10, e
    assert ig["res_true"] < 1e-9


def test_minres_not_converged_and_zero_rhs(glnk):
    mg, mo = make_pair(glnk, CASES[0])
    psi = dev(inputs.random_phase_state(mo.n, seed=8))
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    rc, info = glnk.gl_jacobian_solve(mg, psi, None, dev(inputs.random_complex(mo.n, 9)), x,
                                      rtol=1e-14, max_iter=3)
    assert rc == 4 and info["iterations"] == 3 and not info["converged"]
    rc, info = glnk.gl_jacobian_solve(mg, psi, None, torch.zeros_like(x), x)
    assert rc == 0 and info["iterations"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_singular_preconditioner(glnk):
    mg = glnk.Mesh(2, (9, 9), (5.0, 5.0), mu=0.0)
    with pytest.raises(glnk.GlnkError) as e:
        glnk.Precond(mg, torch.zeros(81, dtype=torch.complex128, device="cuda"))
    assert e.value.code == 7


def test_newton_config0(glnk):
    """Config 0: 33 x 33, side 5, mu 0.8, psi0 = 0.9 exp(i theta); Newton +
    MINRES(R_1, 1e-10) to ||GL||_D < 1e-10.  Step-by-step residual history and
    Krylov counts follow the oracle's trajectory."""
    case = CASES[0]
    mg, mo = make_pair(glnk, case)
    psi0 = inputs.random_phase_state(mo.n, seed=0)
    pso, io = oracle.newton(mo, psi0, tol=1e-10, max_steps=50, krylov_rtol=1e-10)
    psi = dev(psi0)
    rc, ig = glnk.gl_newton_solve(mg, psi, tol=1e-10, max_steps=50, krylov_rtol=1e-10)
    assert rc == 0 and ig["converged"] and io["converged"]
    assert ig["steps"] == io["steps"]
    for a, b in zip(ig["krylov_iters"], io["krylov_iters"]):
        assert abs(a - b) <= 1
    for a, b in list(zip(ig["res"], io["res"]))[:-1]:
        assert a == pytest.approx(b, rel=1e-6)
    ps = host(psi)
    chi = np.angle(np.vdot(ps, pso)) if np.abs(pso).max() > 1e-8 else 0.0
    # in units of max(|psi|, 1): GL solutions have |psi| <= 1, and this start
    # converges to the normal state psi = 0
    e = np.abs(ps * np.exp(1j * chi) - pso).max() / max(np.abs(pso).max(), 1.0)
    assert e < 1e-10, e
    # FP32 preconditioner reaches the same tolerance
    psi = dev(psi0)
    rc, i32 = glnk.gl_newton_solve(mg, psi, tol=1e-10, max_steps=50, precision=glnk.GL_FP32)
    assert rc == 0 and i32["converged"]


@pytest.mark.parametrize("case", [CASES[0], CASES[2]], ids=["2d-33x33", "3d-9^3"])
def test_fp32_preconditioned_solve_reaches_fp64_accuracy(glnk, case):
    """FP32 V-cycle under FP64 refinement: the solution matches the FP64
    oracle solve to the 1e-10 level and the true residual is below 1e-9."""
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=10)
    b = inputs.random_complex(mo.n, seed=11)
    amg = oracle.Amg.for_state(mo, psi)
    xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-13, max_iter=2000)
    pre = glnk.Precond(mg, dev(psi), precision=glnk.GL_FP32)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")

    def check(info):
        # the solution's residual in the oracle's Jacobian, and its distance
        # from the oracle's 1e-13 solve
        assert info["converged"]
        xs = host(x)
        rr = mo.norm(mo.jac(psi, xs) - b) / mo.norm(b)
        assert rr < 1e-10 and info["res_true"] < 1e-10, (rr, info)
        e = relerr(xs, xo)
        assert e < 1e-9, e

    rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-11, max_iter=2000)
    assert rc == 0
    check(info)
    # one recurrence: FP64 V-cycle down to 1e-3, the reduced precision after
    for prec in (glnk.GL_FP32, glnk.GL_MIXED):
        pre.update(dev(psi), precision=prec)
        rc, info = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-11, max_iter=2000,
                                          relax_rtol=1e-3)
        assert rc == 0
        check(info)


def test_repeated_solves_bitwise_identical(glnk):
    """Deterministic reductions and graph replay: two solves give identical bits."""
    mg, mo = make_pair(glnk, CASES[1])
    psi = dev(inputs.random_phase_state(mo.n, seed=12))
    b = dev(inputs.random_complex(mo.n, seed=13))
    pre = glnk.Precond(mg, psi)
    x1 = torch.empty_like(b)
    x2 = torch.empty_like(b)
    rc1, i1 = glnk.gl_jacobian_solve(mg, psi, pre, b, x1, rtol=1e-10)
    rc2, i2 = glnk.gl_jacobian_solve(mg, psi, pre, b, x2, rtol=1e-10)
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("max_coarse", [64, 512])
def test_vcycle_and_solve_deeper_hierarchy(glnk, max_coarse):
    """129 x 129 grid: a coarse level above 512 rows (multi-kernel sweeps), the
    single-work-group bottom levels and the dense coarsest solve, FP64 and FP32;
    then MINRES counts and solutions against the oracle."""
    mg = glnk.Mesh(2, (129, 129), (10.0, 10.0), mu=1.0)
    mo = oracle.Mesh(2, (129, 129), (10.0, 10.0), mu=1.0)
    psi = inputs.random_phase_state(mo.n, seed=14)
    r = inputs.random_complex(mo.n, seed=15)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=max_coarse)
    pre = glnk.Precond(mg, dev(psi), max_coarse=max_coarse)
    assert pre.info()["sizes"] == [L["n"] for L in amg.levels]
    z = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    pre.apply(dev(r), z)
    ref = amg.precond(mo, r)
    assert relerr(host(z), ref) < 1e-11
    pre.update(dev(psi), precision=glnk.GL_FP32)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-5
    # every split between multi-kernel levels, the single-work-group bottom
    # and a sub-cycle applied as an explicit matrix (none, the level above the
    # coarsest, or every level >= 1)
    sizes = pre.info()["sizes"]
    for dense in (0, 512, 4096):
        for rows in (512, 4096, 65536):
            glnk.gl_precond_set_tiles(pre, 0, rows, dense)
            assert glnk.gl_precond_get_tiles(pre) == {"lane_shift": 0, "bottom_rows": rows, "dense_rows": dense,
                                                      "l0_tiled": 0}
            for prec, tol in ((glnk.GL_FP64, 1e-11), (glnk.GL_FP32, 1e-5), (glnk.GL_MIXED, 1e-5)):
                pre.update(dev(psi), precision=prec)
                pre.apply(dev(r), z)
                assert relerr(host(z), ref) < tol, (dense, rows, prec, sizes)
    with pytest.raises(glnk.GlnkError):
        glnk.gl_precond_set_tiles(pre, 0, 0, 8193)
    # the explicit sub-cycle with the values of a later setup (graphs keep
    # its address), then MINRES through it against the oracle
    xo, io, _ = oracle.minres(mo, psi, r, amg=amg, rtol=1e-10, max_iter=3000)
    assert io["converged"]
    for tiles in ((0, 0, 4096), (0, 0)):
        glnk.gl_precond_set_tiles(pre, *tiles)
        pre.update(dev(psi), precision=glnk.GL_FP64)
        rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(r), z, rtol=1e-10, max_iter=3000)
        assert ig["converged"]
        assert abs(ig["iterations"] - io["iterations"]) <= 1
        xk = xo if ig["iterations"] == io["iterations"] else \
            oracle.minres(mo, psi, r, amg=amg, rtol=0.0, max_iter=ig["iterations"])[0]
        e = relerr(host(z), xk)
        assert e < 1e-10, (tiles, e)


def test_secant_predictor(glnk):
    from oracle import continuation as oc
    mg, mo = make_pair(glnk, CASES[1])
    a = inputs.random_complex(mo.n, seed=16)
    b = inputs.random_complex(mo.n, seed=17)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    glnk.gl_secant_predict(mg, dev(a), dev(b), 0.7, out)
    assert relerr(host(out), oc.secant_predict(mo, a, b, 0.7)) < 1e-13


def test_continuation_falls_back_to_secant(glnk):
    """A predicted start that Newton cannot correct (here a non-finite one,
    which Newton rejects at its first residual) is replaced by the secant
    start for that step: the path, its records and its final state equal the
    secant-only path's."""
    from paper_1204_5125_amd import continuation as gc
    mg = glnk.Mesh(2, (33, 33), (8.0, 8.0), mu=0.0)
    ones = torch.ones(33 * 33, dtype=torch.complex128, device="cuda")
    r0, p0 = gc.continuation(mg, ones, 0.0, 0.05, 4)
    calls = []

    def bad(psi, prev, mu_prev, mu, mu_next):
        calls.append(mu_next)
        return torch.full_like(psi, float("nan")) if len(calls) == 3 else None

    r1, p1 = gc.continuation(mg, ones, 0.0, 0.05, 4, predictor=bad)
    assert len(calls) == 4 and len(r1) == len(r0) == 5
    assert all(r["status"] == 0 for r in r1)
    assert r1[3]["predictor"] == "custom->secant" and r1[3]["failed_newton_steps"] == 0
    assert [r["predictor"] for r in r1[1:3] + r1[4:]] == [r["predictor"] for r in r0[1:3] + r0[4:]]
    assert [r["newton_steps"] for r in r1] == [r["newton_steps"] for r in r0]
    assert torch.equal(p0, p1)


def test_continuation_matches_oracle(glnk):
    """Natural continuation from psi = 1 at mu = 0 in steps of 0.05 on a 33 x 33
    grid of side 8: Newton steps per continuation step equal the oracle's, MINRES
    counts of each Newton step but the last within 1, final states equal up to
    a global phase (1e-10).  The last Newton step of a continuation step is
    not compared: its right-hand side GL(psi) is at the rounding level of psi,
    and the oracle's own count there moves by up to 15 when its start is only
    rotated by a global phase (test_oracle_continuation), while every earlier
    count stays put."""
    from oracle import continuation as oc
    from paper_1204_5125_amd import continuation as gc
    N, side = (33, 33), (8.0, 8.0)
    ro, pso = oc.continuation(2, N, side, (0, 0, 1), np.ones(33 * 33, complex), 0.0, 0.05, 6)
    mg = glnk.Mesh(2, N, side, mu=0.0)
    rg, psg = gc.continuation(mg, torch.ones(33 * 33, dtype=torch.complex128, device="cuda"), 0.0, 0.05, 6)
    assert len(rg) == len(ro)
    for a, b in zip(rg, ro):
        assert a["status"] == 0 and b["status"] == 0
        assert a["newton_steps"] == b["newton_steps"]
        for x, y in zip(a["krylov_iters"][:-1], b["krylov_iters"][:-1]):
            assert abs(x - y) <= 1, (a, b)
    ps = host(psg)
    chi = np.angle(np.vdot(ps, pso))
    e = np.abs(ps * np.exp(1j * chi) - pso).max() / max(np.abs(pso).max(), 1.0)
    assert e < 1e-10, e


def test_mesh_independent_iteration_counts(glnk):
    """Fig. 3 protocol in 2D (psi = 1, b = 1, x0 = 0, rtol 1e-11, R_1, mu = 1,
    side 10): the MINRES count stays flat as the grid is refined, and on the
    smallest grid it equals the oracle's within 1."""
    counts = []
    for n in (65, 129, 257):
        mg = glnk.Mesh(2, (n, n), (10.0, 10.0), mu=1.0)
        ones = torch.ones(mg.n, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(ones)
        pre = glnk.Precond(mg, ones, max_coarse=64)
        rc, info = glnk.gl_jacobian_solve(mg, ones, pre, ones, x, rtol=1e-11, max_iter=500)
        assert rc == 0 and info["res_true"] < 1e-9
        counts.append(info["iterations"])
        if n == 65:
            mo = oracle.Mesh(2, (n, n), (10.0, 10.0), mu=1.0)
            o1 = np.ones(mo.n, dtype=np.complex128)
            amg = oracle.Amg.for_state(mo, o1, max_coarse=64)
            _, io, _ = oracle.minres(mo, o1, o1, amg=amg, rtol=1e-11, max_iter=500)
            assert abs(io["iterations"] - info["iterations"]) <= 1
    assert max(counts) <= 1.25 * min(counts), counts


@pytest.mark.parametrize("grid", [((33, 33), (5.0, 5.0), 0.8), ((37, 23), (6.0, 4.0), 1.1),
                                  ((24, 17), (5.0, 4.0), 0.9), ((129, 129), (10.0, 10.0), 1.0),
                                  ((70, 45), (7.0, 4.5), 0.6), ((5, 3), (2.0, 1.0), 0.9)],
                         ids=["33x33", "37x23", "24x17", "129x129", "70x45", "5x3"])
def test_level0_tiles_bitwise(glnk, grid):
    """2D level 0 in two LDS-tiled kernels, each tile shape, against one
    dispatch per pass (the default): the V-cycle's output agrees to rounding (every node value is the
    same expression in the same order; the compiler may contract its
    multiply-adds differently in the two kernels), FP64 within 1e-13, FP32
    and mixed within 1e-6; k = 3 cycles (the accumulating output); tiles with
    ragged edges."""
    N, side, mu = grid
    mg = glnk.Mesh(2, N, side, mu=mu)
    n = N[0] * N[1]
    psi = dev(inputs.random_phase_state(n, seed=17))
    r = dev(inputs.random_complex(n, seed=18))
    pre = glnk.Precond(mg, psi, max_coarse=16)
    z1 = torch.empty_like(r)
    z2 = torch.empty_like(r)
    for prec, cycles in ((glnk.GL_FP64, 1), (glnk.GL_FP32, 1), (glnk.GL_MIXED, 1), (glnk.GL_FP64, 3)):
        pre.update(psi, precision=prec, cycles=cycles)
        glnk.gl_precond_set_tiles(pre, 0, 0, 0, 0)
        pre.apply(r, z2)
        for shape in (1, 2, 3):
            glnk.gl_precond_set_tiles(pre, 0, 0, 0, shape)
            pre.apply(r, z1)
            e = relerr(host(z1), host(z2))
            assert e < (1e-13 if prec == glnk.GL_FP64 else 1e-6), (prec, cycles, shape, e)
    # and MINRES through the tiled level 0 against the oracle (fixed count)
    mo = oracle.Mesh(2, N, side, mu=mu)
    hp = host(psi)
    amg = oracle.Amg.for_state(mo, hp, max_coarse=16)
    b = inputs.random_complex(n, seed=19)
    pre.update(psi, precision=glnk.GL_FP64, cycles=1)
    glnk.gl_precond_set_tiles(pre, 0, 0, 0, 1)
    xo, io, _ = oracle.minres(mo, hp, b, amg=amg, rtol=0.0, max_iter=5)
    rc, ig = glnk.gl_jacobian_solve(mg, psi, pre, dev(b), z1, rtol=0.0, max_iter=5, poll_every=2)
    assert relerr(host(z1), xo) < 1e-12


def test_level0_tiles_full_size(glnk):
    """The benchmark's 1025 x 1025 grid (4225 tiles of 16 x 16 nodes, a
    one-node ragged row and column of tiles for every shape): each tiled form
    against one dispatch per pass, FP64 within 1e-13 and FP32 within 1e-6."""
    N = (1025, 1025)
    mg = glnk.Mesh(2, N, (10.0, 10.0), mu=1.0)
    n = N[0] * N[1]
    psi = dev(inputs.random_phase_state(n, seed=21))
    r = dev(inputs.random_complex(n, seed=22))
    pre = glnk.Precond(mg, psi, max_coarse=512)
    z1 = torch.empty_like(r)
    z2 = torch.empty_like(r)
    for prec in (glnk.GL_FP64, glnk.GL_FP32):
        pre.update(psi, precision=prec)
        glnk.gl_precond_set_tiles(pre, 0, 64, 4096, 0)
        pre.apply(r, z2)
        ref = host(z2)
        for shape in (1, 2, 3):
            glnk.gl_precond_set_tiles(pre, 0, 64, 4096, shape)
            pre.apply(r, z1)
            e = relerr(host(z1), ref)
            assert e < (1e-13 if prec == glnk.GL_FP64 else 1e-6), (prec, shape, e)
