"""The GPU path on simplicial meshes of the paper's test domains (Sec. 4.1:
the triangle, the disc, the tetrahedron and the ball of circumradius 5;
paper_1204_5125_amd/meshes.py) against the oracle, through the C-ABI: the operators (FP64 within 1e-12),
the hierarchy (integer arrays bit-exact, values within 1e-12; level 0
coloured like the coarse levels), the V-cycle (FP64 1e-11, FP32 and mixed
1e-5, k = 3, R_inf), MINRES iterates (1e-12) and counts (within 1), Newton
(states within 1e-10 after phase alignment), the deflated solve, the
parameter derivative, batches bitwise equal to single solves, and the
errors the call reports.  Meshes span several 256-node tiles with ragged
tails; uniform field A_z and the dipole A_d (m = e_z, x0 = (0, 0, 1) in 2D,
(0, 0, 6) in 3D).  Level 0 is checked to be exactly Hermitian."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import arclength as oal
from paper_1204_5125_amd import inputs, meshes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIPOLE_2D = ((0.0, 0.0, 1.0), (0.0, 0.0, 1.0))
DIPOLE_3D = ((0.0, 0.0, 1.0), (0.0, 0.0, 6.0))


def jittered_disc(k, seed):
    xy, tri = meshes.disc(k)
    rng = np.random.default_rng(seed)
    r = np.hypot(xy[:, 0], xy[:, 1])
    inner = r < meshes.RADIUS * (1 - 0.5 / k)
    xy = xy.copy()
    xy[inner] += rng.uniform(-1, 1, (inner.sum(), 2)) * 0.1 * meshes.RADIUS / k
    return xy, tri


def jittered_tet(k, seed):
    x, t = meshes.tetrahedron(k)
    rng = np.random.default_rng(seed)
    B = np.linalg.solve(np.vstack([meshes.TET_VERTICES.T, np.ones(4)]), np.vstack([x.T, np.ones(len(x))]))
    inner = np.all(B > 1e-9, axis=0)
    x = x.copy()
    x[inner] += rng.uniform(-1, 1, (inner.sum(), 3)) * 0.08 * 5 * np.sqrt(8 / 3) / k
    return x, t


MESHES = {"tri-24": meshes.triangle(24), "circ-14": meshes.disc(14), "circ-jitter-9": jittered_disc(9, 5),
          "tet-12": meshes.tetrahedron(12), "tet-jitter-9": jittered_tet(9, 6), "ball-7": meshes.ball(7)}
CASES = [(name, pot) for name in MESHES for pot in ("Az", "Ad")]
IDS = [f"{n}-{p}" for n, p in CASES]


@pytest.fixture(scope="module")
def glnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5125_amd import glnk as g
    g.lib()
    return g


def make_pair(glnk, case, mu=0.8):
    name, pot = case
    x, cells = MESHES[name]
    kw = dipole_kw(x, pot)
    return glnk.Mesh.simplicial(x, cells, mu=mu, **kw), oracle.Mesh.simplices(x, cells, mu=mu, **kw)


def dipole_kw(x, pot):
    if pot != "Ad":
        return {}
    return dict(dipole=DIPOLE_2D if x.shape[1] == 2 else DIPOLE_3D)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_operators(glnk, case):
    """GL(psi), its D-norm and J(psi) phi against the oracle."""
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=1)
    phi = inputs.random_complex(mo.n, seed=2)
    out = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    nrm = glnk.gl_residual(mg, dev(psi), out)
    ref = mo.gl(psi)
    assert relerr(host(out), ref) < 1e-12
    assert nrm == pytest.approx(mo.norm(ref), rel=1e-12)
    glnk.gl_jacobian_apply(mg, dev(psi), dev(phi), out)
    assert relerr(host(out), mo.jac(psi, phi)) < 1e-12
    # the field can be changed in place
    mg.set_field(1.3)
    kw = dipole_kw(MESHES[case[0]][0], case[1])
    m2 = oracle.Mesh.simplices(*MESHES[case[0]], mu=1.3, **kw)
    glnk.gl_residual(mg, dev(psi), out)
    assert relerr(host(out), m2.gl(psi)) < 1e-12


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_hierarchy_bit_exact(glnk, case):
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=3)
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    info = pre.info()
    assert info["nlev"] == amg.nlev >= 2
    assert info["ncolors"][0] >= 3  # no red-black parity on triangles or tetrahedra
    # level 0 exactly Hermitian: both entries of an edge computed alike
    Ag = sp.csr_matrix((pre.export(0, "A_v"), pre.export(0, "A_ci"), pre.export(0, "A_rp")), shape=(mo.n, mo.n))
    assert (Ag - Ag.conj().T).count_nonzero() == 0
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
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=4)
    r = inputs.random_complex(mo.n, seed=5)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    ref = amg.precond(mo, r)
    z = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    pre.apply(dev(r), z)
    assert relerr(host(z), ref) < 1e-11
    for prec in (glnk.GL_FP32, glnk.GL_MIXED):
        pre.update(dev(psi), precision=prec)
        pre.apply(dev(r), z)
        assert relerr(host(z), ref) < 1e-5, prec
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=3)
    pre.apply(dev(r), z)
    assert relerr(host(z), amg.precond(mo, r, cycles=3)) < 1e-11
    # R_inf = H^-1 D (CG with the V-cycle, its step count calibrated at setup)
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=0)
    pre.apply(dev(r), z)
    assert relerr(host(z), oracle.precond_exact(mo, psi, r)) < 1e-10
    # every lane count and bottom-kernel split
    pre.update(dev(psi), precision=glnk.GL_FP64, cycles=1)
    for tiles in ((1, 64, 0), (-1, 8192, 0), (0, 0, 4096)):
        glnk.gl_precond_set_tiles(pre, *tiles)
        pre.apply(dev(r), z)
        assert relerr(host(z), ref) < 1e-11, tiles


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_minres_iterates(glnk, case):
    mg, mo = make_pair(glnk, case)
    psi = inputs.random_phase_state(mo.n, seed=6)
    b = inputs.random_complex(mo.n, seed=7)
    amg = oracle.Amg.for_state(mo, psi, max_coarse=16)
    pre = glnk.Precond(mg, dev(psi), max_coarse=16)
    x = torch.empty(mo.n, dtype=torch.complex128, device="cuda")
    for k in (1, 2, 5):
        xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=k)
        rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=0.0, max_iter=k, poll_every=2)
        assert ig["iterations"] == k
        assert relerr(host(x), xo) < 1e-12, k
    xo, io, _ = oracle.minres(mo, psi, b, amg=amg, rtol=1e-10, max_iter=2000)
    rc, ig = glnk.gl_jacobian_solve(mg, dev(psi), pre, dev(b), x, rtol=1e-10, max_iter=2000)
    assert io["converged"] and ig["converged"]
    assert abs(ig["iterations"] - io["iterations"]) <= 1
    xk, _, _ = oracle.minres(mo, psi, b, amg=amg, rtol=0.0, max_iter=ig["iterations"])
    assert relerr(host(x), xk) < 1e-10


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_newton_from_psi_one(glnk, case):
    """Newton from psi = 1 (the experiments' state) converges to the oracle's
    solution with the same step count; deflated Newton too (mu = 0.5: from
    psi = 1 plain Newton does not converge on the triangle at mu = 0.9, in
    the oracle either)."""
    mg, mo = make_pair(glnk, case, mu=0.5)
    po, io = oracle.newton(mo, np.ones(mo.n, complex), max_steps=30, max_coarse=16)
    psi = torch.ones(mo.n, dtype=torch.complex128, device="cuda")
    rc, ig = glnk.gl_newton_solve(mg, psi, max_steps=30, max_coarse=16)
    assert rc == 0 and io["converged"] and ig["converged"]
    assert ig["steps"] == io["steps"]
    ps = host(psi)
    ip = np.vdot(ps, po)
    e = np.abs(ps * (ip / abs(ip)) - po).max() / max(np.abs(po).max(), 1.0)
    assert e < 1e-10, e
    pd, idf = oracle.newton(mo, np.ones(mo.n, complex), max_steps=30, max_coarse=16, deflate=True)
    psi = torch.ones(mo.n, dtype=torch.complex128, device="cuda")
    rc, ig = glnk.gl_newton_solve(mg, psi, max_steps=30, max_coarse=16, deflate=True)
    assert rc == 0 and ig["steps"] == idf["steps"]
    if not all(abs(a - b) <= 1 for a, b in zip(ig["krylov_iters"], idf["krylov_iters"])):
        # the oracle's own counts move under rounding: the same start rotated
        # by exact phases (a symmetry of GL) spreads them by up to 2 on the
        # ball; the GPU's count must lie within 1 of that spread
        runs = [oracle.newton(mo, np.full(mo.n, np.exp(2j * np.pi * r / 8)), max_steps=30, max_coarse=16,
                              deflate=True)[1]["krylov_iters"] for r in range(8)]
        lo, hi = np.min(runs, axis=0), np.max(runs, axis=0)
        assert np.all((np.array(ig["krylov_iters"]) >= lo - 1) & (np.array(ig["krylov_iters"]) <= hi + 1)), \
            (ig["krylov_iters"], lo, hi)


@pytest.mark.parametrize("name", ["circ-jitter-9", "tet-jitter-9"])
def test_parameter_derivative(glnk, name):
    """gl_residual_dmu against the oracle's GL_mu (uniform field) and central
    differences in mu (both potentials)."""
    xy, tri = MESHES[name]
    psi = inputs.random_phase_state(len(xy), seed=8)
    out = torch.empty(len(xy), dtype=torch.complex128, device="cuda")
    mg = glnk.Mesh.simplicial(xy, tri, mu=0.7)
    mo = oracle.Mesh.simplices(xy, tri, mu=0.7)
    glnk.gl_residual_dmu(mg, dev(psi), out)
    assert relerr(host(out), oal.gl_dmu(mo, psi, (0.0, 0.0, 1.0))) < 1e-12
    for pot in ("Az", "Ad"):
        kw = dipole_kw(xy, pot)
        mg = glnk.Mesh.simplicial(xy, tri, mu=0.7, **kw)
        glnk.gl_residual_dmu(mg, dev(psi), out)
        h = 1e-5
        fd = (oracle.Mesh.simplices(xy, tri, mu=0.7 + h, **kw).gl(psi)
              - oracle.Mesh.simplices(xy, tri, mu=0.7 - h, **kw).gl(psi)) / (2 * h)
        assert relerr(host(out), fd) < 1e-8


def test_batch_equals_single(glnk):
    ms, p0 = [], []
    for name, pot in CASES[:4] + CASES[-2:]:
        m, _ = make_pair(glnk, (name, pot), mu=0.5)
        ms.append(m)
        p0.append(inputs.random_phase_state(m.n, seed=9))
    kw = dict(tol=1e-10, max_steps=30, krylov_max_iter=2000, max_coarse=16)
    singles = []
    for m, p in zip(ms, p0):
        psi = dev(p)
        rc, info = glnk.gl_newton_solve(m, psi, **kw)
        singles.append((rc, info, host(psi)))
    batch = glnk.Batch(ms)
    psis = [dev(p) for p in p0]
    rc, infos = batch.newton_solve(psis, **kw)
    for (rc1, i1, ps1), i2, psi in zip(singles, infos, psis):
        assert rc1 == 0 and i1["converged"] and i2["converged"]
        assert i1["res"] == i2["res"] and i1["krylov_iters"] == i2["krylov_iters"]
        assert np.array_equal(ps1, host(psi))


def test_errors(glnk):
    xy, tri = meshes.triangle(4)
    m = glnk.Mesh.simplicial(xy, tri, mu=0.5)
    with pytest.raises(RuntimeError, match="no axes"):
        m.export_links(0)
    net = glnk.UNet(3, 32)
    psi = torch.ones(m.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="square 2D grid"):
        net.predict(m, psi, psi, 0.5, 0.02, torch.empty_like(psi))
    bad = tri.copy()
    bad[0, 0] = len(xy)
    with pytest.raises(RuntimeError, match="out of range"):
        glnk.Mesh.simplicial(xy, bad)
    bad = tri.copy()
    bad[0] = (bad[0, 0], bad[0, 0], bad[0, 1])
    with pytest.raises(RuntimeError, match="degenerate"):
        glnk.Mesh.simplicial(xy, bad)
    with pytest.raises(RuntimeError, match="more than two"):
        glnk.Mesh.simplicial(xy, np.concatenate([tri, tri[:1]]))
    xy2 = np.concatenate([xy, [[9.0, 9.0]]])
    with pytest.raises(RuntimeError, match="no cell"):
        glnk.Mesh.simplicial(xy2, tri)
    # tetrahedra: a flat cell, a face in three cells
    x3, t3 = meshes.tetrahedron(3)
    glnk.Mesh.simplicial(x3, t3, mu=0.5)
    flat = t3.copy()
    flat[0, 3] = flat[0, 2]
    with pytest.raises(RuntimeError, match="degenerate"):
        glnk.Mesh.simplicial(x3, flat)
    with pytest.raises(RuntimeError, match="more than two"):
        glnk.Mesh.simplicial(x3, np.concatenate([t3, t3[:1]]))
    with pytest.raises(ValueError):
        glnk.Mesh.simplicial(x3, tri)
