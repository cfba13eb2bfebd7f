"""Pins of the oracle on simplicial meshes of the paper's 2D test domains
(Sec. 3, Sec. 4.1): the triangle and the disc of circumradius 5
(paper_1204_5125_amd/meshes.py).

The oracle takes the edge coefficients from the Corollary's system
M alpha = b per triangle and the control volumes from the nodes' shares
1/4 alpha_e |e|^2 of their triangles' edges.  Pinned against: the Remark's
cotangent formula (a second route), the Corollary's identity
sum alpha e e^T = |Omega| I for the whole mesh, the equilateral lattice's
closed forms, the circumcentric (Voronoi) kite areas computed geometrically,
quadrature of the dipole's link integral, finite differences of GL, the
gauge identities, and a converged Newton solve."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs, meshes

DIPOLE_2D = ((0.0, 0.0, 1.0), (0.0, 0.0, 1.0))   # Sec. 4.1: m = e_z, x0 = (0, 0, 1) for the 2D domains


def areas(xy, tri):
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    u, v = b - a, c - a
    return 0.5 * np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])


def jittered_disc(k, seed):
    """The disc mesh with interior nodes moved by up to 10 % of the ring
    spacing (no longer symmetric; still a valid triangulation)."""
    xy, tri = meshes.disc(k)
    rng = np.random.default_rng(seed)
    r = np.hypot(xy[:, 0], xy[:, 1])
    inner = r < meshes.RADIUS * (1 - 0.5 / k)
    xy = xy.copy()
    xy[inner] += rng.uniform(-1, 1, (inner.sum(), 2)) * 0.1 * meshes.RADIUS / k
    return xy, tri


MESHES = [("tri", *meshes.triangle(6)), ("circ", *meshes.disc(5)), ("circ-jitter", *jittered_disc(5, 3))]
IDS = [m[0] for m in MESHES]


def test_meshes_cover_the_domains():
    for k in (1, 3, 8):
        xy, tri = meshes.triangle(k)
        assert len(xy) == (k + 1) * (k + 2) // 2 and len(tri) == k * k
        assert areas(xy, tri).sum() == pytest.approx(3 * np.sqrt(3) / 4 * 25, rel=1e-13)
        np.testing.assert_allclose(np.hypot(*xy[[0, k, -1]].T), 5.0, rtol=1e-14)  # the three corners
        xy, tri = meshes.disc(k)
        assert len(xy) == 1 + 3 * k * (k + 1) and len(tri) == 6 * k * k
        # the inscribed 6k-gon of the circle of radius 5
        assert areas(xy, tri).sum() == pytest.approx(0.5 * 6 * k * 25 * np.sin(2 * np.pi / (6 * k)), rel=1e-13)
        # every edge in one or two triangles, and non-obtuse triangles
        a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
        for p, q, r in ((a, b, c), (b, c, a), (c, a, b)):
            assert np.all(np.sum((q - p) * (r - p), axis=1) >= -1e-12)


@pytest.mark.parametrize("mesh", MESHES, ids=IDS)
def test_coefficients_follow_the_remark(mesh):
    """alpha of each edge equals the sum over its triangles of 1/2 cot of the
    opposite angle (Remark), computed here independently."""
    _, xy, tri = mesh
    m = oracle.Mesh.triangles(xy, tri, mu=0.7)
    want = {}
    for t in tri:
        for i in range(3):
            p, q, r = t[i], t[(i + 1) % 3], t[(i + 2) % 3]
            u, v = xy[p] - xy[r], xy[q] - xy[r]
            cot = (u @ v) / abs(u[0] * v[1] - u[1] * v[0])
            key = (max(p, q), min(p, q))
            want[key] = want.get(key, 0.0) + 0.5 * cot
    got = {(int(j), int(k)): a for j, k, a in zip(m.ej, m.ek, m.alpha)}
    assert set(got) == set(want)
    for key, a in got.items():
        assert a == pytest.approx(want[key], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("mesh", MESHES, ids=IDS)
def test_corollary_identity_and_volumes(mesh):
    """sum_edges alpha e e^T = |Omega| I and sum |V_j| = |Omega| (the
    Corollary summed over the triangles); the volumes are the circumcentric
    kite areas (the triangle's part of each Voronoi region), each computed as
    a polygon area from the circumcentre and the edge midpoints."""
    _, xy, tri = mesh
    m = oracle.Mesh.triangles(xy, tri, mu=0.7)
    area = areas(xy, tri).sum()
    S = np.zeros((2, 2))
    for j, k, a in zip(m.ej, m.ek, m.alpha):
        e = xy[j] - xy[k]
        S += a * np.outer(e, e)
    np.testing.assert_allclose(S, area * np.eye(2), atol=1e-11 * area)
    assert m.vol.sum() == pytest.approx(area, rel=1e-13)
    kite = np.zeros(len(xy))
    for t in tri:
        P = xy[t]
        d = 2 * (P[0, 0] * (P[1, 1] - P[2, 1]) + P[1, 0] * (P[2, 1] - P[0, 1]) + P[2, 0] * (P[0, 1] - P[1, 1]))
        s2 = np.sum(P ** 2, axis=1)
        cc = np.array([s2 @ (P[[1, 2, 0], 1] - P[[2, 0, 1], 1]), s2 @ (P[[2, 0, 1], 0] - P[[1, 2, 0], 0])]) / d
        for i in range(3):
            poly = np.array([P[i], 0.5 * (P[i] + P[(i + 1) % 3]), cc, 0.5 * (P[i] + P[(i + 2) % 3])])
            x, y = poly[:, 0], poly[:, 1]
            kite[t[i]] += 0.5 * abs(x @ np.roll(y, -1) - y @ np.roll(x, -1))
    np.testing.assert_allclose(m.vol, kite, rtol=1e-11)


def test_equilateral_lattice_closed_forms():
    """Triangle split into equilateral triangles of side s: interior edges
    alpha = 1/sqrt3 (two 60-degree angles), boundary edges 1/(2 sqrt3);
    interior nodes |V| = sqrt3/2 s^2 (the hexagonal Voronoi cell)."""
    k = 6
    xy, tri = meshes.triangle(k)
    s = 5 * np.sqrt(3) / k
    m = oracle.Mesh.triangles(xy, tri, mu=0.0)
    counts = {}
    for t in tri:
        for i in range(3):
            key = (max(t[i], t[(i + 1) % 3]), min(t[i], t[(i + 1) % 3]))
            counts[key] = counts.get(key, 0) + 1
    for j, kk, a in zip(m.ej, m.ek, m.alpha):
        want = 1 / np.sqrt(3) if counts[(int(j), int(kk))] == 2 else 0.5 / np.sqrt(3)
        assert a == pytest.approx(want, rel=1e-13)
    deg = np.bincount(np.concatenate([m.ej, m.ek]), minlength=m.n)
    np.testing.assert_allclose(m.vol[deg == 6], np.sqrt(3) / 2 * s * s, rtol=1e-13)


def test_dipole_links_on_the_disc():
    """The closed-form link phases of mu A_d (x0 = (0, 0, 1), m = e_z) on the
    disc mesh against adaptive quadrature of the line integral."""
    from scipy.integrate import quad
    xy, tri = meshes.disc(3)
    mu = 0.9
    m = oracle.Mesh.triangles(xy, tri, mu=mu, dipole=DIPOLE_2D)
    mm, x0 = np.asarray(DIPOLE_2D[0]), np.asarray(DIPOLE_2D[1])
    phases = -np.angle(m.U)
    for q in range(m.ne):
        xk, xj = m.x[m.ek[q]], m.x[m.ej[q]]
        e = xj - xk

        def f(t):
            r = xk + t * e - x0
            return e @ np.cross(mm, r) / np.linalg.norm(r) ** 3
        ref = mu * quad(f, 0.0, 1.0, epsabs=1e-17, epsrel=1e-13, limit=200)[0]
        assert phases[q] == pytest.approx(ref, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("pot", ["Az", "Ad"])
@pytest.mark.parametrize("mesh", MESHES, ids=IDS)
def test_operators_on_simplicial_meshes(mesh, pot):
    """K-hat Hermitian positive definite (semidefinite with constants in the
    kernel at A = 0); GL(1) = 0 at A = 0; J the derivative of GL (central
    differences), self-adjoint in <.,.>_R; J(psi)(i psi) = i GL(psi); the
    gauge covariance K-hat -> G K-hat G^H under A -> A + grad chi."""
    _, xy, tri = mesh
    kw = dict(mu=0.8, dipole=DIPOLE_2D) if pot == "Ad" else dict(mu=0.8)
    m = oracle.Mesh.triangles(xy, tri, **kw)
    K = m.khat.toarray()
    assert np.abs(K - K.conj().T).max() == 0.0
    assert np.linalg.eigvalsh(K).min() > 0
    m0 = oracle.Mesh.triangles(xy, tri, mu=0.0)
    np.testing.assert_allclose(m0.khat @ np.ones(m0.n), 0.0, atol=1e-13)
    np.testing.assert_allclose(m0.gl(np.ones(m0.n, complex)), 0.0, atol=1e-13)
    psi = inputs.random_complex(m.n, seed=41)
    phi = inputs.random_complex(m.n, seed=42)
    chi = inputs.random_complex(m.n, seed=43)
    eps = 1e-6
    fd = (m.gl(psi + eps * phi) - m.gl(psi - eps * phi)) / (2 * eps)
    J = m.jac(psi, phi)
    assert np.abs(fd - J).max() < 1e-7 * np.abs(J).max()
    assert m.inner(chi, m.jac(psi, phi)) == pytest.approx(m.inner(m.jac(psi, chi), phi), rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(m.jac(psi, 1j * psi), 1j * m.gl(psi), atol=1e-12 * np.abs(m.gl(psi)).max())
    if pot == "Az":
        # A' = A + grad chi with chi = r^T S r / 2 (S symmetric): the links pick
        # up exp(-i (chi_j - chi_k)), so K-hat' = G K-hat G^H, G = diag(e^{-i chi})
        S = np.array([[0.3, -0.2, 0.0], [-0.2, 0.5, 0.0], [0.0, 0.0, 0.0]])
        amat = oracle.field_matrix(0.8, (0.0, 0.0, 1.0))
        mg = oracle.Mesh.triangles(xy, tri, amat=amat + S)
        g = np.exp(-0.5j * np.einsum("ij,jk,ik->i", m.x, S, m.x))
        Kp = (g[:, None] * m.khat.toarray()) * g.conj()[None, :]
        assert np.abs(mg.khat.toarray() - Kp).max() < 1e-12 * np.abs(Kp).max()


def test_newton_converges_and_gauge_kernel():
    xy, tri = meshes.disc(6)
    m = oracle.Mesh.triangles(xy, tri, mu=0.8)
    psi, info = oracle.newton(m, np.ones(m.n, complex), max_steps=30, max_coarse=16)
    assert info["converged"] and info["res"][-1] < 1e-10
    # at a solution i psi spans the kernel of J (eq. jacobian nullspace)
    assert m.norm(m.jac(psi, 1j * psi)) < 1e-9 * m.norm(psi)
    # the hierarchy colours level 0 greedily (no red-black parity on triangles)
    amg = oracle.Amg.for_state(m, psi, max_coarse=16)
    assert amg.levels[0]["ncolors"] >= 3
