"""Pins of the oracle on simplicial meshes of the paper's test domains
(Sec. 3, Sec. 4.1): the triangle, the disc, the tetrahedron and the ball of
circumradius 5 (paper_1204_5125_amd/meshes.py).

The oracle takes the edge coefficients from the Corollary's system
M alpha = b per triangle and the control volumes from the nodes' shares
1/4 alpha_e |e|^2 of their triangles' edges; in 3D the same system per
tetrahedron, with shares 1/6 alpha_e |e|^2.  Pinned against: the Remark's cotangent formula (a second
route; in 3D the dihedral-angle cotangents), the Corollary's identity
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


# ---------------------------------------------------------------- tetrahedra
DIPOLE_3D = ((0.0, 0.0, 1.0), (0.0, 0.0, 6.0))   # Sec. 4.1: x0 = (0, 0, 6) for the 3D domains
TET_VOLUME = 5 ** 3 * 8 / (9 * np.sqrt(3))       # regular tetrahedron of circumradius 5


def tet_volumes(x, t):
    P = x[t]
    return np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6


def jittered_tet(k, seed):
    """The tetrahedron mesh with interior lattice nodes moved by up to 8 % of
    the lattice edge (still a valid mesh; coefficients of either sign)."""
    x, t = meshes.tetrahedron(k)
    rng = np.random.default_rng(seed)
    x = x.copy()
    # interior: strictly inside all four faces (barycentric coordinates > 0)
    B = np.linalg.solve(np.vstack([meshes.TET_VERTICES.T, np.ones(4)]), np.vstack([x.T, np.ones(len(x))]))
    inner = np.all(B > 1e-9, axis=0)
    x[inner] += rng.uniform(-1, 1, (inner.sum(), 3)) * 0.08 * 5 * np.sqrt(8 / 3) / k
    return x, t


TETS = [("tet", *meshes.tetrahedron(4)), ("tet-jitter", *jittered_tet(5, 7)), ("ball", *meshes.ball(6))]
TET_IDS = [m[0] for m in TETS]


def test_tet_mesh_covers_the_domain():
    for k in (1, 2, 5):
        x, t = meshes.tetrahedron(k)
        assert len(x) == (k + 1) * (k + 2) * (k + 3) // 6 + (k - 1) * k * (k + 1) // 6
        v = tet_volumes(x, t)
        assert v.min() > 0 and v.sum() == pytest.approx(TET_VOLUME, rel=1e-13)
        faces = {}
        for c in t:
            for f in range(4):
                key = tuple(sorted(np.delete(c, f)))
                faces[key] = faces.get(key, 0) + 1
        assert max(faces.values()) <= 2
        # the faces in one cell tile the surface: four equilateral triangles of side s
        once = np.array([f for f, c in faces.items() if c == 1])
        area = 0.5 * np.linalg.norm(np.cross(x[once[:, 1]] - x[once[:, 0]], x[once[:, 2]] - x[once[:, 0]]), axis=1)
        assert area.sum() == pytest.approx(4 * np.sqrt(3) / 4 * (5 * np.sqrt(8 / 3)) ** 2, rel=1e-13)


@pytest.mark.parametrize("mesh", TETS, ids=TET_IDS)
def test_tet_coefficients_follow_the_dihedral_cotangents(mesh):
    """In 3D the Corollary's alpha of an edge is the sum over its tetrahedra
    of |e'| cot(theta') / 6, e' the opposite edge and theta' the dihedral
    angle there (the linear finite-element stiffness), computed here from
    face normals; the sum alpha e e^T is |Omega| I; the volumes add up to
    |Omega|."""
    _, x, t = mesh
    m = oracle.Mesh.simplices(x, t, mu=0.7)
    want = {}
    for c in t:
        for a in range(4):
            for b in range(a + 1, 4):
                o = [v for v in range(4) if v not in (a, b)]
                p, q = x[c[o[0]]], x[c[o[1]]]
                eo = q - p
                na, nb = np.cross(eo, x[c[a]] - p), np.cross(eo, x[c[b]] - p)
                cos = na @ nb / (np.linalg.norm(na) * np.linalg.norm(nb))
                key = (max(c[a], c[b]), min(c[a], c[b]))
                want[key] = want.get(key, 0.0) + np.linalg.norm(eo) * cos / np.sqrt(1 - cos * cos) / 6
    got = {(int(j), int(kk)): a for j, kk, a in zip(m.ej, m.ek, m.alpha)}
    assert set(got) == set(want)
    for key, a in got.items():
        assert a == pytest.approx(want[key], rel=1e-11, abs=1e-13)
    S = np.zeros((3, 3))
    for j, kk, a in zip(m.ej, m.ek, m.alpha):
        e = x[j] - x[kk]
        S += a * np.outer(e, e)
    omega = tet_volumes(x, t).sum()
    np.testing.assert_allclose(S, omega * np.eye(3), atol=1e-11 * omega)
    assert m.vol.sum() == pytest.approx(omega, rel=1e-13)


def test_tet_regular_cell_closed_forms():
    """k = 1: one regular tetrahedron of edge s = 5 sqrt(8/3); every dihedral
    angle is arccos(1/3), so every edge has alpha = s / (6 sqrt 8) and every
    vertex |V| = 3 shares of alpha s^2 / 6 = |T| / 4."""
    x, t = meshes.tetrahedron(1)
    m = oracle.Mesh.simplices(x, t, mu=0.0)
    s = 5 * np.sqrt(8 / 3)
    np.testing.assert_allclose(m.alpha, s / (6 * np.sqrt(8)), rtol=1e-13)
    np.testing.assert_allclose(m.vol, TET_VOLUME / 4, rtol=1e-13)


def test_tet_dipole_links():
    """The closed-form link phases of mu A_d (x0 = (0, 0, 6), m = e_z) on a
    tetrahedron mesh against adaptive quadrature of the line integral."""
    from scipy.integrate import quad
    x, t = meshes.tetrahedron(3)
    mu = 0.9
    m = oracle.Mesh.simplices(x, t, mu=mu, dipole=DIPOLE_3D)
    mm, x0 = np.asarray(DIPOLE_3D[0]), np.asarray(DIPOLE_3D[1])
    phases = -np.angle(m.U)
    for q in range(m.ne):
        xk, xj = m.x[m.ek[q]], m.x[m.ej[q]]
        e = xj - xk

        def f(s_):
            r = xk + s_ * e - x0
            return e @ np.cross(mm, r) / np.linalg.norm(r) ** 3
        ref = mu * quad(f, 0.0, 1.0, epsabs=1e-17, epsrel=1e-13, limit=200)[0]
        assert phases[q] == pytest.approx(ref, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("pot", ["Az", "Ad"])
@pytest.mark.parametrize("mesh", TETS, ids=TET_IDS)
def test_tet_operators(mesh, pot):
    """As on triangles: K-hat Hermitian, positive definite in a field and
    with constants in its kernel at A = 0; J the derivative of GL, self-adjoint
    in <.,.>_R, with J(psi)(i psi) = i GL(psi); gauge covariance."""
    _, x, t = mesh
    kw = dict(mu=0.8, dipole=DIPOLE_3D) if pot == "Ad" else dict(mu=0.8)
    m = oracle.Mesh.simplices(x, t, **kw)
    K = m.khat.toarray()
    assert np.abs(K - K.conj().T).max() == 0.0
    assert np.linalg.eigvalsh(K).min() > 0
    m0 = oracle.Mesh.simplices(x, t, mu=0.0)
    np.testing.assert_allclose(m0.khat @ np.ones(m0.n), 0.0, atol=1e-12)
    psi = inputs.random_complex(m.n, seed=51)
    phi = inputs.random_complex(m.n, seed=52)
    chi = inputs.random_complex(m.n, seed=53)
    eps = 1e-6
    fd = (m.gl(psi + eps * phi) - m.gl(psi - eps * phi)) / (2 * eps)
    J = m.jac(psi, phi)
    assert np.abs(fd - J).max() < 1e-7 * np.abs(J).max()
    assert m.inner(chi, m.jac(psi, phi)) == pytest.approx(m.inner(m.jac(psi, chi), phi), rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(m.jac(psi, 1j * psi), 1j * m.gl(psi), atol=1e-12 * np.abs(m.gl(psi)).max())
    if pot == "Az":
        S = np.array([[0.3, -0.2, 0.1], [-0.2, 0.5, 0.0], [0.1, 0.0, -0.4]])
        amat = oracle.field_matrix(0.8, (0.0, 0.0, 1.0))
        mg = oracle.Mesh.simplices(x, t, amat=amat + S)
        g = np.exp(-0.5j * np.einsum("ij,jk,ik->i", m.x, S, m.x))
        Kp = (g[:, None] * m.khat.toarray()) * g.conj()[None, :]
        assert np.abs(mg.khat.toarray() - Kp).max() < 1e-12 * np.abs(Kp).max()


def test_tet_newton_converges():
    x, t = meshes.tetrahedron(8)
    m = oracle.Mesh.simplices(x, t, mu=0.5)
    psi, info = oracle.newton(m, np.ones(m.n, complex), max_steps=30, max_coarse=16)
    assert info["converged"] and info["res"][-1] < 1e-10
    assert m.norm(m.jac(psi, 1j * psi)) < 1e-9 * m.norm(psi)


def test_ball_mesh_and_closed_forms():
    """The body-centred cubic ball: every cell the same tetrahedron (volume
    h^3 / 12), no face in more than two cells, the volume within 0.3 % of
    the ball's from m = 16 on.  In the Corollary's coefficients the lattice's
    long edges (length h, dihedral angle 90 degrees opposite) get 0 and a
    short edge (length h sqrt3 / 2) with all six cells around it gets
    6 (h sqrt3 / 2) cot(60 deg) / 6 = h / 2; a node with all 24 of its cells
    present has |V| = h^3 / 2, the lattice's Voronoi cell (a truncated
    octahedron)."""
    for m in (4, 7, 16):
        x, t = meshes.ball(m)
        h = 10.0 / m
        v = tet_volumes(x, t)
        np.testing.assert_allclose(v, h ** 3 / 12, rtol=1e-12)
        faces = {}
        for c in t:
            for f in range(4):
                key = tuple(sorted(np.delete(c, f)))
                faces[key] = faces.get(key, 0) + 1
        assert max(faces.values()) <= 2
        ball = 4 / 3 * np.pi * 125
        assert abs(v.sum() - ball) < (0.003 if m >= 16 else 0.05) * ball
        if m == 16:
            continue
        mo = oracle.Mesh.simplices(x, t, mu=0.0)
        L = np.linalg.norm(x[mo.ej] - x[mo.ek], axis=1)
        long = np.abs(L - h) < 1e-9 * h
        assert np.all(np.abs(L[~long] - h * np.sqrt(3) / 2) < 1e-9 * h)
        assert np.all(np.abs(mo.alpha[long]) < 1e-12 * h)
        assert mo.alpha.min() > -1e-12 * h
        full = np.bincount(t.ravel(), minlength=len(x)) == 24
        assert full.sum() > 0
        np.testing.assert_allclose(mo.vol[full], h ** 3 / 2, rtol=1e-12)
        inner = ~long & full[mo.ej] & full[mo.ek]
        assert inner.sum() > 0
        np.testing.assert_allclose(mo.alpha[inner], h / 2, rtol=1e-12)


def test_ball_newton_converges():
    x, t = meshes.ball(8)
    m = oracle.Mesh.simplices(x, t, mu=0.5, dipole=DIPOLE_3D)
    psi, info = oracle.newton(m, np.ones(m.n, complex), max_steps=30, max_coarse=16)
    assert info["converged"] and info["res"][-1] < 1e-10
    m = oracle.Mesh.simplices(x, t, mu=0.5)
    psi, info = oracle.newton(m, np.ones(m.n, complex), max_steps=30, max_coarse=16)
    assert info["converged"] and info["res"][-1] < 1e-10
    assert m.norm(m.jac(psi, 1j * psi)) < 1e-9 * m.norm(psi)
