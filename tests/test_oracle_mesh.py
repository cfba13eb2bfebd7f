"""Pins of the oracle's geometry and of K-hat against what the paper and the
mathematics fix (Sec. 3), independent of the oracle's own formulas."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs


def grid_coords(mesh):
    return mesh.x[:, :mesh.dim]


@pytest.mark.parametrize("dim,N,L", [(2, (9, 9), (5.0, 5.0)), (2, (7, 11), (3.0, 5.0)),
                                     (3, (5, 5, 5), (5.0, 5.0, 5.0)), (3, (4, 5, 6), (2.0, 3.0, 4.0))])
def test_volumes_partition_domain(dim, N, L):
    """Voronoi regions clipped to the box tile it: sum |V_i| = |Omega|; interior
    cells are full boxes, each boundary axis halves the cell."""
    m = oracle.Mesh(dim, N, L)
    assert m.vol.sum() == pytest.approx(np.prod(L), rel=1e-14)
    h = np.array(L) / (np.array(N) - 1)
    idx = np.stack(np.unravel_index(np.arange(m.n), N[::-1])[::-1], axis=1)
    nb = ((idx == 0) | (idx == np.array(N) - 1)).sum(axis=1)
    np.testing.assert_allclose(m.vol, np.prod(h) * 0.5 ** nb, rtol=1e-14)


@pytest.mark.parametrize("dim,N,L", [(2, (9, 9), (5.0, 5.0)), (2, (6, 10), (2.0, 7.0)),
                                     (3, (5, 5, 5), (5.0, 5.0, 5.0)), (3, (4, 6, 5), (1.0, 2.0, 3.0))])
def test_edge_coefficients_reproduce_identity(dim, N, L):
    """Corollary (simplex edge coefficients): sum over edges alpha e e^T equals
    |S| I on every simplex, hence |Omega| I over the whole mesh."""
    m = oracle.Mesh(dim, N, L)
    X = grid_coords(m)
    E = X[m.ej] - X[m.ek]
    S = np.einsum("e,ei,ej->ij", m.alpha, E, E)
    np.testing.assert_allclose(S, np.prod(L) * np.eye(dim), rtol=1e-13, atol=1e-13)


def _triangle_alpha(p):
    """Solve the Corollary's M alpha = b for one triangle with vertices p (3x2)."""
    edges = [(0, 1), (1, 2), (2, 0)]
    e = np.array([p[a] - p[b] for a, b in edges])
    u, v = e[0], -e[2]
    area = 0.5 * abs(u[0] * v[1] - u[1] * v[0])
    M = (e @ e.T) ** 2
    b = area * (e * e).sum(axis=1)
    return edges, np.linalg.solve(M, b)


@pytest.mark.parametrize("hx,hy", [(1.0, 1.0), (0.5, 1.25)])
def test_alpha_2d_matches_simplex_system(hx, hy):
    """2D coefficients accumulated over adjacent triangles equal the solution of
    M alpha = b (Corollary) summed the same way; the Remark's cot formula and
    the linear system must agree."""
    N = (5, 4)
    m = oracle.Mesh(2, N, (hx * (N[0] - 1), hy * (N[1] - 1)))
    tri_alpha = {}
    for cy in range(N[1] - 1):
        for cx in range(N[0] - 1):
            ids = [cx + N[0] * cy, cx + 1 + N[0] * cy, cx + 1 + N[0] * (cy + 1), cx + N[0] * (cy + 1)]
            for tri in ([ids[0], ids[1], ids[2]], [ids[0], ids[3], ids[2]]):
                pts = m.x[tri, :2]
                edges, al = _triangle_alpha(pts)
                for (a, b), v in zip(edges, al):
                    key = (min(tri[a], tri[b]), max(tri[a], tri[b]))
                    tri_alpha[key] = tri_alpha.get(key, 0.0) + v
    for j, k, a in zip(m.ej, m.ek, m.alpha):
        assert a == pytest.approx(tri_alpha[(k, j)], rel=1e-12)
    # diagonals carry zero weight (right angle opposite)
    diag = [v for (k, j), v in tri_alpha.items() if j - k == N[0] + 1]
    np.testing.assert_allclose(diag, 0.0, atol=1e-12)


def test_link_variables_closed_form_uniform_field():
    """U_jk = exp(-i h A(midpoint) . e) for A = mu/2 (-y, x): x-edges carry
    exp(+i mu h y / 2), y-edges exp(-i mu h x / 2); |U| = 1."""
    mu, N, L = 0.8, (6, 6), (5.0, 5.0)
    m = oracle.Mesh(2, N, L, mu=mu)
    h = L[0] / (N[0] - 1)
    np.testing.assert_allclose(np.abs(m.U), 1.0, rtol=0, atol=1e-15)
    for j, k, u in zip(m.ej, m.ek, m.U):
        mid = 0.5 * (m.x[j] + m.x[k])
        if j - k == 1:
            ref = np.exp(1j * mu * h * mid[1] / 2)
        else:
            ref = np.exp(-1j * mu * h * mid[0] / 2)
        assert abs(u - ref) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_gauge_sign_curl_free_potential(dim):
    """For a curl-free A = grad chi the discrete K-hat annihilates exp(-i chi)
    and not exp(+i chi): the link-variable sign of Sec. 3 (reading: the discrete
    operator is the paper's eq. with A -> -A)."""
    c = 0.7
    if dim == 2:
        N, L = (9, 9), (5.0, 5.0)
        amat = c * np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0]], dtype=float)  # grad(c x y)
        chi = lambda X: c * X[:, 0] * X[:, 1]
    else:
        N, L = (5, 6, 5), (3.0, 4.0, 3.0)
        amat = c * np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=float)  # grad(c (xy + yz))
        chi = lambda X: c * (X[:, 0] * X[:, 1] + X[:, 1] * X[:, 2])
    m = oracle.Mesh(dim, N, L, amat=amat)
    ch = chi(m.x)
    assert np.abs(m.khat_apply(np.exp(-1j * ch))).max() < 1e-13
    assert np.abs(m.khat_apply(np.exp(1j * ch))).max() > 1e-2


@pytest.mark.parametrize("dim,N,mu,bdir", [(2, (9, 9), 0.8, (0, 0, 1)), (2, (12, 7), 1.3, (0, 0, 1)),
                                           (3, (5, 5, 5), 0.6, (1, 1, 1)), (3, (4, 5, 3), 2.0, (0, 1, 0))])
def test_khat_hermitian_positive(dim, N, mu, bdir):
    """K-hat is Hermitian (Remark on K = D^-1 K-hat) and positive semidefinite
    (Lemma, eq. posdef), strictly positive for a nonzero field."""
    bdir = np.array(bdir, float) / np.linalg.norm(bdir)
    m = oracle.Mesh(dim, N, [5.0] * dim, mu=mu, bdir=bdir)
    K = m.khat.toarray()
    assert np.array_equal(K, K.conj().T)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > 1e-6


def test_khat_semidefinite_zero_field_nullvector():
    """A = 0: psi = 1 is in the null space; K-hat stays semidefinite."""
    m = oracle.Mesh(2, (8, 8), (5.0, 5.0), mu=0.0)
    assert np.abs(m.khat_apply(np.ones(m.n))).max() < 1e-14
    ev = np.linalg.eigvalsh(m.khat.toarray())
    assert ev.min() > -1e-12 and abs(ev.min()) < 1e-12


@pytest.mark.parametrize("dim,N,L", [(2, (9, 9), (5.0, 5.0)), (2, (7, 10), (3.0, 4.0)),
                                     (3, (5, 4, 6), (2.0, 3.0, 2.5))])
def test_zero_field_is_neumann_laplacian(dim, N, L):
    """At A = 0, K = D^-1 K-hat is the Neumann Laplacian (Sec. 3); on a tensor
    grid its eigenvalues are the DCT-I values sum_a 4/h_a^2 sin^2(pi k_a / (2(N_a-1)))."""
    m = oracle.Mesh(dim, N, L, mu=0.0)
    Dm = np.diag(m.vol ** -0.5)
    ev = np.sort(np.linalg.eigvalsh(Dm @ m.khat.toarray().real @ Dm))
    h = np.array(L) / (np.array(N) - 1)
    one_d = [4 / h[a] ** 2 * np.sin(np.pi * np.arange(N[a]) / (2 * (N[a] - 1))) ** 2
             for a in range(dim)]
    grid = one_d[0]
    for a in range(1, dim):
        grid = np.add.outer(grid, one_d[a]).ravel()
    np.testing.assert_allclose(ev, np.sort(grid), rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("mu", [0.3, 1.7])
def test_rayleigh_quotient_of_constant(mu):
    """<1, K 1> / <1, 1> = |Omega|^-1 sum alpha |2 sin(arg U / 2)|^2 (eq. smallest
    lambda, exact form), computed from the CSR operator and from the edge list."""
    m = oracle.Mesh(2, (10, 10), (5.0, 5.0), mu=mu)
    one = np.ones(m.n, complex)
    lhs = m.inner(one, m.khat_apply(one) / m.vol) / m.inner(one, one)
    rhs = (m.alpha * np.abs(2 * np.sin(np.angle(m.U) / 2)) ** 2).sum() / 25.0
    assert lhs == pytest.approx(rhs, rel=1e-13)


DIPOLE_3D = ((0.0, 0.0, 1.0), (0.0, 0.0, 6.0))   # Sec. 4.1: m = e_z, x0 = (0, 0, 6) in 3D
DIPOLE_2D = ((0.0, 0.0, 1.0), (0.0, 0.0, 1.0))   # x0 = (0, 0, 1) above the 2D domains


def test_dipole_links_equal_the_edge_integral():
    """The closed-form link phases of mu A_d against adaptive quadrature of
    the line integral along every edge (3D cube of circumradius 5 and the
    2D square), and |U| = 1."""
    from scipy.integrate import quad
    for dim, N, L, (mm, x0) in ((3, (5, 4, 6), (5.77, 5.77, 5.77), DIPOLE_3D),
                                (2, (7, 6), (7.07, 7.07), DIPOLE_2D)):
        mu = 0.8
        m = oracle.Mesh(dim, N, L, mu=mu, dipole=(mm, x0))
        mm, x0 = np.asarray(mm), np.asarray(x0)
        phases = -np.angle(m.U)
        for q in range(m.ne):
            xk, xj = m.x[m.ek[q]], m.x[m.ej[q]]
            e = xj - xk

            def f(t):
                r = xk + t * e - x0
                return e @ np.cross(mm, r) / np.linalg.norm(r) ** 3
            ref = mu * quad(f, 0.0, 1.0, epsabs=1e-17, epsrel=1e-13, limit=200)[0]
            assert phases[q] == pytest.approx(ref, rel=1e-11, abs=1e-15)
        np.testing.assert_allclose(np.abs(m.U), 1.0, rtol=1e-15)


def test_dipole_khat_hermitian_and_jacobian_identities():
    """K-hat in the dipole potential is Hermitian positive definite; J is the
    derivative of GL (central differences), self-adjoint in <.,.>_R, and
    J(psi)(i psi) = i GL(psi)."""
    m = oracle.Mesh(3, (5, 5, 5), (5.77, 5.77, 5.77), mu=1.0, dipole=DIPOLE_3D)
    K = m.khat.toarray()
    assert np.abs(K - K.conj().T).max() == 0.0
    assert np.linalg.eigvalsh(K).min() > 0
    psi = inputs.random_complex(m.n, seed=91)
    phi = inputs.random_complex(m.n, seed=92)
    chi = inputs.random_complex(m.n, seed=93)
    eps = 1e-6
    fd = (m.gl(psi + eps * phi) - m.gl(psi - eps * phi)) / (2 * eps)
    jp = m.jac(psi, phi)
    assert np.abs(fd - jp).max() < 1e-8 * np.abs(jp).max()
    assert m.inner(phi, m.jac(psi, chi)) == pytest.approx(m.inner(m.jac(psi, phi), chi), rel=1e-12)
    assert np.abs(m.jac(psi, 1j * psi) - 1j * m.gl(psi)).max() < 1e-12 * np.abs(m.gl(psi)).max()
