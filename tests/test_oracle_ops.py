"""Pins of the oracle's GL residual, Jacobian and energy (Sec. 2, Sec. 3)."""
import numpy as np
import pytest

import oracle
from paper_1204_5125_amd import inputs


def _mesh2(mu=0.8, N=(9, 9)):
    return oracle.Mesh(2, N, (5.0, 5.0), mu=mu)


def _mesh3(mu=0.6):
    return oracle.Mesh(3, (5, 4, 5), (5.0, 4.0, 5.0), mu=mu, bdir=np.ones(3) / np.sqrt(3))


MESHES = [_mesh2, _mesh3]


def test_constant_state_solves_zero_field():
    """psi = 1 solves the A = 0 problem (Sec. 3, the constant null vector)."""
    for dim in (2, 3):
        m = oracle.Mesh(dim, [6] * dim, [5.0] * dim, mu=0.0)
        assert np.abs(m.gl(np.ones(m.n))).max() < 1e-13


@pytest.mark.parametrize("mk", MESHES)
def test_gl_normal_state_and_gauge_covariance(mk):
    """GL(0) = 0 for any A; GL(exp(i chi) psi) = exp(i chi) GL(psi) (Sec. 2)."""
    m = mk()
    assert np.abs(m.gl(np.zeros(m.n))).max() == 0.0
    psi = inputs.random_complex(m.n, seed=3)
    g = m.gl(psi)
    chi = 1.234
    np.testing.assert_allclose(m.gl(np.exp(1j * chi) * psi), np.exp(1j * chi) * g,
                               rtol=1e-13, atol=1e-12)
    # <i psi, GL(psi)>_R = 0: GL is orthogonal to the gauge direction
    assert abs(m.inner(1j * psi, g)) < 1e-12 * m.norm(psi) * m.norm(g)


@pytest.mark.parametrize("mk", MESHES)
def test_gl_is_energy_gradient(mk):
    """Euler-Lagrange of the discrete energy: F(psi + e phi) - F(psi - e phi)
    = 4 e <GL(psi), phi>_R + O(e^3) (eqs. discr energy, discr ginla)."""
    m = mk()
    psi = inputs.random_complex(m.n, seed=4) * 0.7
    phi = inputs.random_complex(m.n, seed=5)
    eps = 1e-5
    fd = (m.energy(psi + eps * phi) - m.energy(psi - eps * phi)) / (4 * eps)
    an = m.inner(m.gl(psi), phi)
    assert fd == pytest.approx(an, rel=1e-7)


def test_energy_of_constant_state_zero_field():
    """F(1) = -|Omega| / 2 at A = 0 (mass lumping with psi = 1)."""
    m = oracle.Mesh(2, (7, 7), (5.0, 5.0), mu=0.0)
    assert m.energy(np.ones(m.n)) == pytest.approx(-12.5, rel=1e-14)


@pytest.mark.parametrize("mk", MESHES)
def test_jacobian_matches_finite_differences(mk):
    """J(psi) phi is the derivative of GL in direction phi (eq. jacobian)."""
    m = mk()
    psi = inputs.random_complex(m.n, seed=6)
    phi = inputs.random_complex(m.n, seed=7)
    eps = 1e-6
    fd = (m.gl(psi + eps * phi) - m.gl(psi - eps * phi)) / (2 * eps)
    jp = m.jac(psi, phi)
    assert np.abs(fd - jp).max() <= 1e-7 * np.abs(jp).max()


@pytest.mark.parametrize("mk", MESHES)
def test_jacobian_self_adjoint_real_linear(mk):
    """J(psi) is self-adjoint in <.,.>_R (eq. disc inner2), real-linear and
    not complex-linear."""
    m = mk()
    psi = inputs.random_complex(m.n, seed=8)
    u = inputs.random_complex(m.n, seed=9)
    v = inputs.random_complex(m.n, seed=10)
    a, b = m.inner(u, m.jac(psi, v)), m.inner(m.jac(psi, u), v)
    assert a == pytest.approx(b, rel=1e-12)
    np.testing.assert_allclose(m.jac(psi, 2.5 * u - 0.5 * v),
                               2.5 * m.jac(psi, u) - 0.5 * m.jac(psi, v), rtol=1e-12, atol=1e-11)
    assert np.abs(m.jac(psi, 1j * u) - 1j * m.jac(psi, u)).max() > 1e-3


@pytest.mark.parametrize("mk", MESHES)
def test_gauge_direction_identity(mk):
    """J(psi)(i psi) = i GL(psi) for every psi; at a solution it gives the
    gauge kernel J(psi_s)(i psi_s) = 0 (eq. jacobian nullspace)."""
    m = mk()
    psi = inputs.random_complex(m.n, seed=11)
    np.testing.assert_allclose(m.jac(psi, 1j * psi), 1j * m.gl(psi), rtol=1e-12, atol=1e-11)


def test_jacobian_at_constant_state_zero_field_spectrum():
    """psi = 1, A = 0: J phi = (K + 2) Re phi + i K Im phi, so the eigenvalues of
    J are the DCT-I values lambda_k and lambda_k + 2."""
    N, L = (6, 7), (3.0, 4.0)
    m = oracle.Mesh(2, N, L, mu=0.0)
    n = m.n
    one = np.ones(n, complex)
    cols = []
    for k in range(n):
        e = np.zeros(n, complex); e[k] = 1.0
        cols.append(m.jac(one, e))
    for k in range(n):
        e = np.zeros(n, complex); e[k] = 1j
        cols.append(m.jac(one, e))
    Jr = np.array([np.concatenate([c.real, c.imag]) for c in cols]).T
    ev = np.sort(np.linalg.eigvals(Jr).real)
    h = np.array(L) / (np.array(N) - 1)
    lam = np.add.outer(4 / h[0] ** 2 * np.sin(np.pi * np.arange(N[0]) / (2 * (N[0] - 1))) ** 2,
                       4 / h[1] ** 2 * np.sin(np.pi * np.arange(N[1]) / (2 * (N[1] - 1))) ** 2).ravel()
    np.testing.assert_allclose(ev, np.sort(np.concatenate([lam, lam + 2])), rtol=1e-10, atol=1e-10)


def test_preconditioner_matrix_hermitian_definite():
    """H = K-hat + 2 D |psi|^2 is Hermitian positive definite except for
    psi = 0 with A = 0 (Sec. 4.1)."""
    m = _mesh2(mu=0.0)
    H0 = m.hmat(np.zeros(m.n)).toarray()
    assert abs(np.linalg.eigvalsh(H0).min()) < 1e-12
    psi = inputs.random_phase_state(m.n, seed=1)
    H = m.hmat(psi).toarray()
    assert np.array_equal(H, H.conj().T)
    assert np.linalg.eigvalsh(H).min() > 1e-3
    m2 = _mesh2(mu=0.8)
    assert np.linalg.eigvalsh(m2.hmat(np.zeros(m2.n)).toarray()).min() > 1e-3
