"""Pins of the oracle's pseudo-arclength continuation (Sec. 4, numerical
parameter continuation: predict along the curve, correct perpendicularly)."""
import numpy as np
import pytest

import oracle
from oracle import arclength as al
from oracle import continuation as oc
from paper_1204_5125_amd import inputs

N, L, B = (33, 33), (8.0, 8.0), (0, 0, 1)


def test_gl_dmu_is_the_parameter_derivative():
    """GL_mu against central differences of GL in mu (separate meshes), and
    orthogonal to the gauge mode (<i psi, GL(psi; mu)>_R = 0 for every mu)."""
    for dim, n_ax, side, bdir, mu in (((2, (13, 11), (5.0, 4.0), (0, 0, 1), 0.7)),
                                      ((3, (7, 6, 5), (3.0, 2.5, 2.0), (0.3, 0.5, 1.0), 0.9))):
        bdir = np.asarray(bdir) / np.linalg.norm(bdir)
        m = oracle.Mesh(dim, n_ax, side, mu=mu, bdir=bdir)
        psi = inputs.random_complex(m.n, seed=51)
        eps = 1e-5
        fd = (oracle.Mesh(dim, n_ax, side, mu=mu + eps, bdir=bdir).gl(psi)
              - oracle.Mesh(dim, n_ax, side, mu=mu - eps, bdir=bdir).gl(psi)) / (2 * eps)
        an = al.gl_dmu(m, psi, bdir)
        assert np.abs(fd - an).max() < 1e-9 * np.abs(an).max()
        assert abs(m.inner(1j * psi, an)) < 1e-13 * m.norm(an) * m.norm(psi)


def test_tangent_is_unit_and_annihilated_by_the_bordered_jacobian():
    """At a solution the tangent (t_psi, t_mu) has unit arclength norm,
    points towards growing mu, and J t_psi + GL_mu t_mu is a multiple of the
    gauge mode i psi (zero on its complement)."""
    m = oracle.Mesh(2, N, L, mu=0.3, bdir=B)
    psi, info = oracle.newton(m, np.ones(m.n, complex), tol=1e-12, max_steps=20, krylov_rtol=1e-12,
                              deflate=True)
    assert info["converged"]
    area = 64.0
    tp, tm = al.tangent_at(m, psi, B, area, krylov_rtol=1e-13)
    assert m.inner(tp, tp) / area + tm * tm == pytest.approx(1.0, rel=1e-12)
    assert tm > 0
    r = m.jac(psi, tp) + tm * al.gl_dmu(m, psi, B)
    u = 1j * psi
    pr = r - u * m.inner(u, r) / m.inner(u, u)
    assert m.norm(pr) < 1e-10 * m.norm(tp)


def test_arclength_agrees_with_natural_continuation_away_from_folds():
    """The first points of the path (mu < 0.3, far below the fold) are the
    states Newton finds at the same mu from psi = 1."""
    recs, states = al.arclength(2, N, L, B, np.ones(33 * 33, complex), 0.0, 0.1, 3)
    assert all(r["converged"] for r in recs)
    for mu, p in states[1:]:
        assert 0.0 < mu < 0.3
        m = oracle.Mesh(2, N, L, mu=mu, bdir=B)
        q, info = oracle.newton(m, np.ones(m.n, complex), tol=1e-12, max_steps=30, krylov_rtol=1e-12)
        assert info["converged"]
        chi = np.angle(np.vdot(p, q))
        assert np.abs(p * np.exp(1j * chi) - q).max() < 1e-9


def test_arclength_passes_the_fold_where_natural_continuation_jumps():
    """The Meissner branch of the 33 x 33, side-8 square ends in a fold near
    mu = 0.707.  Pseudo-arclength follows it round the turning point: mu
    rises, reaches its maximum and falls again, every point converges in a
    few Newton steps, consecutive points are about one step ds apart along
    the curve (no jump).  Natural continuation in steps of 0.05 steps past
    the fold to mu = 0.75, where Newton wanders for many steps and lands on
    a state far from every point of the traced branch."""
    ds = 0.1
    recs, states = al.arclength(2, N, L, B, np.ones(33 * 33, complex), 0.0, ds, 19)
    assert all(r["converged"] for r in recs)
    assert max(r["newton_steps"] for r in recs[1:]) <= 6
    mus = np.array([mu for mu, _ in states])
    k = int(np.argmax(mus))
    assert 0 < k < len(mus) - 3
    assert 0.70 < mus[k] < 0.72
    assert np.all(np.diff(mus[:k + 1]) > 0) and np.all(np.diff(mus[k:]) < 0)
    area = 64.0
    for (m0, p0), (m1, p1), r in zip(states[:-1], states[1:], recs[1:]):
        ph = np.vdot(p0, p1)
        d = p1 - p0 * ph / abs(ph)
        step = np.sqrt(np.sum(oracle.Mesh(2, N, L, mu=m1, bdir=B).vol * np.abs(d) ** 2) / area + (m1 - m0) ** 2)
        assert step < 2 * ds
    nrec, npsi = oc.continuation(2, N, L, B, np.ones(33 * 33, complex), 0.0, 0.05, 15)
    assert abs(nrec[-1]["mu"] - 0.75) < 1e-12 and nrec[-1]["newton_steps"] >= 10
    dist = min(np.abs(npsi * np.exp(1j * np.angle(np.vdot(npsi, p))) - p).max() for _, p in states)
    assert dist > 0.1
