"""Pins of the oracle's smoothed-aggregation AMG (Sec. 4.1 preconditioner).

The paper fixes smoothed aggregation, 1+1 symmetric Gauss-Seidel and a
Hermitian AMG_k; the remaining choices are readings (oracle/amg.c header).
These tests check every reading against an independent statement of it:
parallel-round versions of the greedy algorithms, dense linear algebra for
the transfer and Galerkin operators, and operator properties of the V-cycle.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_1204_5125_amd import inputs


def fmix32(h):
    h = np.uint64(h) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    return int(h)


def keys(n):
    """Aggregation priority: the smaller index first."""
    return [n - i for i in range(n)]


def colour_keys(nb):
    """Colour priority: the smaller index first."""
    return [len(nb) - i for i in range(len(nb))]


def iterated_greedy(nb, col, passes=2):
    """Greedy again with the vertices taken a colour class at a time, the
    classes in reverse order (Culberson's iterated greedy), `passes` times."""
    col = list(col)
    for _ in range(passes):
        new = [-1] * len(nb)
        for c in range(max(col), -1, -1):
            for i in range(len(nb)):
                if col[i] == c:
                    used = {new[j] for j in nb[i]}
                    k = 0
                    while k in used:
                        k += 1
                    new[i] = k
        col = new
    return col


def power_rho(A, d, steps=20):
    """rho(D^-1 A) estimated by power iteration from the start
    s_i = (h1_i - 1/2) + i (h2_i - 1/2), h = fmix32(i ^ salt) / 2^32."""
    n = A.shape[0]
    x = np.array([fmix32(i ^ 0x2545F491) / 2.0 ** 32 - 0.5 + 1j * (fmix32(i ^ 0x6C8E9CF5) / 2.0 ** 32 - 0.5)
                  for i in range(n)])
    rho = 0.0
    for _ in range(steps):
        y = (A @ x) / d
        rho = np.linalg.norm(y) / np.linalg.norm(x)
        x = y / np.linalg.norm(y)
    return rho


def neighbours(A):
    A = sp.csr_matrix(A)
    return [[j for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j != i] for i in range(A.shape[0])]


def parallel_mis2(nb, key):
    """Rounds: an undecided node joins when its key is the largest among the
    undecided nodes within distance 2; nodes within distance 2 of a new root
    are removed."""
    n = len(nb)
    state = [0] * n  # 0 undecided, 1 root, 2 removed
    while any(s == 0 for s in state):
        ball2 = []
        for i in range(n):
            b = {i} | set(nb[i])
            for j in nb[i]:
                b |= set(nb[j])
            ball2.append(b)
        new = [i for i in range(n) if state[i] == 0 and
               all(key[i] >= key[j] for j in ball2[i] if state[j] == 0)]
        for i in new:
            state[i] = 1
        for i in new:
            for j in ball2[i]:
                if state[j] == 0:
                    state[j] = 2
    return sorted(i for i in range(n) if state[i] == 1)


def jones_plassmann(nb, key):
    n = len(nb)
    col = [-1] * n
    while any(c < 0 for c in col):
        ready = [i for i in range(n) if col[i] < 0 and
                 all(col[j] >= 0 or key[j] < key[i] for j in nb[i])]
        for i in ready:
            used = {col[j] for j in nb[i] if col[j] >= 0}
            c = 0
            while c in used:
                c += 1
            col[i] = c
    return col


def hierarchy_cases():
    m2 = oracle.Mesh(2, (17, 17), (5.0, 5.0), mu=0.8)
    m3 = oracle.Mesh(3, (6, 6, 6), (5.0, 5.0, 5.0), mu=0.6, bdir=np.ones(3) / np.sqrt(3))
    return [(m2, inputs.random_phase_state(m2.n, seed=0)),
            (m3, inputs.random_phase_state(m3.n, seed=1))]


@pytest.fixture(scope="module")
def hierarchies():
    out = []
    for m, psi in hierarchy_cases():
        out.append((m, psi, oracle.Amg.for_state(m, psi, max_coarse=10)))
    return out


def test_aggregation_invariants(hierarchies):
    """Aggregates partition the nodes, roots are pairwise at distance >= 3, every
    node lies within distance 2 of its root, and numbering follows the roots."""
    for m, psi, amg in hierarchies:
        assert amg.nlev >= 3
        for l, L in enumerate(amg.levels[:-1]):
            agg, root, n, nc = L["agg"], L["root"], L["n"], L["nc"]
            assert agg.min() >= 0 and agg.max() == nc - 1
            assert np.all(np.diff(root) > 0)
            assert np.array_equal(agg[root], np.arange(nc))
            G = L["A"].copy()
            G.setdiag(0)
            G.eliminate_zeros()
            G = sp.csr_matrix((np.ones(G.nnz), G.indices, G.indptr), shape=G.shape)
            D = shortest_path(G, unweighted=True, indices=root)
            Dr = D[:, root]
            np.fill_diagonal(Dr, np.inf)
            assert Dr.min() >= 3
            assert np.all(D[agg, np.arange(n)] <= 2)
            assert np.all(D.min(axis=0) <= 2)


def test_mis2_greedy_equals_parallel_rounds(hierarchies):
    """The serial greedy (ascending index) roots equal the roots of the
    parallel rounds with the same priorities, on every level."""
    for m, psi, amg in hierarchies:
        for l, L in enumerate(amg.levels[:-1]):
            if L["n"] > 400:
                continue
            nb = neighbours(L["A"])
            roots = parallel_mis2(nb, keys(L["n"]))
            assert roots == list(L["root"])


def test_aggregate_assignment_rules(hierarchies):
    """Phase A: neighbours of a root join it.  Phase B: the rest join the
    phase-A neighbour whose root has the smallest index."""
    for m, psi, amg in hierarchies:
        for l, L in enumerate(amg.levels[:-1]):
            nb = neighbours(L["A"])
            key = keys(L["n"])
            root = set(L["root"].tolist())
            rootA = {}
            for i in range(L["n"]):
                if i in root:
                    rootA[i] = i
                else:
                    rs = [j for j in nb[i] if j in root]
                    assert len(rs) <= 1
                    if rs:
                        rootA[i] = rs[0]
            root_of = np.full(L["n"], -1)
            for i in range(L["n"]):
                if i in rootA:
                    root_of[i] = rootA[i]
                else:
                    cands = [rootA[j] for j in nb[i] if j in rootA]
                    root_of[i] = max(cands, key=lambda r: key[r])
            idx = {r: a for a, r in enumerate(L["root"])}
            assert np.array_equal(L["agg"], np.array([idx[r] for r in root_of]))


def test_colouring_proper_and_greedy(hierarchies):
    """Level 0 of a grid: red-black parity; coarser levels: proper colourings
    equal to Jones-Plassmann rounds with the colour priorities followed by two
    iterated-greedy passes, with no more colours than the rounds alone."""
    for m, psi, amg in hierarchies:
        L0 = amg.levels[0]
        idx = np.stack(np.unravel_index(np.arange(m.n), m.N[::-1])[::-1], axis=1)
        assert np.array_equal(L0["color"], idx.sum(axis=1) % 2)
        for l, L in enumerate(amg.levels):
            A = sp.coo_matrix(L["A"])
            off = A.row != A.col
            assert np.all(L["color"][A.row[off]] != L["color"][A.col[off]])
            assert L["ncolors"] == L["color"].max() + 1
            if l > 0 and L["n"] <= 400:
                nb = neighbours(L["A"])
                jp = jones_plassmann(nb, colour_keys(nb))
                assert iterated_greedy(nb, jp) == list(L["color"])
                assert L["ncolors"] <= max(jp) + 1


def test_transfer_and_galerkin_operators(hierarchies):
    """P = T - omega D^-1 A T with T = 1/sqrt(|a|) on the aggregates and
    omega = (4/3)/rho~, rho~ the 20-step power-iteration estimate of
    rho(D^-1 A) from the counter-hash start, a lower bound of the true spectral
    radius within a few per cent; R = P^H; A_{l+1} = R A P exactly
    Hermitian with real diagonal; pattern of P = pattern of T u A T."""
    for m, psi, amg in hierarchies:
        for l, L in enumerate(amg.levels[:-1]):
            A = L["A"].toarray()
            n, nc = L["n"], L["nc"]
            T = np.zeros((n, nc))
            sizes = np.bincount(L["agg"], minlength=nc)
            T[np.arange(n), L["agg"]] = 1 / np.sqrt(sizes[L["agg"]])
            d = np.diag(A).real
            rho = power_rho(A, d)
            assert L["omega"] == pytest.approx(4 / 3 / rho, rel=1e-12)
            true_rho = np.abs(np.linalg.eigvals(A / d[:, None])).max()
            assert 0.9 * true_rho <= rho <= true_rho * (1 + 1e-12)
            P = T - (L["omega"] / d)[:, None] * (A @ T)
            np.testing.assert_allclose(L["P"].toarray(), P, rtol=1e-12, atol=1e-13)
            struct = ((np.abs(A) > 0).astype(int) @ (T > 0).astype(int) + (T > 0)) > 0
            assert np.array_equal(L["P"].toarray() != 0, struct) or \
                np.array_equal(sp.csr_matrix(struct.astype(float)).indices, L["P"].indices)
            assert np.array_equal(L["R"].toarray(), L["P"].toarray().conj().T)
            Ac = amg.levels[l + 1]["A"].toarray()
            np.testing.assert_allclose(Ac, P.conj().T @ A @ P, rtol=1e-11, atol=1e-12 * np.abs(Ac).max())
            assert np.array_equal(Ac, Ac.conj().T)


def test_sgs_is_symmetric_gauss_seidel(hierarchies):
    """One sweep from x = 0 equals (D+U)^-1 D (D+L)^-1 b in the colour order,
    the symmetric Gauss-Seidel operator."""
    m, psi, amg = hierarchies[0]
    for l in (0, 1):
        L = amg.levels[l]
        A = L["A"].toarray()
        perm = np.argsort(L["color"], kind="stable")
        Ap = A[np.ix_(perm, perm)]
        Dg = np.diag(np.diag(Ap))
        Lo, Up = np.tril(Ap, -1), np.triu(Ap, 1)
        S = np.linalg.solve(Dg + Up, Dg @ np.linalg.inv(Dg + Lo))
        b = inputs.random_complex(L["n"], seed=l)
        x = amg.sgs(l, np.zeros(L["n"]), b)
        np.testing.assert_allclose(x[perm], S @ b[perm], rtol=1e-11, atol=1e-12)


def vcycle_matrix(amg, n, cycles=1):
    cols = []
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1.0
        cols.append(amg.solve(e, cycles))
    return np.array(cols).T


def test_vcycle_hermitian_positive_definite_contracting():
    """AMG_1 is Hermitian (Sec. 4.1) and positive definite; the two-level
    error propagator I - V H contracts."""
    m = oracle.Mesh(2, (9, 9), (5.0, 5.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=0)
    amg = oracle.Amg.for_state(m, psi, max_coarse=20)
    assert amg.nlev == 2
    H = m.hmat(psi).toarray()
    V = vcycle_matrix(amg, m.n)
    assert np.abs(V - V.conj().T).max() < 1e-13 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.conj().T)).min() > 0
    rho = np.abs(np.linalg.eigvals(np.eye(m.n) - V @ H)).max()
    assert rho < 0.5


def dense_vcycle(amg, l):
    """The V-cycle of level l as a dense matrix, restated from its definition
    (Sec. 4.1: one pre- and one post-smoothing symmetric Gauss-Seidel sweep
    around the coarse correction): with S = (D+U)^-1 D (D+L)^-1 in the colour
    order (one sweep, x += S (b - A x)), x1 = S b, x2 = x1 + P B_{l+1} R (b - A x1),
    x3 = x2 + S (b - A x2); the last level is A^-1.  Uses only the stored
    operators, transfers and colours."""
    L = amg.levels[l]
    A = L["A"].toarray()
    n = A.shape[0]
    if l == amg.nlev - 1:
        return np.linalg.inv(A)
    perm = np.argsort(L["color"], kind="stable")
    Ap = A[np.ix_(perm, perm)]
    Dg = np.diag(np.diag(Ap))
    Sp = np.linalg.solve(Dg + np.triu(Ap, 1), Dg @ np.linalg.inv(Dg + np.tril(Ap, -1)))
    S = np.zeros_like(Sp)
    S[np.ix_(perm, perm)] = Sp
    P, R = L["P"].toarray(), L["R"].toarray()
    Bc = dense_vcycle(amg, l + 1)
    I = np.eye(n)
    X1 = S
    X2 = X1 + P @ Bc @ R @ (I - A @ X1)
    return X2 + S @ (I - A @ X2)


@pytest.mark.parametrize("grid,max_coarse", [((17, 17), 8), ((13, 11), 6), ((7, 6, 5), 6)])
def test_deep_vcycle_operator(grid, max_coarse):
    """A hierarchy of at least three levels: the oracle's recursive V-cycle
    (columns from unit vectors) equals the dense restatement of the cycle,
    and it is Hermitian and positive definite (it is the preconditioner of
    MINRES, Sec. 4) with a contracting error propagator I - V H."""
    dim = len(grid)
    m = oracle.Mesh(dim, grid, (5.0,) * dim, mu=0.8, bdir=(0.3, 0.5, 1.0) if dim == 3 else (0, 0, 1))
    psi = inputs.random_phase_state(m.n, seed=7)
    amg = oracle.Amg.for_state(m, psi, max_coarse=max_coarse)
    assert amg.nlev >= 3
    V = vcycle_matrix(amg, m.n)
    Vd = dense_vcycle(amg, 0)
    assert np.abs(V - Vd).max() < 1e-12 * np.abs(Vd).max()
    assert np.abs(V - V.conj().T).max() < 1e-12 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.conj().T)).min() > 0
    H = m.hmat(psi).toarray()
    assert np.abs(np.linalg.eigvals(np.eye(m.n) - V @ H)).max() < 1.0


def test_single_level_is_exact_inverse():
    """A hierarchy with one level solves the coarse problem by Cholesky, i.e.
    applies H^-1 exactly."""
    m = oracle.Mesh(2, (6, 6), (5.0, 5.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=2)
    amg = oracle.Amg.for_state(m, psi, max_coarse=64)
    assert amg.nlev == 1
    H = m.hmat(psi).toarray()
    b = inputs.random_complex(m.n, seed=3)
    np.testing.assert_allclose(amg.solve(b), np.linalg.solve(H, b), rtol=1e-12, atol=1e-12)


def test_cycles_converge_to_inverse():
    """R_k -> R_inf = H^-1 D as k grows (eq. prec1; the paper's k = 10 is R_inf
    to machine precision)."""
    m = oracle.Mesh(2, (17, 17), (5.0, 5.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=4)
    amg = oracle.Amg.for_state(m, psi, max_coarse=10)
    H = m.hmat(psi).toarray()
    b = inputs.random_complex(m.n, seed=5)
    ref = np.linalg.solve(H, b)
    errs = [np.linalg.norm(amg.solve(b, k) - ref) / np.linalg.norm(ref) for k in (1, 2, 5, 40)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-12


def test_singular_preconditioner_detected():
    """psi = 0 with A = 0 makes H singular (Sec. 4.1): the coarse Cholesky fails."""
    m = oracle.Mesh(2, (9, 9), (5.0, 5.0), mu=0.0)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Amg.for_state(m, np.zeros(m.n))
    assert e.value.code == oracle.ORC_ERR_SINGULAR


def test_exact_preconditioner_is_the_limit_of_the_cycles():
    """R_inf = H^-1 D by a sparse direct solve (eq. prec1) equals the dense
    inverse, and R_k reaches it to 1e-12 as k grows (the paper's R_10 stands
    in for R_inf)."""
    m = oracle.Mesh(2, (17, 17), (5.0, 5.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=8)
    r = inputs.random_complex(m.n, seed=9)
    ex = oracle.precond_exact(m, psi, r)
    H = m.hmat(psi).toarray()
    np.testing.assert_allclose(ex, np.linalg.solve(H, m.vol * r), rtol=1e-12, atol=1e-13)
    amg = oracle.Amg.for_state(m, psi, max_coarse=10)
    errs = [np.abs(amg.precond(m, r, k) - ex).max() / np.abs(ex).max() for k in (1, 5, 40)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-12


def test_minres_with_exact_preconditioner():
    """MINRES with R_inf solves J x = b (dense check) and needs fewer
    iterations than with R_1 (Fig. 1: R_inf is the ideal SPD preconditioner)."""
    m = oracle.Mesh(2, (17, 17), (5.0, 5.0), mu=0.8)
    psi = inputs.random_phase_state(m.n, seed=10)
    b = inputs.random_complex(m.n, seed=11)
    x, info, _ = oracle.minres_exact_precond(m, psi, b, rtol=1e-12, max_iter=500)
    assert info["converged"]
    r = b - m.jac(psi, x)
    assert m.norm(r) < 1e-10 * m.norm(b)
    amg = oracle.Amg.for_state(m, psi, max_coarse=10)
    _, i1, _ = oracle.minres(m, psi, b, amg=amg, rtol=1e-12, max_iter=500)
    assert info["iterations"] < i1["iterations"]
