"""Python access to the plain FP64 C oracle (ctypes + numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and
by the CPU-baseline leg of bench.py.  The GPU library never imports it.

Every array crossing this boundary is a host numpy array (complex128 for
states, float64 / int64 for geometry and indices).
"""
import ctypes as C

import numpy as np
import scipy.sparse as sp

from . import build as _build

_lib = None

ORC_OK, ORC_ERR_ARG, ORC_ERR_SINGULAR, ORC_ERR_BREAKDOWN, ORC_ERR_NOT_CONVERGED, \
    ORC_ERR_AGGREGATION = range(6)
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "singular", 3: "breakdown",
                4: "not converged", 5: "aggregation failed"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS_NAMES.get(code, code)}")
        self.code = code


_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("N", C.c_int64 * 3), ("L", C.c_double * 3),
                ("h", C.c_double * 3), ("amat", C.c_double * 9), ("n", C.c_int64),
                ("x", _d), ("vol", _d), ("ne", C.c_int64), ("ej", _i64), ("ek", _i64),
                ("alpha", _d), ("U", _d), ("rp", _i64), ("ci", _i64), ("kv", _d), ("grid", C.c_int)]


class _Level(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rp", _i64), ("ci", _i64), ("v", _d),
                ("nc", C.c_int64), ("agg", _i64), ("root", _i64), ("prp", _i64), ("pci", _i64),
                ("pv", _d), ("rrp", _i64), ("rci", _i64), ("rv", _d),
                ("color", C.POINTER(C.c_int32)), ("ncolors", C.c_int), ("omega", C.c_double)]


class _Amg(C.Structure):
    _fields_ = [("nlev", C.c_int), ("lev", _Level * 16), ("chol", _d),
                ("grid_N", C.c_int64 * 3), ("grid_dim", C.c_int)]


class _KInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("eta0", C.c_double),
                ("eta", C.c_double), ("res_true", C.c_double)]


class _NInfo(C.Structure):
    _fields_ = [("steps", C.c_int), ("converged", C.c_int), ("res", C.c_double * 64),
                ("krylov_iters", C.c_int * 64), ("alpha", C.c_double * 64)]


_OP = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_mesh_build.argtypes = [C.c_int, _i64, _d, _d, C.POINTER(C.POINTER(_Mesh))]
        L.orc_mesh_build_dipole.argtypes = [C.c_int, _i64, _d, C.c_double, _d, _d, C.POINTER(C.POINTER(_Mesh))]
        L.orc_mesh_build_tri.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, _d, C.POINTER(C.POINTER(_Mesh))]
        L.orc_mesh_build_tri_dipole.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_double, _d, _d,
                                                C.POINTER(C.POINTER(_Mesh))]
        L.orc_mesh_build_tet.argtypes = L.orc_mesh_build_tri.argtypes
        L.orc_mesh_build_tet_dipole.argtypes = L.orc_mesh_build_tri_dipole.argtypes
        L.orc_mesh_free.argtypes = [C.POINTER(_Mesh)]
        for f in ("orc_khat_apply",):
            getattr(L, f).argtypes = [C.POINTER(_Mesh), vp, vp]
        L.orc_gl.argtypes = [C.POINTER(_Mesh), vp, vp]
        L.orc_jac.argtypes = [C.POINTER(_Mesh), vp, vp, vp]
        L.orc_inner.argtypes = [C.POINTER(_Mesh), vp, vp]
        L.orc_inner.restype = C.c_double
        L.orc_energy.argtypes = [C.POINTER(_Mesh), vp]
        L.orc_energy.restype = C.c_double
        L.orc_hmat_values.argtypes = [C.POINTER(_Mesh), vp, vp]
        L.orc_amg_build.argtypes = [C.c_int64, vp, vp, vp, C.c_int, vp, C.c_int, C.c_int,
                                    C.POINTER(C.POINTER(_Amg))]
        L.orc_amg_free.argtypes = [C.POINTER(_Amg)]
        L.orc_amg_solve.argtypes = [C.POINTER(_Amg), vp, vp, C.c_int]
        L.orc_sgs.argtypes = [C.POINTER(_Level), vp, vp]
        L.orc_minres.argtypes = [C.POINTER(_Mesh), vp, C.POINTER(_Amg), C.c_int, vp, vp,
                                 C.c_double, C.c_int, C.c_int, vp, C.POINTER(_KInfo)]
        L.orc_minres_generic.argtypes = [C.c_int64, vp, _OP, vp, _OP, vp, vp, vp, C.c_double,
                                         C.c_int, vp, C.POINTER(_KInfo)]
        L.orc_minres_reorth_generic.argtypes = [C.c_int64, vp, _OP, vp, _OP, vp, vp, vp, C.c_double,
                                                C.c_int, C.c_int, vp, C.POINTER(_KInfo)]
        L.orc_minres_deflated.argtypes = L.orc_minres.argtypes
        L.orc_newton.argtypes = [C.POINTER(_Mesh), vp, C.c_double, C.c_int, C.c_int, C.c_double,
                                 C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 C.POINTER(_NInfo)]
        _lib = L
    return _lib


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _arr(ptr, count, dtype):
    if count == 0:
        return np.zeros(0, dtype=dtype)
    if dtype == np.complex128:
        raw = np.ctypeslib.as_array(C.cast(ptr, _d), shape=(2 * count,))
        return raw.view(np.complex128).copy()
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


def field_matrix(mu, bdir=(0.0, 0.0, 1.0)):
    """3x3 matrix M with A(r) = M r = mu/2 (b x r): the uniform-field potential
    (Sec. 4 experiments use A_z = (-y, x, 0)/2, i.e. b = e_z, mu = 1)."""
    b = np.asarray(bdir, dtype=np.float64)
    cross = np.array([[0.0, -b[2], b[1]], [b[2], 0.0, -b[0]], [-b[1], b[0], 0.0]])
    return 0.5 * mu * cross


class Mesh:
    """Tensor grid on [-L/2, L/2]^dim with Voronoi volumes, edge coefficients,
    link variables and K-hat (Sec. 3)."""

    def __init__(self, dim, N, L, amat=None, mu=None, bdir=(0.0, 0.0, 1.0), dipole=None):
        """dipole = (m, x0): the potential mu A_d(x) = mu m x (x - x0) / |x - x0|^3
        (Sec. 4.1) instead of a linear one."""
        if amat is None:
            amat = field_matrix(0.0 if mu is None else mu, bdir) if dipole is None else np.zeros((3, 3))
        N = list(N) + [1] * (3 - len(N))
        L = list(L) + [0.0] * (3 - len(L))
        Na = (C.c_int64 * 3)(*N)
        La = (C.c_double * 3)(*L)
        am = (C.c_double * 9)(*np.asarray(amat, dtype=np.float64).ravel())
        p = C.POINTER(_Mesh)()
        if dipole is not None:
            dm = (C.c_double * 3)(*[float(v) for v in dipole[0]])
            dx = (C.c_double * 3)(*[float(v) for v in dipole[1]])
            rc = lib().orc_mesh_build_dipole(dim, Na, La, 1.0 if mu is None else float(mu), dm, dx, C.byref(p))
        else:
            rc = lib().orc_mesh_build(dim, Na, La, am, C.byref(p))
        if rc != ORC_OK:
            raise OracleError(rc, "orc_mesh_build")
        self._adopt(p, amat)

    @classmethod
    def simplices(cls, x, cells, amat=None, mu=None, bdir=(0.0, 0.0, 1.0), dipole=None):
        """Simplicial mesh: nodes x (n x 2 or n x 3), cells (m x 3 triangles
        or m x 4 tetrahedra); edge coefficients by the Corollary's system per
        simplex, control volumes as the nodes' shares of their simplices
        (oracle/oracle.h)."""
        if amat is None:
            amat = field_matrix(0.0 if mu is None else mu, bdir) if dipole is None else np.zeros((3, 3))
        x = np.ascontiguousarray(x, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        dim = x.shape[1]
        if dim not in (2, 3) or cells.ndim != 2 or cells.shape[1] != dim + 1:
            raise ValueError("x must be n x 2 with triangles or n x 3 with tetrahedra")
        name = "orc_mesh_build_tri" if dim == 2 else "orc_mesh_build_tet"
        p = C.POINTER(_Mesh)()
        if dipole is not None:
            dm = (C.c_double * 3)(*[float(v) for v in dipole[0]])
            dx = (C.c_double * 3)(*[float(v) for v in dipole[1]])
            rc = getattr(lib(), name + "_dipole")(len(x), _ptr(x), len(cells), _ptr(cells),
                                                  1.0 if mu is None else float(mu), dm, dx, C.byref(p))
        else:
            am = (C.c_double * 9)(*np.asarray(amat, dtype=np.float64).ravel())
            rc = getattr(lib(), name)(len(x), _ptr(x), len(cells), _ptr(cells), am, C.byref(p))
        if rc != ORC_OK:
            raise OracleError(rc, name)
        self = cls.__new__(cls)
        self._adopt(p, amat)
        self.cells = cells.copy()
        return self

    triangles = simplices

    def _adopt(self, p, amat):
        self._p = p
        m = p.contents
        dim = m.dim
        self.grid = bool(m.grid)
        self.dim, self.n, self.ne = dim, m.n, m.ne
        self.N = tuple(m.N[:dim]) if self.grid else None
        self.h = tuple(m.h[:dim]) if self.grid else None
        self.Lside = tuple(m.L[:dim]) if self.grid else None
        self.amat = np.array(amat, dtype=np.float64).reshape(3, 3)
        self.x = _arr(m.x, 3 * m.n, np.float64).reshape(m.n, 3)
        self.vol = _arr(m.vol, m.n, np.float64)
        self.ej = _arr(m.ej, m.ne, np.int64)
        self.ek = _arr(m.ek, m.ne, np.int64)
        self.alpha = _arr(m.alpha, m.ne, np.float64)
        self.U = _arr(m.U, m.ne, np.complex128)
        nnz = m.rp[m.n]
        self.khat = sp.csr_matrix((_arr(m.kv, nnz, np.complex128), _arr(m.ci, nnz, np.int64),
                                   _arr(m.rp, m.n + 1, np.int64)), shape=(m.n, m.n))

    def __del__(self):
        if getattr(self, "_p", None) is not None and _lib is not None:
            _lib.orc_mesh_free(self._p)
            self._p = None

    def _unary(self, fn, x):
        x = _c128(x)
        y = np.empty_like(x)
        fn(self._p, _ptr(x), _ptr(y))
        return y

    def khat_apply(self, x):
        return self._unary(lib().orc_khat_apply, x)

    def gl(self, psi):
        return self._unary(lib().orc_gl, psi)

    def jac(self, psi, phi):
        psi, phi = _c128(psi), _c128(phi)
        y = np.empty_like(phi)
        lib().orc_jac(self._p, _ptr(psi), _ptr(phi), _ptr(y))
        return y

    def inner(self, u, v):
        u, v = _c128(u), _c128(v)
        return lib().orc_inner(self._p, _ptr(u), _ptr(v))

    def norm(self, u):
        return float(np.sqrt(self.inner(u, u)))

    def energy(self, psi):
        psi = _c128(psi)
        return lib().orc_energy(self._p, _ptr(psi))

    def hmat(self, psi):
        """H = K-hat + 2 D |psi|^2 as CSR (same pattern as K-hat)."""
        psi = _c128(psi)
        hv = np.empty(self.khat.nnz, dtype=np.complex128)
        lib().orc_hmat_values(self._p, _ptr(psi), _ptr(hv))
        return sp.csr_matrix((hv, self.khat.indices.copy(), self.khat.indptr.copy()),
                             shape=self.khat.shape)


class Amg:
    """Smoothed-aggregation hierarchy of a Hermitian positive definite CSR
    matrix (oracle reading of Sec. 4.1; see oracle/amg.c)."""

    def __init__(self, A, grid_N=None, max_coarse=64, max_levels=16):
        A = sp.csr_matrix(A, dtype=np.complex128)
        A.sort_indices()
        n = A.shape[0]
        rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        ci = np.ascontiguousarray(A.indices, dtype=np.int64)
        v = _c128(A.data)
        gdim = 0 if grid_N is None else len(grid_N)
        gN = np.ascontiguousarray(list(grid_N or []) + [1] * (3 - gdim), dtype=np.int64)
        p = C.POINTER(_Amg)()
        rc = lib().orc_amg_build(n, _ptr(rp), _ptr(ci), _ptr(v), gdim, _ptr(gN), max_coarse,
                                 max_levels, C.byref(p))
        if rc != ORC_OK:
            raise OracleError(rc, "orc_amg_build")
        self._p = p
        self.n = n
        a = p.contents
        self.nlev = a.nlev
        self.levels = []
        for l in range(a.nlev):
            L = a.lev[l]
            nnz = L.rp[L.n]
            d = {"n": L.n, "ncolors": L.ncolors, "omega": L.omega,
                 "A": sp.csr_matrix((_arr(L.v, nnz, np.complex128), _arr(L.ci, nnz, np.int64),
                                     _arr(L.rp, L.n + 1, np.int64)), shape=(L.n, L.n)),
                 "color": _arr(L.color, L.n, np.int32), "nc": L.nc}
            if l < a.nlev - 1:
                pn = L.prp[L.n]
                d["agg"] = _arr(L.agg, L.n, np.int64)
                d["root"] = _arr(L.root, L.nc, np.int64)
                d["P"] = sp.csr_matrix((_arr(L.pv, pn, np.complex128), _arr(L.pci, pn, np.int64),
                                        _arr(L.prp, L.n + 1, np.int64)), shape=(L.n, L.nc))
                d["R"] = sp.csr_matrix((_arr(L.rv, pn, np.complex128), _arr(L.rci, pn, np.int64),
                                        _arr(L.rrp, L.nc + 1, np.int64)), shape=(L.nc, L.n))
            self.levels.append(d)

    @classmethod
    def for_state(cls, mesh, psi, **kw):
        """Hierarchy of H = K-hat + 2 D |psi|^2 on a grid mesh (red-black level 0)."""
        return cls(mesh.hmat(psi), grid_N=mesh.N if mesh.grid else None, **kw)

    def __del__(self):
        if getattr(self, "_p", None) is not None and _lib is not None:
            _lib.orc_amg_free(self._p)
            self._p = None

    def solve(self, b, cycles=1):
        """x = AMG_k(A_0, b), k = cycles V-cycles from x = 0."""
        b = _c128(b)
        x = np.empty_like(b)
        lib().orc_amg_solve(self._p, _ptr(b), _ptr(x), cycles)
        return x

    def precond(self, mesh, r, cycles=1):
        """R_k(psi) r = AMG_k(H, D r) (eq. prec2)."""
        return self.solve(mesh.vol * _c128(r), cycles)

    def sgs(self, level, x, b):
        x = _c128(x).copy()
        b = _c128(b)
        lib().orc_sgs(C.byref(self._p.contents.lev[level]), _ptr(x), _ptr(b))
        return x


def precond_exact(mesh, psi, r):
    """R_inf(psi) r = H^-1 D r with H = K-hat + 2 D |psi|^2 (eq. prec1): the
    preconditioner the V-cycles approximate, by a sparse direct solve."""
    import scipy.sparse.linalg as spla
    H = mesh.hmat(psi).tocsc()
    return spla.spsolve(H, mesh.vol * _c128(r))


def minres_exact_precond(mesh, psi, b, rtol=1e-10, max_iter=1000):
    """MINRES for J(psi) x = b preconditioned by R_inf (one sparse LU of H,
    reused for every application).  Returns (x, info, history)."""
    import scipy.sparse.linalg as spla
    psi = _c128(psi)
    lu = spla.splu(mesh.hmat(psi).tocsc())
    return minres_generic(mesh.vol, lambda x: mesh.jac(psi, x), b,
                          minv=lambda r: lu.solve(mesh.vol * r), rtol=rtol, max_iter=max_iter)


def _kinfo(ki):
    return {"iterations": ki.iterations, "converged": bool(ki.converged), "eta0": ki.eta0,
            "eta": ki.eta, "res_true": ki.res_true}


def minres(mesh, psi, b, amg=None, cycles=1, rtol=1e-10, max_iter=1000, deflate=False, reorth=0):
    """MINRES for J(psi) x = b in the D-weighted real product, preconditioned
    by R_k = AMG_k(H, D .) when amg is given; with deflate, on the complement
    of the gauge mode i psi (orc_minres_deflated); with reorth > 0, the
    Krylov basis (at most reorth vectors) stored and reorthogonalised in
    every step.  Returns (x, info, history)."""
    psi, b = _c128(psi), _c128(b)
    x = np.empty_like(b)
    hist = np.zeros(max_iter + 1)
    ki = _KInfo()
    fn = lib().orc_minres_deflated if deflate else lib().orc_minres
    rc = fn(mesh._p, _ptr(psi), amg._p if amg is not None else None, cycles,
            _ptr(b), _ptr(x), rtol, max_iter, int(reorth), _ptr(hist), C.byref(ki))
    info = _kinfo(ki)
    info["status"] = rc
    return x, info, hist[:ki.iterations + 1].copy()


def minres_generic(w, A, b, minv=None, rtol=1e-10, max_iter=1000, reorth=0):
    """MINRES for a callable A (self-adjoint in Re sum w conj(u) v) with an
    optional SPD callable preconditioner minv; reorth > 0 as in minres."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    b = _c128(b)
    n = b.size

    def wrap(f):
        def cb(ctx, xp, yp):
            xa = np.ctypeslib.as_array(C.cast(xp, _d), shape=(2 * n,)).view(np.complex128)
            ya = np.ctypeslib.as_array(C.cast(yp, _d), shape=(2 * n,)).view(np.complex128)
            ya[:] = f(xa.copy())
        return _OP(cb)

    Acb = wrap(A)
    Mcb = wrap(minv) if minv is not None else _OP()
    x = np.empty_like(b)
    hist = np.zeros(max_iter + 1)
    ki = _KInfo()
    if reorth > 0:
        rc = lib().orc_minres_reorth_generic(n, _ptr(w), Acb, None, Mcb, None, _ptr(b), _ptr(x), rtol,
                                             max_iter, int(reorth), _ptr(hist), C.byref(ki))
    else:
        rc = lib().orc_minres_generic(n, _ptr(w), Acb, None, Mcb, None, _ptr(b), _ptr(x), rtol,
                                      max_iter, _ptr(hist), C.byref(ki))
    info = _kinfo(ki)
    info["status"] = rc
    return x, info, hist[:ki.iterations + 1].copy()


def newton(mesh, psi0, tol=1e-10, max_steps=50, fixed_steps=0, krylov_rtol=1e-10,
           krylov_max_iter=1000, use_amg=True, cycles=1, max_coarse=64, deflate=False, linesearch=0, reorth=0):
    """Newton for GL(psi) = 0 with MINRES + R_k inner solves (Sec. 2, Sec. 4);
    with deflate, each step is solved on the complement of i psi; with
    linesearch > 0, backtracking on ||GL||_D (at most that many halvings of
    the step, a globalisation the paper does not use); reorth > 0: the
    solves store and reorthogonalise their Krylov basis."""
    psi = _c128(psi0).copy()
    ni = _NInfo()
    rc = lib().orc_newton(mesh._p, _ptr(psi), tol, max_steps, fixed_steps, krylov_rtol,
                          krylov_max_iter, int(use_amg), cycles, max_coarse, int(deflate), int(linesearch),
                          int(reorth), C.byref(ni))
    info = {"status": rc, "steps": ni.steps, "converged": bool(ni.converged),
            "res": list(ni.res[:ni.steps + 1]), "krylov_iters": list(ni.krylov_iters[:ni.steps]),
            "alpha": list(ni.alpha[:ni.steps])}
    return psi, info
