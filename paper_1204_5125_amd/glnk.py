"""ctypes binding of libglnk.so (include/glnk.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Vectors are torch.complex128 tensors on the GPU (contiguous); the
current torch stream is passed to the library unless a stream is given.
The binding raises if the shared library has not been built.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglnk.so")

GL_OK = 0
STATUS = {0: "GL_OK", 1: "GL_ERR_INVALID_ARGUMENT", 2: "GL_ERR_HIP", 3: "GL_ERR_OUT_OF_MEMORY",
          4: "GL_ERR_NOT_CONVERGED", 5: "GL_ERR_BREAKDOWN", 6: "GL_ERR_NONFINITE",
          7: "GL_ERR_SINGULAR", 8: "GL_ERR_UNSUPPORTED"}
GL_FP64, GL_FP32, GL_MIXED = 0, 1, 2

# gl_precond_export array identifiers
EXPORT = {"agg": 0, "root": 1, "color": 2, "A_rp": 3, "A_ci": 4, "A_v": 5, "P_rp": 6, "P_ci": 7,
          "P_v": 8, "R_rp": 9, "R_ci": 10, "R_v": 11}

EXPORTED_SYMBOLS = [
    "gl_mesh_create_grid", "gl_mesh_create_simplicial", "gl_mesh_set_field", "gl_mesh_num_nodes", "gl_mesh_export_links",
    "gl_mesh_destroy", "gl_residual", "gl_residual_noalloc", "gl_residual_dmu", "gl_inner", "gl_axpby",
    "gl_jacobian_apply", "gl_secant_predict", "gl_precond_setup",
    "gl_precond_apply", "gl_precond_inner_steps",
    "gl_precond_info", "gl_precond_export", "gl_precond_destroy", "gl_jacobian_solve",
    "gl_newton_solve", "gl_precond_set_tiles", "gl_precond_get_tiles", "gl_batch_create",
    "gl_batch_newton_solve", "gl_batch_set_tiles", "gl_batch_stats", "gl_batch_destroy",
    "gl_unet_create", "gl_unet_num_params", "gl_unet_set_params", "gl_unet_get_params", "gl_unet_predict",
    "gl_unet_loss_grad", "gl_unet_train_step", "gl_unet_destroy",
    "gl_profile_start", "gl_profile_stop", "gl_set_allocator", "gl_status_string", "gl_last_error",
]
_VOID = ("gl_mesh_destroy", "gl_precond_destroy", "gl_batch_destroy", "gl_unet_destroy", "gl_status_string",
         "gl_last_error")


class GlnkError(RuntimeError):
    def __init__(self, code, what, detail=""):
        super().__init__(f"{what}: {STATUS.get(code, code)} {detail}".strip())
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_axis", C.c_int64 * 3), ("side", C.c_double * 3),
                ("potential", C.c_int), ("mu", C.c_double), ("b_dir", C.c_double * 3),
                ("a_matrix", C.c_double * 9), ("dipole_m", C.c_double * 3), ("dipole_x0", C.c_double * 3)]


class SimplicialDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_nodes", C.c_int64), ("x", C.c_void_p), ("n_cells", C.c_int64),
                ("cells", C.c_void_p), ("potential", C.c_int), ("mu", C.c_double),
                ("b_dir", C.c_double * 3), ("a_matrix", C.c_double * 9), ("dipole_m", C.c_double * 3),
                ("dipole_x0", C.c_double * 3)]


class AmgOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("cycles", C.c_int), ("max_coarse", C.c_int),
                ("max_levels", C.c_int)]


class KrylovOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("poll_every", C.c_int),
                ("inner_rtol", C.c_double), ("relax_rtol", C.c_double), ("deflate", C.c_int),
                ("reorth", C.c_int)]


class KrylovInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("eta0", C.c_double),
                ("res_est", C.c_double), ("res_true", C.c_double)]


class NewtonOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_steps", C.c_int), ("fixed_steps", C.c_int),
                ("use_precond", C.c_int), ("krylov", KrylovOpts), ("amg", AmgOpts), ("linesearch", C.c_int)]


class Tiles(C.Structure):
    _fields_ = [("lane_shift", C.c_int), ("bottom_rows", C.c_int), ("dense_rows", C.c_int),
                ("l0_tiled", C.c_int)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("steps", C.c_int), ("converged", C.c_int), ("res", C.c_double * 64),
                ("krylov_iters", C.c_int * 64), ("alpha", C.c_double * 64)]


_lib = None
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_allocator_refs = []   # callbacks handed to the library stay alive for its lifetime


def lib():
    """Load libglnk.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libglnk.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    P = C.POINTER
    L.gl_mesh_create_grid.argtypes = [P(GridDesc), vp, P(vp)]
    L.gl_mesh_create_simplicial.argtypes = [P(SimplicialDesc), vp, P(vp)]
    L.gl_mesh_set_field.argtypes = [vp, C.c_double, vp]
    L.gl_mesh_num_nodes.argtypes = [vp, P(C.c_int64)]
    L.gl_mesh_export_links.argtypes = [vp, C.c_int, vp]
    L.gl_mesh_destroy.argtypes = [vp]
    L.gl_mesh_destroy.restype = None
    L.gl_residual.argtypes = [vp, vp, vp, P(C.c_double), vp]
    L.gl_residual_noalloc.argtypes = [vp, vp, vp, P(C.c_double), vp]
    L.gl_residual_dmu.argtypes = [vp, vp, vp, vp]
    L.gl_inner.argtypes = [vp, vp, vp, P(C.c_double), vp]
    L.gl_axpby.argtypes = [vp, C.c_double, vp, C.c_double, vp, vp, vp]
    L.gl_jacobian_apply.argtypes = [vp, vp, vp, vp, vp]
    L.gl_secant_predict.argtypes = [vp, vp, vp, C.c_double, vp, vp]
    L.gl_precond_setup.argtypes = [vp, vp, P(AmgOpts), P(vp), vp]
    L.gl_precond_apply.argtypes = [vp, vp, vp, vp]
    L.gl_precond_inner_steps.argtypes = [vp, P(C.c_int)]
    L.gl_precond_info.argtypes = [vp, P(C.c_int), P(C.c_int64), P(C.c_int64), P(C.c_int)]
    L.gl_precond_export.argtypes = [vp, C.c_int, C.c_int, vp, P(C.c_size_t)]
    L.gl_precond_destroy.argtypes = [vp]
    L.gl_precond_destroy.restype = None
    L.gl_jacobian_solve.argtypes = [vp, vp, vp, vp, vp, P(KrylovOpts), P(KrylovInfo), vp]
    L.gl_newton_solve.argtypes = [vp, vp, P(NewtonOpts), P(vp), P(NewtonInfo), vp]
    L.gl_precond_set_tiles.argtypes = [vp, P(Tiles)]
    L.gl_precond_get_tiles.argtypes = [vp, P(Tiles)]
    L.gl_batch_create.argtypes = [C.c_int, P(vp), P(vp)]
    L.gl_batch_newton_solve.argtypes = [vp, P(vp), P(NewtonOpts), P(NewtonInfo), vp]
    L.gl_batch_set_tiles.argtypes = [vp, C.c_int, P(Tiles)]
    L.gl_batch_stats.argtypes = [vp, P(C.c_int64), P(C.c_int64), P(C.c_int), P(C.c_double)]
    L.gl_batch_destroy.argtypes = [vp]
    L.gl_batch_destroy.restype = None
    L.gl_unet_create.argtypes = [C.c_int, C.c_int, P(vp)]
    L.gl_unet_num_params.argtypes = [vp, P(C.c_int64)]
    L.gl_unet_set_params.argtypes = [vp, vp]
    L.gl_unet_get_params.argtypes = [vp, vp]
    L.gl_unet_predict.argtypes = [vp, vp, vp, vp, C.c_double, C.c_double, vp, vp]
    L.gl_unet_loss_grad.argtypes = [vp, vp, vp, vp, C.c_double, C.c_double, vp, P(C.c_double), vp, vp]
    L.gl_unet_train_step.argtypes = [vp, vp, C.c_int, P(vp), P(vp), P(C.c_double), P(C.c_double), P(vp),
                                     P(AdamOpts), P(C.c_double), vp]
    L.gl_unet_destroy.argtypes = [vp]
    L.gl_unet_destroy.restype = None
    L.gl_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    L.gl_profile_start.argtypes = [C.c_int]
    L.gl_profile_stop.argtypes = [P(C.c_double), P(C.c_double), P(C.c_int64)]
    L.gl_status_string.argtypes = [st]
    L.gl_status_string.restype = C.c_char_p
    L.gl_last_error.argtypes = []
    L.gl_last_error.restype = C.c_char_p
    for name in EXPORTED_SYMBOLS:
        if name not in _VOID:
            getattr(L, name).restype = st
    _lib = L
    return L


def _check(rc, what, allow=()):
    if rc != GL_OK and rc not in allow:
        raise GlnkError(rc, what, lib().gl_last_error().decode())
    return rc


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vec(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name}: expected a complex128 CUDA tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected a contiguous tensor of {n} elements")
    return C.c_void_p(t.data_ptr())


class Mesh:
    """gl_mesh handle: a tensor grid with its link variables on the GPU."""

    def __init__(self, dim, n_axis, side, mu=0.0, b_dir=(0.0, 0.0, 1.0), a_matrix=None, dipole=None,
                 stream=None):
        """dipole = (m, x0): the potential mu A_d(r) = mu m x (r - x0) / |r - x0|^3."""
        d = GridDesc()
        d.dim = dim
        for a in range(3):
            d.n_axis[a] = int(n_axis[a]) if a < len(n_axis) else 1
            d.side[a] = float(side[a]) if a < len(side) else 1.0
        d.mu = mu
        for a in range(3):
            d.b_dir[a] = b_dir[a]
        if a_matrix is not None:
            d.potential = 1
            for k, v in enumerate(np.asarray(a_matrix, dtype=np.float64).ravel()):
                d.a_matrix[k] = v
        if dipole is not None:
            d.potential = 2
            for a in range(3):
                d.dipole_m[a] = float(dipole[0][a])
                d.dipole_x0[a] = float(dipole[1][a])
        h = C.c_void_p()
        _check(lib().gl_mesh_create_grid(C.byref(d), _stream(stream), C.byref(h)), "gl_mesh_create_grid")
        self._h = h
        self.dim = dim
        self.shape = tuple(int(v) for v in n_axis[:dim])
        self.side = tuple(float(v) for v in side[:dim])
        nn = C.c_int64()
        _check(lib().gl_mesh_num_nodes(h, C.byref(nn)), "gl_mesh_num_nodes")
        self.n = nn.value

    @classmethod
    def simplicial(cls, x, cells, mu=0.0, b_dir=(0.0, 0.0, 1.0), a_matrix=None, dipole=None, stream=None):
        """gl_mesh_create_simplicial: nodes x (n x 2 or n x 3) and cells
        (m x 3 triangles or m x 4 tetrahedra, node indices); the potential as
        for the grid."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        if x.ndim != 2 or x.shape[1] not in (2, 3) or cells.ndim != 2 or cells.shape[1] != x.shape[1] + 1:
            raise ValueError("x must be n x 2 with triangles m x 3, or n x 3 with tetrahedra m x 4")
        d = SimplicialDesc()
        d.dim = x.shape[1]
        d.n_nodes, d.n_cells = len(x), len(cells)
        d.x, d.cells = x.ctypes.data, cells.ctypes.data
        d.mu = mu
        for a in range(3):
            d.b_dir[a] = b_dir[a]
        if a_matrix is not None:
            d.potential = 1
            for k, v in enumerate(np.asarray(a_matrix, dtype=np.float64).ravel()):
                d.a_matrix[k] = v
        if dipole is not None:
            d.potential = 2
            for a in range(3):
                d.dipole_m[a] = float(dipole[0][a])
                d.dipole_x0[a] = float(dipole[1][a])
        h = C.c_void_p()
        _check(lib().gl_mesh_create_simplicial(C.byref(d), _stream(stream), C.byref(h)),
               "gl_mesh_create_simplicial")
        self = cls.__new__(cls)
        self._h = h
        self.dim = x.shape[1]
        self.shape = None
        self.side = None
        self.n = len(x)
        return self

    @property
    def handle(self):
        return self._h

    def set_field(self, mu, stream=None):
        _check(lib().gl_mesh_set_field(self._h, mu, _stream(stream)), "gl_mesh_set_field")

    def export_links(self, axis):
        out = np.empty(self.n, dtype=np.complex128)
        _check(lib().gl_mesh_export_links(self._h, axis, out.ctypes.data_as(C.c_void_p)),
               "gl_mesh_export_links")
        return out

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gl_mesh_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def gl_mesh_create_grid(dim, n_axis, side, **kw):
    return Mesh(dim, n_axis, side, **kw)


def gl_mesh_create_simplicial(xy, triangles, **kw):
    return Mesh.simplicial(xy, triangles, **kw)


def gl_residual(mesh, psi, out=None, norm=True, stream=None):
    """out = GL(psi); returns ||GL(psi)||_D when norm is True."""
    nd = C.c_double()
    _check(lib().gl_residual(mesh.handle, _vec(psi, mesh.n, "psi"),
                             _vec(out, mesh.n, "out") if out is not None else None,
                             C.byref(nd) if norm else None, _stream(stream)), "gl_residual")
    return nd.value if norm else None


def gl_residual_noalloc(mesh, psi, out=None, norm=True, stream=None):
    """gl_residual with its reduction scratch in the library's static device
    array (no allocation); returns ||GL(psi)||_D when norm is True."""
    nd = C.c_double()
    _check(lib().gl_residual_noalloc(mesh.handle, _vec(psi, mesh.n, "psi"),
                                     _vec(out, mesh.n, "out") if out is not None else None,
                                     C.byref(nd) if norm else None, _stream(stream)), "gl_residual_noalloc")
    return nd.value if norm else None


def gl_residual_dmu(mesh, psi, out, stream=None):
    """out = d GL(psi; mu) / d mu at the mesh's current mu."""
    _check(lib().gl_residual_dmu(mesh.handle, _vec(psi, mesh.n, "psi"), _vec(out, mesh.n, "out"),
                                 _stream(stream)), "gl_residual_dmu")


def gl_inner(mesh, u, v, stream=None):
    """<u, v>_R = Re sum |V_i| conj(u_i) v_i."""
    r = C.c_double()
    _check(lib().gl_inner(mesh.handle, _vec(u, mesh.n, "u"), _vec(v, mesh.n, "v"), C.byref(r), _stream(stream)),
           "gl_inner")
    return r.value


def gl_axpby(mesh, a, x, b, y, out, stream=None):
    """out = a x + b y (real a, b; out may alias x or y)."""
    _check(lib().gl_axpby(mesh.handle, float(a), _vec(x, mesh.n, "x"), float(b), _vec(y, mesh.n, "y"),
                          _vec(out, mesh.n, "out"), _stream(stream)), "gl_axpby")


def gl_jacobian_apply(mesh, psi, phi, out, stream=None):
    """out = J(psi) phi."""
    _check(lib().gl_jacobian_apply(mesh.handle, _vec(psi, mesh.n, "psi"), _vec(phi, mesh.n, "phi"),
                                   _vec(out, mesh.n, "out"), _stream(stream)), "gl_jacobian_apply")


def gl_secant_predict(mesh, psi_m, psi_prev, ratio, out, stream=None):
    """out = psi_m + ratio (psi_m - e^{i chi} psi_prev), chi = arg <psi_prev, psi_m>."""
    _check(lib().gl_secant_predict(mesh.handle, _vec(psi_m, mesh.n, "psi_m"), _vec(psi_prev, mesh.n, "psi_prev"),
                                   float(ratio), _vec(out, mesh.n, "out"), _stream(stream)), "gl_secant_predict")


class Precond:
    """gl_precond handle: R_k(psi) = AMG_k(K-hat + 2 D |psi|^2, D .)."""

    def __init__(self, mesh, psi, precision=GL_FP64, cycles=1, max_coarse=64, max_levels=16,
                 stream=None):
        self.mesh = mesh
        o = AmgOpts(precision, cycles, max_coarse, max_levels)
        h = C.c_void_p()
        _check(lib().gl_precond_setup(mesh.handle, _vec(psi, mesh.n, "psi"), C.byref(o), C.byref(h),
                                      _stream(stream)), "gl_precond_setup")
        self._h = h
        self.opts = o

    @property
    def handle(self):
        return self._h

    def update(self, psi, precision=None, cycles=None, stream=None):
        """Recompute the values for a new psi (the hierarchy is kept)."""
        o = AmgOpts(self.opts.precision if precision is None else precision,
                    self.opts.cycles if cycles is None else cycles, self.opts.max_coarse,
                    self.opts.max_levels)
        h = self._h
        _check(lib().gl_precond_setup(self.mesh.handle, _vec(psi, self.mesh.n, "psi"), C.byref(o),
                                      C.byref(h), _stream(stream)), "gl_precond_setup")
        self.opts = o

    def apply(self, r, z, stream=None):
        _check(lib().gl_precond_apply(self._h, _vec(r, self.mesh.n, "r"), _vec(z, self.mesh.n, "z"),
                                      _stream(stream)), "gl_precond_apply")

    def inner_steps(self):
        """V-cycles per application: k for R_k, the CG steps m for R_inf (cycles 0)."""
        k = C.c_int()
        _check(lib().gl_precond_inner_steps(self._h, C.byref(k)), "gl_precond_inner_steps")
        return k.value

    def info(self):
        nlev = C.c_int()
        sizes = (C.c_int64 * 16)()
        nnz = (C.c_int64 * 16)()
        nc = (C.c_int * 16)()
        _check(lib().gl_precond_info(self._h, C.byref(nlev), sizes, nnz, nc), "gl_precond_info")
        k = nlev.value
        return {"nlev": k, "sizes": list(sizes[:k]), "nnz": list(nnz[:k]), "ncolors": list(nc[:k])}

    def export(self, level, what):
        code = EXPORT[what] if isinstance(what, str) else int(what)
        nbytes = C.c_size_t(0)
        _check(lib().gl_precond_export(self._h, level, code, None, C.byref(nbytes)), "gl_precond_export")
        dtype = np.complex128 if code in (5, 8, 11) else np.int32
        out = np.empty(nbytes.value // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib().gl_precond_export(self._h, level, code, out.ctypes.data_as(C.c_void_p),
                                       C.byref(nbytes)), "gl_precond_export")
        return out

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gl_precond_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def gl_set_allocator(alloc=None, release=None):
    """Device workspaces of handles created from now on come from
    alloc(nbytes) -> int pointer and go back through release(ptr); None for
    both restores hipMalloc / hipFree."""
    if alloc is None and release is None:
        _check(lib().gl_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "gl_set_allocator")
        return
    fa = _ALLOC_FN(lambda nbytes, stream, ctx: alloc(nbytes) or None)
    fr = _FREE_FN(lambda ptr, stream, ctx: release(ptr))
    _allocator_refs.append((fa, fr))
    _check(lib().gl_set_allocator(fa, fr, None), "gl_set_allocator")


def use_torch_allocator():
    """Route the handles' device workspaces through PyTorch's caching allocator."""
    import torch
    gl_set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                     lambda p: torch.cuda.caching_allocator_delete(p))


def gl_profile_start(kernel_id):
    _check(lib().gl_profile_start(kernel_id), "gl_profile_start")


def gl_profile_stop():
    """Returns (kernel ms summed, algorithmic bytes summed, launches)."""
    ms, by, nl = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().gl_profile_stop(C.byref(ms), C.byref(by), C.byref(nl)), "gl_profile_stop")
    return ms.value, by.value, nl.value


def gl_precond_setup(mesh, psi, **kw):
    return Precond(mesh, psi, **kw)


def gl_precond_apply(pre, r, z, stream=None):
    pre.apply(r, z, stream)


def gl_jacobian_solve(mesh, psi, pre, b, x, rtol=1e-10, max_iter=1000, poll_every=8, inner_rtol=0.0,
                      relax_rtol=0.0, deflate=False, reorth=0, stream=None, raise_on_fail=True):
    """Solve J(psi) x = b by preconditioned MINRES (with deflate: on the
    complement of the gauge mode i psi; with reorth > 0: the Krylov basis of
    at most reorth vectors stored and reorthogonalised); returns (status,
    info dict)."""
    o = KrylovOpts(rtol, max_iter, poll_every, inner_rtol, relax_rtol, int(deflate), int(reorth))
    ki = KrylovInfo()
    rc = lib().gl_jacobian_solve(mesh.handle, _vec(psi, mesh.n, "psi"),
                                 pre.handle if pre is not None else None, _vec(b, mesh.n, "b"),
                                 _vec(x, mesh.n, "x"), C.byref(o), C.byref(ki), _stream(stream))
    if raise_on_fail:
        _check(rc, "gl_jacobian_solve", allow=(4,))
    return rc, {"iterations": ki.iterations, "converged": bool(ki.converged), "eta0": ki.eta0,
                "res_est": ki.res_est, "res_true": ki.res_true}


class PrecondHandle:
    """Owner of a gl_precond built inside gl_newton_solve (reused across calls)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self._h = C.c_void_p()

    @property
    def handle(self):
        if self._h is None:
            self._h = C.c_void_p()
        return self._h

    # the handle's hierarchy (once a Newton solve has built it)
    info = Precond.info
    export = Precond.export
    inner_steps = Precond.inner_steps

    def close(self):
        if self._h and _lib is not None:
            _lib.gl_precond_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: ctypes may be gone
            pass


def gl_newton_solve(mesh, psi, tol=1e-10, max_steps=50, fixed_steps=0, use_precond=True,
                    krylov_rtol=1e-10, krylov_max_iter=1000, poll_every=8, inner_rtol=0.0,
                    relax_rtol=0.0, precision=GL_FP64, cycles=1, max_coarse=64, max_levels=16, precond=None,
                    deflate=False, linesearch=0, reorth=0, stream=None, raise_on_fail=True):
    """Newton for GL(psi) = 0 in place; returns (status, info dict).  precond:
    an optional PrecondHandle whose hierarchy is reused (and filled on first use);
    deflate: each step under the phase condition <i psi, dpsi>_R = 0;
    linesearch: at most this many halvings of a step that does not reduce
    ||GL||_D enough (0: full steps); reorth: the solves' Krylov basis size
    (0: plain MINRES)."""
    o = NewtonOpts(tol, max_steps, fixed_steps, int(use_precond),
                   KrylovOpts(krylov_rtol, krylov_max_iter, poll_every, inner_rtol, relax_rtol, int(deflate),
                              int(reorth)),
                   AmgOpts(precision, cycles, max_coarse, max_levels), int(linesearch))
    ni = NewtonInfo()
    rc = lib().gl_newton_solve(mesh.handle, _vec(psi, mesh.n, "psi"), C.byref(o),
                               C.byref(precond.handle) if precond is not None else None, C.byref(ni),
                               _stream(stream))
    if raise_on_fail:
        _check(rc, "gl_newton_solve", allow=(4,))
    return rc, _newton_info(ni)


def _newton_info(ni):
    return {"steps": ni.steps, "converged": bool(ni.converged), "res": list(ni.res[:ni.steps + 1]),
            "krylov_iters": list(ni.krylov_iters[:ni.steps]), "alpha": list(ni.alpha[:ni.steps])}


def gl_precond_set_tiles(pre, lane_shift=0, bottom_rows=0, dense_rows=0, l0_tiled=0):
    _check(lib().gl_precond_set_tiles(pre.handle, C.byref(Tiles(lane_shift, bottom_rows, dense_rows, l0_tiled))),
           "gl_precond_set_tiles")


def gl_precond_get_tiles(pre):
    t = Tiles()
    _check(lib().gl_precond_get_tiles(pre.handle, C.byref(t)), "gl_precond_get_tiles")
    return {"lane_shift": t.lane_shift, "bottom_rows": t.bottom_rows, "dense_rows": t.dense_rows,
            "l0_tiled": t.l0_tiled}


class Batch:
    """gl_batch: Newton on many meshes at once (one preconditioner each)."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = C.c_void_p()
        _check(lib().gl_batch_create(len(self.meshes), arr, C.byref(h)), "gl_batch_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_tiles(self, lane_shift=0, bottom_rows=0, dense_rows=0, l0_tiled=0, index=-1):
        _check(lib().gl_batch_set_tiles(self._h, index,
                                        C.byref(Tiles(lane_shift, bottom_rows, dense_rows, l0_tiled))),
               "gl_batch_set_tiles")

    def newton_solve(self, psis, tol=1e-10, max_steps=50, fixed_steps=0, use_precond=True,
                     krylov_rtol=1e-10, krylov_max_iter=1000, poll_every=8, inner_rtol=0.0,
                     precision=GL_FP64, cycles=1, max_coarse=64, max_levels=16, deflate=False, linesearch=0,
                     reorth=0, stream=None, raise_on_fail=True):
        """Newton on every instance in place (psis[i] on meshes[i]); returns
        (status, [info dict per instance]).  reorth: the solves' Krylov basis
        size (0: plain MINRES)."""
        if len(psis) != len(self.meshes):
            raise ValueError("one psi per mesh")
        ptrs = (C.c_void_p * len(psis))(*[_vec(p, m.n, "psi") for p, m in zip(psis, self.meshes)])
        o = NewtonOpts(tol, max_steps, fixed_steps, int(use_precond),
                       KrylovOpts(krylov_rtol, krylov_max_iter, poll_every, inner_rtol, 0.0, int(deflate),
                                  int(reorth)),
                       AmgOpts(precision, cycles, max_coarse, max_levels), int(linesearch))
        infos = (NewtonInfo * len(psis))()
        rc = lib().gl_batch_newton_solve(self._h, ptrs, C.byref(o), infos, _stream(stream))
        if raise_on_fail:
            _check(rc, "gl_batch_newton_solve", allow=(4,))
        return rc, [_newton_info(ni) for ni in infos]

    def stats(self):
        a, b, g = C.c_int64(), C.c_int64(), C.c_int()
        sec = (C.c_double * 3)()
        _check(lib().gl_batch_stats(self._h, C.byref(a), C.byref(b), C.byref(g), sec), "gl_batch_stats")
        return {"graph_launches": a.value, "dispatches_per_graph": b.value, "groups": g.value,
                "seconds": {"residual": sec[0], "setup": sec[1], "solve": sec[2]}}

    def close(self):
        if self._h and _lib is not None:
            _lib.gl_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: ctypes may be gone
            pass


def unet_layer_shapes(levels, base, in_ch=6, out_ch=2):
    """(c_in, c_out, k) of the library's U-Net layers, in parameter order."""
    shapes, c = [], in_ch
    for l in range(levels):
        shapes += [(c, base << l, 3), (base << l, base << l, 3)]
        c = base << l
    for l in range(levels - 2, -1, -1):
        shapes += [(c + (base << l), base << l, 3), (base << l, base << l, 3)]
        c = base << l
    shapes.append((c, out_ch, 1))
    return shapes


class UNet:
    """gl_unet: the learned continuation predictor."""

    def __init__(self, levels=4, base=32):
        h = C.c_void_p()
        _check(lib().gl_unet_create(levels, base, C.byref(h)), "gl_unet_create")
        self._h = h
        self.levels, self.base = levels, base
        n = C.c_int64()
        _check(lib().gl_unet_num_params(h, C.byref(n)), "gl_unet_num_params")
        self.n_params = n.value

    @property
    def handle(self):
        return self._h

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().gl_unet_set_params(self._h, theta.ctypes.data_as(C.c_void_p)), "gl_unet_set_params")

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().gl_unet_get_params(self._h, out.ctypes.data_as(C.c_void_p)), "gl_unet_get_params")
        return out

    def predict(self, mesh, psi, psi_base, mu, dmu, out, stream=None):
        _check(lib().gl_unet_predict(self._h, mesh.handle, _vec(psi, mesh.n, "psi"),
                                     _vec(psi_base, mesh.n, "psi_base"), mu, dmu, _vec(out, mesh.n, "out"),
                                     _stream(stream)), "gl_unet_predict")

    def loss_grad(self, mesh, psi, psi_base, mu, dmu, target, want_grad=True, stream=None):
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _check(lib().gl_unet_loss_grad(self._h, mesh.handle, _vec(psi, mesh.n, "psi"),
                                       _vec(psi_base, mesh.n, "psi_base"), mu, dmu,
                                       _vec(target, mesh.n, "target"), C.byref(loss),
                                       g.ctypes.data_as(C.c_void_p) if g is not None else None,
                                       _stream(stream)), "gl_unet_loss_grad")
        return loss.value, g

    def train_step(self, mesh, psis, bases, mus, dmus, targets, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   stream=None):
        k = len(psis)
        pp = (C.c_void_p * k)(*[_vec(p, mesh.n, "psi") for p in psis])
        bb = (C.c_void_p * k)(*[_vec(p, mesh.n, "psi_base") for p in bases])
        tt = (C.c_void_p * k)(*[_vec(t, mesh.n, "target") for t in targets])
        mm = (C.c_double * k)(*mus)
        dd = (C.c_double * k)(*dmus)
        loss = C.c_double()
        _check(lib().gl_unet_train_step(self._h, mesh.handle, k, pp, bb, mm, dd, tt,
                                        C.byref(AdamOpts(lr, beta1, beta2, eps)), C.byref(loss),
                                        _stream(stream)), "gl_unet_train_step")
        return loss.value

    def close(self):
        if self._h and _lib is not None:
            _lib.gl_unet_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: ctypes may be gone
            pass
