"""ctypes binding of libpmcorr.so (include/pmcorr.h).

Argument marshalling only: every step of the corrector path runs in the HIP
library.  PyTorch provides device memory (tensors) and the current HIP
stream.  Functions carry the C names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmcorr.so")

PM_OK, PM_MAXIT, PM_STAGNATED = 0, 1, 2
PM_PREC_JACOBI, PM_PREC_CHEBYSHEV = 0, 1
PM_INVALID_ARG, PM_BAD_MESH, PM_NOT_DELAUNAY, PM_SINGULAR = -1, -2, -3, -4
PM_NONFINITE, PM_BREAKDOWN, PM_HIP_ERROR = -5, -6, -7
PM_CP1X, PM_CP1Y, PM_CP2 = 0, 1, 2
PM_FP64, PM_MIXED = 0, 1


class pm_mesh_stats(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("n_nodes", C.c_int32), ("nnz", C.c_int32),
        ("n_interior_sides", C.c_int32), ("n_boundary_sides", C.c_int32),
        ("bandwidth", C.c_int32), ("n_components", C.c_int32), ("index_bits", C.c_int32),
        ("max_T", C.c_double), ("min_cot_sum", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pm_cell_params(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("eps", "logk", "chi", "g11", "g12", "g22")]


class pm_opts(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_it", C.c_int32), ("precision", C.c_int32),
        ("replace_every", C.c_int32), ("x0_is_zero", C.c_int32), ("block", C.c_int32),
        ("tile_rows", C.c_int32), ("stag_checks", C.c_int32), ("precond", C.c_int32),
        ("cheb_degree", C.c_int32), ("iter_shape", C.c_int32),
    ]


class pm_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res_true", C.c_double),
                ("bnorm", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)} ({status}): {msg}")
        self.status = status


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, D = C.c_void_p, C.c_int32, C.c_double
        sig = {
            "pm_opts_default": (None, [P]),
            "pm_status_string": (C.c_char_p, [C.c_int]),
            "pm_last_error": (C.c_int, [C.c_char_p, I32]),
            "pm_structure_host": (C.c_int, [I32, P, I32, P, P, P, P, P, I32, P, P]),
            "pm_mesh_create": (C.c_int, [I32, P, I32, P, P, C.POINTER(P)]),
            "pm_mesh_destroy": (None, [P]),
            "pm_mesh_get_stats": (C.c_int, [P, P]),
            "pm_mesh_export": (C.c_int, [P, P, P, P]),
            "pm_mesh_set_index_bits": (C.c_int, [P, I32]),
            "assemble_corrector": (C.c_int, [P, I32, P, D, D, P, P, P, P, P, P]),
            "pcg_solve": (C.c_int, [P, P, P, P, P, P, P]),
            "pm_batch_create": (C.c_int, [I32, P, C.POINTER(P)]),
            "pm_batch_destroy": (None, [P]),
            "pm_batch_offsets": (C.c_int, [P, P, P]),
            "pcg_solve_batched": (C.c_int, [P, P, P, P, P, P, P]),
            "pcg_adjoint": (C.c_int, [P, I32, P, D, D, P, P, P, P, P, P, P, P, P, P]),
            "pm_time_kernel": (C.c_int, [P, I32, I32, P, P, P]),
            "pm_last_launch": (C.c_int, [P, P, P, P]),
            "cp2_cross_rhs": (C.c_int, [P, P, D, D, P, P, P, P, P]),
            "pm_time_cross": (C.c_int, [P, P, D, D, P, P, P, P, I32, P, P, P]),
            "cp2_solve_two_step": (C.c_int, [P, P, P, D, D, P, P, P, P, P, P, P]),
            "cp1_solve_coupled": (C.c_int, [P, P, D, D, P, P, P, P, P, P, D, I32, P, P, P, P,
                                            P]),
            "cp1_solve_coupled_pcg": (C.c_int, [P, P, D, D, P, P, P, P, P, P, P, P, P]),
            "flux_average": (C.c_int, [P, P, P, P, P, P, P, P]),
            "rt0_update": (C.c_int, [P, P, D, D, P, P, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().pm_status_string(int(s)).decode()


def last_error() -> str:
    buf = C.create_string_buffer(512)
    lib().pm_last_error(buf, 512)
    return buf.value.decode()


def _check(status, allow_positive=True):
    if status < 0 or (status > 0 and not allow_positive):
        raise PMError(status, last_error())
    return status


def _ptr(a):
    """Address of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(stream=None):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def pm_structure_host(xy, tri, side_tag):
    """Host-only analysis: returns perm, row_ptr, col, T [n,3] and stats."""
    xy = _host(xy, np.float64)
    tri = _host(tri, np.int32)
    tag = _host(side_tag, np.int8)
    n = tri.shape[0]
    perm = np.empty(n, np.int32)
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(4 * n, np.int32)
    T = np.empty((n, 3), np.float64)
    st = pm_mesh_stats()
    _check(lib().pm_structure_host(xy.shape[0], _ptr(xy), n, _ptr(tri), _ptr(tag), _ptr(perm),
                                   _ptr(row_ptr), _ptr(col), 4 * n, _ptr(T), C.addressof(st)))
    return perm, row_ptr, col[: st.nnz].copy(), T, st.as_dict()


class Mesh:
    """Owns a pm_mesh handle (structure + device workspace)."""

    def __init__(self, xy, tri, side_tag):
        xy = _host(xy, np.float64)
        tri = _host(tri, np.int32)
        tag = _host(side_tag, np.int8)
        h = C.c_void_p()
        _check(lib().pm_mesh_create(xy.shape[0], _ptr(xy), tri.shape[0], _ptr(tri), _ptr(tag),
                                    C.byref(h)))
        self.handle = h
        st = pm_mesh_stats()
        _check(lib().pm_mesh_get_stats(h, C.addressof(st)))
        self.stats = st.as_dict()
        self.n = st.n_cells
        self.nnz = st.nnz

    def export(self):
        perm = np.empty(self.n, np.int32)
        row_ptr = np.empty(self.n + 1, np.int32)
        col = np.empty(self.nnz, np.int32)
        _check(lib().pm_mesh_export(self.handle, _ptr(perm), _ptr(row_ptr), _ptr(col)))
        return perm, row_ptr, col

    def set_index_bits(self, bits: int):
        """Width of the solver's column offsets (16 or 32)."""
        _check(lib().pm_mesh_set_index_bits(self.handle, int(bits)))
        st = pm_mesh_stats()
        _check(lib().pm_mesh_get_stats(self.handle, C.addressof(st)))
        self.stats = st.as_dict()

    def close(self):
        if self.handle:
            lib().pm_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pm_mesh_create(xy, tri, side_tag) -> Mesh:
    return Mesh(xy, tri, side_tag)


def _params(params):
    p = pm_cell_params()
    keep = []
    for k in ("eps", "logk", "chi", "g11", "g12", "g22"):
        t = params.get(k)
        if t is not None:
            keep.append(t)
        setattr(p, k, _ptr(t))
    return p, keep


def assemble_corrector(mesh: Mesh, kind: int, params: dict, nu: float, dt: float, g_dirichlet=None,
                       val32=False, dinv=False, b_lift=False, stream=None):
    """Returns a dict with val64 (and val32 / dinv / b_lift if requested) as device tensors."""
    import torch

    dev = params["eps"].device
    out = {"val64": torch.empty(mesh.nnz, dtype=torch.float64, device=dev)}
    if val32:
        out["val32"] = torch.empty(mesh.nnz, dtype=torch.float32, device=dev)
    if dinv:
        out["dinv"] = torch.empty(mesh.n, dtype=torch.float64, device=dev)
    if b_lift:
        out["b_lift"] = torch.empty(mesh.n, dtype=torch.float64, device=dev)
    p, _keep = _params(params)
    _check(lib().assemble_corrector(mesh.handle, kind, C.addressof(p), nu, dt, _ptr(g_dirichlet),
                                    _ptr(out["val64"]), _ptr(out.get("val32")), _ptr(out.get("dinv")),
                                    _ptr(out.get("b_lift")), _stream(stream)))
    return out


def make_opts(tol=1e-10, max_it=200000, precision=PM_FP64, replace_every=50, x0_is_zero=True,
              block=0, tile_rows=0, stag_checks=40, iter_shape=0, precond=0,
              cheb_degree=4) -> pm_opts:
    o = pm_opts()
    lib().pm_opts_default(C.addressof(o))
    o.tol, o.max_it, o.precision, o.replace_every = tol, max_it, precision, replace_every
    o.x0_is_zero, o.block, o.tile_rows = int(bool(x0_is_zero)), block, tile_rows
    o.stag_checks = stag_checks
    o.iter_shape = iter_shape
    o.precond, o.cheb_degree = precond, cheb_degree
    return o


def pcg_solve(mesh: Mesh, val64, b, x=None, stream=None, **opts):
    """Solve A x = b on the device; returns (x, info dict).  Positive statuses
    (iteration limit) are returned in info, negative ones raise."""
    import torch

    if x is None:
        x = torch.zeros_like(b)
        opts.setdefault("x0_is_zero", True)
    o = make_opts(**opts)
    info = pm_info()
    _check(lib().pcg_solve(mesh.handle, _ptr(val64), _ptr(b), _ptr(x), C.addressof(o),
                           C.addressof(info), _stream(stream)))
    return x, info.as_dict()


class Batch:
    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.handle for m in self.meshes])
        h = C.c_void_p()
        _check(lib().pm_batch_create(len(self.meshes), arr, C.byref(h)))
        self.handle = h
        k = len(self.meshes)
        self.val_off = np.empty(k + 1, np.int64)
        self.vec_off = np.empty(k + 1, np.int64)
        _check(lib().pm_batch_offsets(h, _ptr(self.val_off), _ptr(self.vec_off)))

    def close(self):
        if self.handle:
            lib().pm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pm_batch_create(meshes) -> Batch:
    return Batch(meshes)


def pcg_solve_batched(batch: Batch, val64, b, x=None, stream=None, **opts):
    import torch

    if x is None:
        x = torch.zeros_like(b)
        opts.setdefault("x0_is_zero", True)
    o = make_opts(**opts)
    infos = (pm_info * len(batch.meshes))()
    st = lib().pcg_solve_batched(batch.handle, _ptr(val64), _ptr(b), _ptr(x), C.addressof(o),
                                 C.addressof(infos), _stream(stream))
    if st in (PM_INVALID_ARG, PM_HIP_ERROR):
        raise PMError(st, last_error())
    # per-system outcomes (including errors of single systems) are in the infos
    return x, [i.as_dict() for i in infos]


def pcg_adjoint(mesh: Mesh, kind, params, nu, dt, val64, eta, grad_eta, g_dirichlet=None,
                stream=None, **opts):
    """Returns (lambda, grad_logk, grad_eps, info)."""
    import torch

    lam = torch.empty_like(eta)
    gs = torch.empty_like(eta)
    ge = torch.empty_like(eta)
    o = make_opts(**opts)
    info = pm_info()
    p, _keep = _params(params)
    _check(lib().pcg_adjoint(mesh.handle, kind, C.addressof(p), nu, dt, _ptr(g_dirichlet),
                             _ptr(val64), _ptr(eta), _ptr(grad_eta), _ptr(lam), _ptr(gs), _ptr(ge),
                             C.addressof(o), C.addressof(info), _stream(stream)))
    return lam, gs, ge, info.as_dict()


def cp2_cross_rhs(mesh: Mesh, params, nu, dt, eta_tilde, b_in, b_out=None, g_dirichlet=None,
                  stream=None):
    """b_out = b_in + the CP2 cross terms at eta_tilde (device tensors, cell
    order); b_out may be b_in.  Returns b_out."""
    import torch

    if b_out is None:
        b_out = torch.empty_like(b_in)
    p, _keep = _params(params)
    _check(lib().cp2_cross_rhs(mesh.handle, C.addressof(p), nu, dt, _ptr(g_dirichlet),
                               _ptr(eta_tilde), _ptr(b_in), _ptr(b_out), _stream(stream)))
    return b_out


def cp2_solve_two_step(mesh: Mesh, val64, params, nu, dt, b, g_dirichlet=None, stream=None,
                       **opts):
    """The two CP2 solves of one step (eta~, then eta with the cross terms of
    eta~ on the right-hand side).  Returns (eta, eta_tilde, [info1, info2]);
    negative statuses raise."""
    import torch

    eta_t = torch.empty_like(b)
    eta = torch.empty_like(b)
    o = make_opts(**opts)
    infos = (pm_info * 2)()
    p, _keep = _params(params)
    _check(lib().cp2_solve_two_step(mesh.handle, _ptr(val64), C.addressof(p), nu, dt,
                                    _ptr(g_dirichlet), _ptr(b), _ptr(eta_t), _ptr(eta),
                                    C.addressof(o), infos, _stream(stream)))
    return eta, eta_t, [i.as_dict() for i in infos]


def cp1_solve_coupled(mesh: Mesh, params, nu, dt, val_x, val_y, b_x, b_y, toll=1e-4,
                      max_outer=50, stream=None, **opts):
    """Coupled CP1 by the loop of the paper's App. B.  Returns (u, v, info)
    with info = {"status", "outer", "err", "x": info of the x solves,
    "y": ...}; negative statuses raise."""
    import torch

    u = torch.empty_like(b_x)
    v = torch.empty_like(b_y)
    o = make_opts(**opts)
    infos = (pm_info * 2)()
    nout = C.c_int32()
    err = C.c_double()
    p, _keep = _params(params)
    st = _check(lib().cp1_solve_coupled(mesh.handle, C.addressof(p), nu, dt, _ptr(val_x),
                                        _ptr(val_y), _ptr(b_x), _ptr(b_y), _ptr(u), _ptr(v),
                                        float(toll), int(max_outer), C.addressof(o), infos,
                                        C.byref(nout), C.byref(err), _stream(stream)))
    return u, v, {"status": st, "outer": nout.value, "err": err.value,
                  "x": infos[0].as_dict(), "y": infos[1].as_dict()}


def cp1_solve_coupled_pcg(mesh: Mesh, params, nu, dt, val_x, val_y, b_x, b_y, stream=None,
                          **opts):
    """Coupled CP1 by block-Jacobi CG on both components.  Returns (u, v,
    info); negative statuses raise."""
    import torch

    u = torch.empty_like(b_x)
    v = torch.empty_like(b_y)
    o = make_opts(**opts)
    info = pm_info()
    p, _keep = _params(params)
    _check(lib().cp1_solve_coupled_pcg(mesh.handle, C.addressof(p), nu, dt, _ptr(val_x),
                                       _ptr(val_y), _ptr(b_x), _ptr(b_y), _ptr(u), _ptr(v),
                                       C.addressof(o), C.addressof(info), _stream(stream)))
    return u, v, info.as_dict()


def flux_average(mesh: Mesh, u, v, g_u=None, g_v=None, stream=None):
    """Returns (fbar [n, 3], b1 [n]) as device tensors, cell order."""
    import torch

    fbar = torch.empty((mesh.n, 3), dtype=torch.float64, device=u.device)
    b1 = torch.empty_like(u)
    _check(lib().flux_average(mesh.handle, _ptr(u), _ptr(v), _ptr(g_u), _ptr(g_v), _ptr(fbar),
                              _ptr(b1), _stream(stream)))
    return fbar, b1


def rt0_update(mesh: Mesh, params, nu, dt, eta_tilde, eta, fbar, g_dirichlet=None, stream=None):
    """Returns (u, v, Q [n, 3]) as device tensors, cell order."""
    import torch

    u = torch.empty_like(eta)
    v = torch.empty_like(eta)
    q = torch.empty((mesh.n, 3), dtype=torch.float64, device=eta.device)
    p, _keep = _params(params)
    _check(lib().rt0_update(mesh.handle, C.addressof(p), nu, dt, _ptr(g_dirichlet),
                            _ptr(eta_tilde), _ptr(eta), _ptr(fbar), _ptr(u), _ptr(v), _ptr(q),
                            _stream(stream)))
    return u, v, q


def pm_time_cross(mesh: Mesh, params, nu, dt, eta_tilde, b_in, n_launch: int, g_dirichlet=None,
                  stream=None):
    """Mean ms and bytes per launch of the three cross-term kernels."""
    import torch

    b_out = torch.empty_like(b_in)
    ms = (C.c_double * 3)()
    by = (C.c_double * 3)()
    p, _keep = _params(params)
    _check(lib().pm_time_cross(mesh.handle, C.addressof(p), nu, dt, _ptr(g_dirichlet),
                               _ptr(eta_tilde), _ptr(b_in), _ptr(b_out), n_launch, _stream(stream),
                               ms, by))
    return list(ms), list(by)


def pm_time_kernel(mesh: Mesh, which: int, n_launch: int, stream=None):
    """(ms per launch, bytes per launch) of an iteration kernel of the last solve."""
    ms = C.c_double()
    by = C.c_double()
    _check(lib().pm_time_kernel(mesh.handle, which, n_launch, _stream(stream), C.byref(ms),
                                C.byref(by)))
    return ms.value, by.value


def pm_last_launch(mesh: Mesh) -> dict:
    """Launch shape (tile rows, block, iteration schedule) of the last solve on `mesh`."""
    v = [C.c_int32() for _ in range(3)]
    _check(lib().pm_last_launch(mesh.handle, *[C.byref(x) for x in v]))
    return {"tile_rows": v[0].value, "block": v[1].value, "iter_shape": v[2].value}


EXPORTED = [
    "pm_opts_default", "pm_status_string", "pm_last_error", "pm_structure_host", "pm_mesh_create",
    "pm_mesh_destroy", "pm_mesh_get_stats", "pm_mesh_export", "pm_mesh_set_index_bits", "assemble_corrector", "pcg_solve",
    "pm_batch_create", "pm_batch_destroy", "pm_batch_offsets", "pcg_solve_batched", "pcg_adjoint",
    "pm_time_kernel", "pm_last_launch", "cp2_cross_rhs", "pm_time_cross",
    "cp2_solve_two_step", "cp1_solve_coupled", "cp1_solve_coupled_pcg", "flux_average",
    "rt0_update",
]
