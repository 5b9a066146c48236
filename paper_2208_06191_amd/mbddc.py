"""Thin ctypes binding of the C ABI declared in ``include/mbddc.h``.

Argument marshalling only: every step of the solver runs in the HIP library
``libmbddc.so`` built next to this file. If the library is missing the import
of any entry point raises; there is no fallback path.

Arrays may be numpy arrays (host) or torch CUDA/HIP tensors (device); device
tensors are passed as raw pointers with ``on_device=1`` and must be contiguous
float64 tensors on the handle's device.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbddc.so")

MBDDC_OK, MBDDC_ERR_ARG, MBDDC_ERR_OOM, MBDDC_ERR_SINGULAR = 0, -1, -2, -3
MBDDC_ERR_NOCONV, MBDDC_ERR_DEVICE, MBDDC_ERR_STATE, MBDDC_ERR_UNSUPPORTED = -4, -5, -6, -7
MBDDC_HEX8, MBDDC_HEX27 = 1, 2
MBDDC_PRIMAL_V, MBDDC_PRIMAL_E, MBDDC_PRIMAL_F = 1, 2, 4
MBDDC_FP64, MBDDC_MIXED, MBDDC_MIXED_F32FACT = 0, 1, 2
MBDDC_SCALING_COUNTING, MBDDC_SCALING_DELUXE = 0, 1
MBDDC_MAT_SVK, MBDDC_MAT_NEO_HOOKEAN, MBDDC_MAT_GUCCIONE = 1, 2, 3
MBDDC_BC_ROBIN, MBDDC_BC_PRESSURE = 1, 2

_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


class mbddc_mesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("coords", _f64p), ("n_elems", ctypes.c_int32),
                ("elem_type", ctypes.c_int32), ("elem_nodes", _i32p), ("n_sub", ctypes.c_int32),
                ("elem_part", _i32p), ("node_tags", _u32p), ("n_dirichlet", ctypes.c_int32),
                ("dirichlet_dofs", _i32p)]


class mbddc_options(ctypes.Structure):
    _fields_ = [("primal", ctypes.c_uint32), ("levels", ctypes.c_int32), ("coarse_group", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("max_it", ctypes.c_int32), ("symmetric_hint", ctypes.c_int32), ("tune_table", ctypes.c_char_p),
                ("keep_coarse_matrix", ctypes.c_int32), ("coarse_primal", ctypes.c_uint32),
                ("graph_apply", ctypes.c_int32), ("packed_sym", ctypes.c_int32),
                ("nonsym_coarse", ctypes.c_int32), ("nnsp", ctypes.c_int32), ("scaling", ctypes.c_int32)]


class mbddc_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("status", ctypes.c_int32),
                ("bad_subdomain", ctypes.c_int32), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double), ("ms_setup", ctypes.c_double), ("ms_factor", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("applies", ctypes.c_int32), ("applies_graphed", ctypes.c_int32)]


class mbddc_material(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_double * 6)]


class mbddc_boundary(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tag", ctypes.c_uint32), ("instance", ctypes.c_int32),
                ("p", ctypes.c_double * 2)]


class mbddc_sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_dofs", "n_free", "n_interface", "n_coarse", "n_sub",
                                               "n_instances", "n_vertices", "n_edges", "n_faces", "max_local",
                                               "bsr_blocks", "n_sub2", "n_coarse2")]


class mbddc_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class mbddc_request(ctypes.Structure):
    _fields_ = [("mesh", mbddc_mesh), ("opt", mbddc_options), ("n_steps", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("lagged", ctypes.c_int32), ("elem_K", _f64p), ("rhs", _f64p), ("x", _f64p),
                ("material", ctypes.c_void_p), ("frames", _f64p), ("u0", _f64p), ("f_ext", _f64p)]


class mbddc_request_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("iterations", ctypes.c_int32 * 16),
                ("rel_res_true", ctypes.c_double), ("newton_res", ctypes.c_double * 16),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("footprint", ctypes.c_size_t)]


_lib = None

# (name, argtypes) for every entry point of include/mbddc.h
_SIGNATURES = {
    "mbddc_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p],
    "mbddc_default_options": [ctypes.POINTER(mbddc_options)],
    "mbddc_setup_symbolic": [ctypes.c_void_p, ctypes.POINTER(mbddc_mesh), ctypes.POINTER(mbddc_options)],
    "mbddc_setup_symbolic_batch": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(mbddc_mesh),
                                   ctypes.POINTER(mbddc_options)],
    "mbddc_footprint": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "mbddc_estimate_footprint": [ctypes.c_int, ctypes.POINTER(mbddc_mesh), ctypes.POINTER(mbddc_options),
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "mbddc_set_allocator": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "mbddc_release": [ctypes.c_void_p],
    "mbddc_get_iterations": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                             ctypes.POINTER(ctypes.c_int64)],
    "mbddc_get_sizes": [ctypes.c_void_p, ctypes.POINTER(mbddc_sizes)],
    "mbddc_set_tangent": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "mbddc_factor": [ctypes.c_void_p],
    "mbddc_set_material": [ctypes.c_void_p, ctypes.POINTER(mbddc_material), _f64p],
    "mbddc_set_displacement": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
    "mbddc_set_boundary": [ctypes.c_void_p, ctypes.POINTER(mbddc_boundary), ctypes.c_int],
    "mbddc_get_element_tangents": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "mbddc_solve": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                    ctypes.POINTER(mbddc_info)],
    "mbddc_apply": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "mbddc_matvec": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "mbddc_matvec_noalloc": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "mbddc_get_globs": [ctypes.c_void_p, _i32p, _i32p, _i32p, _i32p, _i32p],
    "mbddc_get_coarse_matrix": [ctypes.c_void_p, ctypes.c_int, _f64p, ctypes.c_int64],
    "mbddc_get_bsr": [ctypes.c_void_p, _i32p, _i32p, _f64p],
    "mbddc_inspect_symbolic": [ctypes.POINTER(mbddc_mesh), ctypes.c_uint32, ctypes.POINTER(mbddc_sizes), _i32p,
                               _i32p, _i32p, _i32p, _i32p],
    "mbddc_last_bad_subdomain": [ctypes.c_void_p],
    "mbddc_set_profiling": [ctypes.c_void_p, ctypes.c_uint32],
    "mbddc_autotune": [ctypes.c_void_p, ctypes.c_char_p],
    "mbddc_get_tuning": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "mbddc_profile_family_name": [ctypes.c_int],
    "mbddc_get_profile": [ctypes.c_void_p, ctypes.POINTER(mbddc_kernel_stat), ctypes.c_int,
                          ctypes.POINTER(ctypes.c_int)],
    "mbddc_destroy": [ctypes.c_void_p],
    "mbddc_strerror": [ctypes.c_int],
    "mbddc_server_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_size_t, ctypes.c_int],
    "mbddc_server_submit": [ctypes.c_void_p, ctypes.POINTER(mbddc_request), ctypes.POINTER(ctypes.c_int64)],
    "mbddc_server_wait": [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(mbddc_request_result)],
    "mbddc_server_state": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_size_t)],
    "mbddc_server_destroy": [ctypes.c_void_p],
    "mbddc_server_pool_stats": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
}

# device memory provider callbacks of mbddc_set_allocator
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        try:
            # torch ships its own HIP runtime under the same soname; loading it first makes the
            # library bind to that runtime, so device memory and streams are shared with torch
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("mbddc_strerror", "mbddc_profile_family_name") else ctypes.c_int
        _lib = L
    return _lib


class MbddcError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {lib().mbddc_strerror(status).decode()} ({status})")
        self.status = status


def _check(st: int, where: str):
    if st != MBDDC_OK:
        raise MbddcError(st, where)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


class _MeshArrays:
    """Keeps the numpy buffers of an mbddc_mesh alive."""

    def __init__(self, coords, elem_nodes, elem_type, elem_part, n_sub, node_tags, dirichlet):
        self.coords = None if coords is None else np.ascontiguousarray(coords, dtype=np.float64)
        self.elem_nodes = np.ascontiguousarray(elem_nodes, dtype=np.int32)
        self.elem_part = np.ascontiguousarray(elem_part, dtype=np.int32)
        self.node_tags = None if node_tags is None else np.ascontiguousarray(node_tags, dtype=np.uint32)
        self.dirichlet = np.ascontiguousarray(dirichlet, dtype=np.int32)
        n_nodes = int(self.elem_nodes.max()) + 1 if self.coords is None else self.coords.shape[0]
        self.mesh = mbddc_mesh(n_nodes, _ptr(self.coords, ctypes.c_double), self.elem_nodes.shape[0], elem_type,
                               _ptr(self.elem_nodes, ctypes.c_int32), int(n_sub), _ptr(self.elem_part, ctypes.c_int32),
                               _ptr(self.node_tags, ctypes.c_uint32), len(self.dirichlet),
                               _ptr(self.dirichlet, ctypes.c_int32))


def mesh_from_problem(P) -> _MeshArrays:
    """mbddc_mesh of a workloads.Problem."""
    m = P.mesh
    return _MeshArrays(m.coords, m.elem_nodes, m.elem_type, P.elem_part, P.n_sub, m.node_tags, P.dirichlet)


def default_options(**kw) -> mbddc_options:
    o = mbddc_options()
    _check(lib().mbddc_default_options(ctypes.byref(o)), "mbddc_default_options")
    for k, v in kw.items():
        if k == "tune_table" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def profile_families() -> list:
    """Profiler family names; bit i of a profiling mask selects family i."""
    out = []
    while True:
        n = lib().mbddc_profile_family_name(len(out))
        if not n:
            return out
        out.append(n.decode())


def mbddc_inspect_symbolic(mesh: _MeshArrays, primal: int):
    """Host-only symbolic setup: (sizes, node_glob, glob_kind, coarse_glob, coarse_comp, sub_counts)."""
    L = lib()
    sz = mbddc_sizes()
    _check(L.mbddc_inspect_symbolic(ctypes.byref(mesh.mesh), primal, ctypes.byref(sz), None, None, None, None, None),
           "mbddc_inspect_symbolic")
    ng = sz.n_vertices + sz.n_edges + sz.n_faces
    node_glob = np.empty(mesh.mesh.n_nodes, np.int32)
    kind = np.empty(max(ng, 1), np.int32)
    cg = np.empty(max(sz.n_coarse, 1), np.int32)
    cc = np.empty(max(sz.n_coarse, 1), np.int32)
    sc = np.empty(3 * sz.n_sub, np.int32)
    _check(L.mbddc_inspect_symbolic(ctypes.byref(mesh.mesh), primal, ctypes.byref(sz), _ptr(node_glob, ctypes.c_int32),
                                    _ptr(kind, ctypes.c_int32), _ptr(cg, ctypes.c_int32), _ptr(cc, ctypes.c_int32),
                                    _ptr(sc, ctypes.c_int32)), "mbddc_inspect_symbolic")
    return sz, node_glob, kind[:ng], cg[:sz.n_coarse], cc[:sz.n_coarse], sc.reshape(-1, 3)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def mbddc_estimate_footprint(meshes: Sequence[_MeshArrays], options: Optional[mbddc_options] = None,
                             nrhs: int = 4) -> int:
    """Host-only estimate of the device bytes of a handle for these meshes after a solve of
    nrhs right-hand sides (no device needed)."""
    arr = (mbddc_mesh * len(meshes))(*[m.mesh for m in meshes])
    o = options if options is not None else default_options()
    b = ctypes.c_size_t()
    _check(lib().mbddc_estimate_footprint(len(meshes), arr, ctypes.byref(o), nrhs, ctypes.byref(b)),
           "mbddc_estimate_footprint")
    return b.value


class TorchAllocator:
    """Device memory for a handle from PyTorch's caching allocator (mbddc_set_allocator):
    each block is a uint8 tensor kept alive until the library returns it. Counts calls."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self.blocks = {}
        self.n_alloc = 0
        self.n_free = 0
        self.c_alloc = ALLOC_FN(self._alloc)
        self.c_free = FREE_FN(self._free)

    def _alloc(self, nbytes, _user):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=f"cuda:{self.device}")
        except RuntimeError:
            return None
        self.blocks[t.data_ptr()] = t
        self.n_alloc += 1
        return t.data_ptr()

    def _free(self, ptr, _user):
        self.n_free += 1
        self.blocks.pop(int(ptr), None)


class Server:
    """Serving loop: requests of Newton tangent solves, admitted by footprint, run concurrently."""

    def __init__(self, device: int = 0, hbm_budget: int = 64 << 30, max_active: int = 4):
        self._s = ctypes.c_void_p()
        _check(lib().mbddc_server_create(ctypes.byref(self._s), device, int(hbm_budget), max_active),
               "mbddc_server_create")
        self._keep = {}

    def submit(self, mesh: _MeshArrays, options: mbddc_options, elem_K_steps: np.ndarray, rhs_steps: np.ndarray,
               lagged: bool = True) -> int:
        """elem_K_steps [n_steps, n_elems, 3npe, 3npe]; rhs_steps [n_steps, nrhs, n_dofs]. Returns a ticket."""
        K = np.ascontiguousarray(elem_K_steps, dtype=np.float64)
        b = np.ascontiguousarray(rhs_steps, dtype=np.float64)
        x = np.zeros_like(b)
        q = mbddc_request(mesh.mesh, options, K.shape[0], b.shape[1], 1 if lagged else 0,
                          _ptr(K, ctypes.c_double), _ptr(b, ctypes.c_double), _ptr(x, ctypes.c_double))
        t = ctypes.c_int64()
        _check(lib().mbddc_server_submit(self._s, ctypes.byref(q), ctypes.byref(t)), "mbddc_server_submit")
        self._keep[t.value] = (mesh, K, b, x)
        return t.value

    def submit_newton(self, mesh: _MeshArrays, options: mbddc_options, material, u0: np.ndarray, f_ext: np.ndarray,
                      n_steps: int = 5, lagged: bool = True, frames=None) -> int:
        """On-device Newton request: material (kind, params), u0 and f_ext full DOF vectors;
        the result's x holds the iterates u_1..u_n_steps [n_steps, 1, n_dofs]."""
        mat = mbddc_material()
        mat.kind = material[0]
        for j, v in enumerate(material[1]):
            mat.p[j] = float(v)
        u = np.ascontiguousarray(u0, dtype=np.float64).ravel()
        f = np.ascontiguousarray(f_ext, dtype=np.float64).ravel()
        fr = None if frames is None else np.ascontiguousarray(frames, dtype=np.float64)
        x = np.zeros((n_steps, 1, u.size))
        q = mbddc_request(mesh.mesh, options, n_steps, 1, 1 if lagged else 0, None, None, _ptr(x, ctypes.c_double),
                          ctypes.cast(ctypes.pointer(mat), ctypes.c_void_p), _ptr(fr, ctypes.c_double),
                          _ptr(u, ctypes.c_double), _ptr(f, ctypes.c_double))
        t = ctypes.c_int64()
        _check(lib().mbddc_server_submit(self._s, ctypes.byref(q), ctypes.byref(t)), "mbddc_server_submit")
        self._keep[t.value] = (mesh, (mat, u, f, fr), None, x)
        return t.value

    def wait(self, ticket: int):
        """(result, x [n_steps, nrhs, n_dofs]) of a submitted request."""
        r = mbddc_request_result()
        _check(lib().mbddc_server_wait(self._s, ticket, ctypes.byref(r)), "mbddc_server_wait")
        _, _, _, x = self._keep.pop(ticket)
        return r, x

    def pool_stats(self) -> dict:
        m, f, u, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().mbddc_server_pool_stats(self._s, ctypes.byref(m), ctypes.byref(f), ctypes.byref(u),
                                             ctypes.byref(c)), "mbddc_server_pool_stats")
        return {"device_mallocs": m.value, "device_frees": f.value, "bytes_in_use": u.value, "bytes_cached": c.value}

    def state(self):
        q, a, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().mbddc_server_state(self._s, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b)),
               "mbddc_server_state")
        return q.value, a.value, b.value

    def close(self):
        if self._s:
            lib().mbddc_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One handle: setup_symbolic -> set_tangent -> factor -> solve/apply/matvec."""

    def __init__(self, device: int = 0, stream=None, allocator: Optional[TorchAllocator] = None):
        """allocator: e.g. TorchAllocator(device) to take every device buffer from PyTorch's
        caching allocator (mbddc_set_allocator); None: the library's hipMalloc."""
        self._h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(int(stream))
        _check(lib().mbddc_create(ctypes.byref(self._h), device, s), "mbddc_create")
        self.allocator = allocator
        if allocator is not None:
            _check(lib().mbddc_set_allocator(self._h, ctypes.cast(allocator.c_alloc, ctypes.c_void_p),
                                             ctypes.cast(allocator.c_free, ctypes.c_void_p), None),
                   "mbddc_set_allocator")
        self._meshes = []
        self.n_dofs = 0

    def close(self):
        if self._h:
            lib().mbddc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def mbddc_release(self):
        _check(lib().mbddc_release(self._h), "mbddc_release")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ------------------------------------------------------------------
    def mbddc_setup_symbolic(self, meshes: Sequence[_MeshArrays], options: Optional[mbddc_options] = None):
        self._meshes = list(meshes)
        arr = (mbddc_mesh * len(meshes))(*[m.mesh for m in meshes])
        o = options if options is not None else default_options()
        _check(lib().mbddc_setup_symbolic_batch(self._h, len(meshes), arr, ctypes.byref(o)), "mbddc_setup_symbolic")
        self.n_dofs = self.sizes().n_dofs

    def sizes(self) -> mbddc_sizes:
        s = mbddc_sizes()
        _check(lib().mbddc_get_sizes(self._h, ctypes.byref(s)), "mbddc_get_sizes")
        return s

    def mbddc_footprint(self, nrhs: int = 4) -> int:
        b = ctypes.c_size_t()
        _check(lib().mbddc_footprint(self._h, nrhs, ctypes.byref(b)), "mbddc_footprint")
        return b.value

    def mbddc_get_iterations(self) -> np.ndarray:
        """GMRES iterations of each system of the last solve, [n_instances, nrhs]."""
        n = ctypes.c_int64()
        _check(lib().mbddc_get_iterations(self._h, None, 0, ctypes.byref(n)), "mbddc_get_iterations")
        out = np.zeros(max(n.value, 1), np.int32)
        _check(lib().mbddc_get_iterations(self._h, _ptr(out, ctypes.c_int32), n.value, ctypes.byref(n)),
               "mbddc_get_iterations")
        return out[:n.value].reshape(self.sizes().n_instances, -1)

    def mbddc_set_tangent(self, Ke):
        if isinstance(Ke, np.ndarray):
            Ke = np.ascontiguousarray(Ke, dtype=np.float64)
            _check(lib().mbddc_set_tangent(self._h, Ke.ctypes.data_as(ctypes.c_void_p), 0), "mbddc_set_tangent")
        else:
            _check(lib().mbddc_set_tangent(self._h, _dev_ptr(Ke), 1), "mbddc_set_tangent")

    def mbddc_factor(self):
        _check(lib().mbddc_factor(self._h), "mbddc_factor")

    # -- element kernels ---------------------------------------------------------
    def mbddc_set_material(self, materials, frames=None):
        """materials: one (kind, params) per instance, params as in mbddc.h; frames [n_elems, 3, 3]
        (rows f, s, n) for Guccione instances."""
        arr = (mbddc_material * len(materials))()
        for k, (kind, params) in enumerate(materials):
            arr[k].kind = kind
            for j, v in enumerate(params):
                arr[k].p[j] = float(v)
        fr = None if frames is None else np.ascontiguousarray(frames, dtype=np.float64)
        _check(lib().mbddc_set_material(self._h, arr, _ptr(fr, ctypes.c_double)), "mbddc_set_material")
        self._frames = fr

    def mbddc_set_boundary(self, conditions):
        """conditions: (kind, tag bits, instance (-1: all), params) per boundary condition."""
        arr = (mbddc_boundary * max(1, len(conditions)))()
        for k, (kind, tag, inst, params) in enumerate(conditions):
            arr[k].kind, arr[k].tag, arr[k].instance = kind, tag, inst
            for j, v in enumerate(params):
                arr[k].p[j] = float(v)
        _check(lib().mbddc_set_boundary(self._h, arr, len(conditions)), "mbddc_set_boundary")

    def mbddc_set_displacement(self, u, f_int: bool = False):
        """Device element tangents at u (full DOF vector, numpy or a device tensor); returns the
        internal forces (same kind of array as u) when f_int, else None."""
        if isinstance(u, np.ndarray):
            u2 = np.ascontiguousarray(u, dtype=np.float64).ravel()
            f = np.empty_like(u2) if f_int else None
            _check(lib().mbddc_set_displacement(self._h, u2.ctypes.data_as(ctypes.c_void_p), 0,
                                                None if f is None else f.ctypes.data_as(ctypes.c_void_p), 0),
                   "mbddc_set_displacement")
            return f
        f = u.new_empty(u.shape) if f_int else None
        _check(lib().mbddc_set_displacement(self._h, _dev_ptr(u), 1, None if f is None else _dev_ptr(f), 1),
               "mbddc_set_displacement")
        return f

    def mbddc_get_element_tangents(self, out=None):
        """The element matrices of the current operator (numpy [ke_total], or into a device tensor)."""
        if out is None:
            sz = self.sizes()
            n = sum(int(m.mesh.n_elems) * (3 * (8 if m.mesh.elem_type == MBDDC_HEX8 else 27)) ** 2
                    for m in self._meshes)
            o = np.empty(n)
            _check(lib().mbddc_get_element_tangents(self._h, o.ctypes.data_as(ctypes.c_void_p), 0),
                   "mbddc_get_element_tangents")
            return o
        _check(lib().mbddc_get_element_tangents(self._h, _dev_ptr(out), 1), "mbddc_get_element_tangents")
        return out

    def last_bad_subdomain(self) -> int:
        return lib().mbddc_last_bad_subdomain(self._h)

    # -- per-call ----------------------------------------------------------------
    def _vec_call(self, fn, name, v, out=None):
        if isinstance(v, np.ndarray):
            v2 = np.ascontiguousarray(np.atleast_2d(v), dtype=np.float64)
            o = np.empty_like(v2) if out is None else out
            st = fn(self._h, v2.shape[0], v2.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p), 0)
            _check(st, name)
            return o if v.ndim == 2 else o[0]
        nrhs = 1 if v.dim() == 1 else v.shape[0]
        o = out if out is not None else v.new_empty(v.shape)
        _check(fn(self._h, nrhs, _dev_ptr(v), _dev_ptr(o), 1), name)
        return o

    def mbddc_apply(self, r, out=None):
        return self._vec_call(lib().mbddc_apply, "mbddc_apply", r, out)

    def mbddc_matvec(self, x, out=None):
        return self._vec_call(lib().mbddc_matvec, "mbddc_matvec", x, out)

    def mbddc_matvec_noalloc(self, x, out):
        """y = K x with the library's static scratch buffer (no allocation); x and out are
        contiguous float64 device tensors [nrhs, n_dofs] (or [n_dofs])."""
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(lib().mbddc_matvec_noalloc(self._h, nrhs, _dev_ptr(x), _dev_ptr(out)), "mbddc_matvec_noalloc")
        return out

    def mbddc_solve(self, b, out=None, raise_on_noconv: bool = True):
        info = mbddc_info()
        if isinstance(b, np.ndarray):
            b2 = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
            x = np.empty_like(b2) if out is None else out
            st = lib().mbddc_solve(self._h, b2.shape[0], b2.ctypes.data_as(ctypes.c_void_p),
                                   x.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(info))
            res = x if b.ndim == 2 else x[0]
        else:
            nrhs = 1 if b.dim() == 1 else b.shape[0]
            x = out if out is not None else b.new_empty(b.shape)
            st = lib().mbddc_solve(self._h, nrhs, _dev_ptr(b), _dev_ptr(x), 1, ctypes.byref(info))
            res = x
        if st != MBDDC_OK and (raise_on_noconv or st != MBDDC_ERR_NOCONV):
            raise MbddcError(st, "mbddc_solve")
        return res, info

    # -- tuning --------------------------------------------------------------------
    def mbddc_autotune(self, table_out=None) -> dict:
        """Times the kernel variants on this handle's matrices, keeps the fastest (see mbddc.h)
        and optionally writes the table; returns it."""
        path = None if table_out is None else str(table_out).encode()
        _check(lib().mbddc_autotune(self._h, path), "mbddc_autotune")
        return self.mbddc_get_tuning()

    def mbddc_get_tuning(self) -> dict:
        a64 = (ctypes.c_int32 * 4)()
        a32 = (ctypes.c_int32 * 4)()
        xc = ctypes.c_int32()
        rows = (ctypes.c_int32 * 4)()
        gm = ctypes.c_int32()
        _check(lib().mbddc_get_tuning(self._h, a64, a32, ctypes.byref(xc), rows, ctypes.byref(gm)), "mbddc_get_tuning")
        return {"sym_fp64": list(a64), "sym_fp32": list(a32), "apply_xchunk": xc.value, "apply_rows": list(rows),
                "gemm_mfma": gm.value}

    # -- profiling -----------------------------------------------------------------
    def mbddc_set_profiling(self, mask: int = 0xFFFFFFFF):
        _check(lib().mbddc_set_profiling(self._h, mask & 0xFFFFFFFF), "mbddc_set_profiling")

    def mbddc_get_profile(self) -> dict:
        """{family: {launches, ms, bytes, flops}} since the last call (counters reset)."""
        buf = (mbddc_kernel_stat * 64)()
        n = ctypes.c_int()
        _check(lib().mbddc_get_profile(self._h, buf, 64, ctypes.byref(n)), "mbddc_get_profile")
        return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms, bytes=buf[i].bytes,
                                           flops=buf[i].flops) for i in range(min(n.value, 64))}

    # -- inspection ----------------------------------------------------------------
    def mbddc_get_globs(self):
        sz = self.sizes()
        ng = ctypes.c_int32()
        node_glob = np.empty(sz.n_dofs // 3, np.int32)
        _check(lib().mbddc_get_globs(self._h, _ptr(node_glob, ctypes.c_int32), ctypes.byref(ng), None, None, None),
               "mbddc_get_globs")
        kind = np.empty(max(ng.value, 1), np.int32)
        cg = np.empty(max(sz.n_coarse, 1), np.int32)
        cc = np.empty(max(sz.n_coarse, 1), np.int32)
        _check(lib().mbddc_get_globs(self._h, None, None, _ptr(kind, ctypes.c_int32), _ptr(cg, ctypes.c_int32),
                                     _ptr(cc, ctypes.c_int32)), "mbddc_get_globs")
        return node_glob, kind[:ng.value], cg[:sz.n_coarse], cc[:sz.n_coarse]

    def mbddc_get_coarse_matrix(self, inst: int, n_c: int) -> np.ndarray:
        out = np.empty((n_c, n_c))
        _check(lib().mbddc_get_coarse_matrix(self._h, inst, _ptr(out, ctypes.c_double), n_c),
               "mbddc_get_coarse_matrix")
        return out

    def mbddc_get_bsr(self):
        sz = self.sizes()
        nn = sz.n_dofs // 3
        rowptr = np.empty(nn + 1, np.int32)
        col = np.empty(sz.bsr_blocks, np.int32)
        vals = np.empty(9 * sz.bsr_blocks)
        _check(lib().mbddc_get_bsr(self._h, _ptr(rowptr, ctypes.c_int32), _ptr(col, ctypes.c_int32),
                                   _ptr(vals, ctypes.c_double)), "mbddc_get_bsr")
        return rowptr, col, vals.reshape(-1, 3, 3)
