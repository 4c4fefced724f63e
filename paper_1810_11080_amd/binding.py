"""ctypes binding of libsnsweep.so (argument marshalling only).

Every ``snsw_*`` function of ``include/snsweep.h`` is available under the
same name through :func:`lib`; :class:`Context` and :class:`Problem` wrap the
handles.  Device arrays are PyTorch tensors (float64, contiguous, on the
context's device); only their data pointers cross the boundary.  There is no
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

c_double_p = C.POINTER(C.c_double)
c_int32_p = C.POINTER(C.c_int32)
c_int64_p = C.POINTER(C.c_int64)


class SnswProblemDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32 * 3), ("geom_order", C.c_int32),
                ("dg_order", C.c_int32), ("lattice", c_double_p), ("sn_order", C.c_int32),
                ("n_dirs", C.c_int32), ("omega", c_double_p), ("w", c_double_p),
                ("sigma_t", c_double_p), ("sigma_s", c_double_p), ("q", c_double_p),
                ("q_per_dof", C.c_int32), ("bc_kind", C.c_int32), ("psi_inc", C.c_double),
                ("weighting", C.c_int32), ("exact_scc_max", C.c_int32),
                ("precision", C.c_int32), ("n_threads", C.c_int32), ("schedule", C.c_int32),
                ("cache_inverse", C.c_int32), ("psi_inc_tab", c_double_p),
                ("n_nodes", C.c_int64), ("nodes", c_double_p), ("elem_nodes", C.POINTER(C.c_int64)),
                ("element", C.c_int32), ("face_rule", C.c_int32), ("face_tol", C.c_double),
                ("cache_budget", C.c_double)]


class SnswProblemInfo(C.Structure):
    _fields_ = [("n_elements", C.c_int64), ("n_dofs_per_element", C.c_int64),
                ("n_dirs", C.c_int64), ("n_levels_total", C.c_int64), ("n_pairs", C.c_int64),
                ("n_edges_total", C.c_int64), ("n_removed_total", C.c_int64),
                ("n_kink_faces_total", C.c_int64), ("setup_seconds", C.c_double),
                ("cached_inverse", C.c_int32), ("schedule", C.c_int32), ("tile", C.c_int32),
                ("cached_dirs", C.c_int32), ("inverse_block_bytes", C.c_int64)]


class SnswGraphStats(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("n_scc_simple", C.c_int64), ("n_scc_large", C.c_int64),
                ("n_elements_in_large", C.c_int64), ("max_scc", C.c_int64),
                ("n_removed", C.c_int64), ("n_levels", C.c_int64), ("removed_weight", C.c_int64)]


class SnswSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int32), ("check_every", C.c_int32),
                ("precond", C.c_void_p), ("precond_every", C.c_int32)]


class SnswSolveReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("residual", C.c_double), ("seconds", C.c_double),
                ("history", c_double_p), ("history_cap", C.c_int32), ("n_corrected", C.c_int32),
                ("n_rejected", C.c_int32)]


class SnswNetDesc(C.Structure):
    _fields_ = [("widths", C.c_int32 * 3), ("seed", C.c_uint64)]


class SnswAdam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class SnswBatchOpts(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("use_graph", C.c_int32), ("tune_reps", C.c_int32)]


class SnswBatchClassInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("dg_order", C.c_int32), ("precision", C.c_int32),
                ("persistent", C.c_int32), ("blocks", C.c_int32), ("n_problems", C.c_int32),
                ("n_levels", C.c_int64), ("n_entries", C.c_int64), ("tuned_ms", C.c_double * 4),
                ("tiled", C.c_int32)]


# name -> (restype, argtypes); mirrors include/snsweep.h
SIGNATURES = {
    "snsw_last_error": (C.c_char_p, []),
    "snsw_version": (C.c_char_p, []),
    "snsw_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "snsw_ctx_destroy": (None, [C.c_void_p]),
    "snsw_problem_create": (C.c_int, [C.c_void_p, C.POINTER(SnswProblemDesc), C.POINTER(C.c_void_p)]),
    "snsw_problem_destroy": (None, [C.c_void_p]),
    "snsw_problem_get_info": (C.c_int, [C.c_void_p, C.POINTER(SnswProblemInfo)]),
    "snsw_get_quadrature": (C.c_int, [C.c_void_p, c_double_p, c_double_p]),
    "snsw_get_element_matrices": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, c_double_p, c_double_p]),
    "snsw_problem_set_source": (C.c_int, [C.c_void_p, C.c_int32, c_double_p, C.c_int32, C.c_double, c_double_p]),
    "snsw_get_node_coordinates": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, c_double_p]),
    "snsw_get_volume_rule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, c_int32_p, c_double_p,
                                       c_double_p, c_double_p]),
    "snsw_graph_stats_get": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(SnswGraphStats)]),
    "snsw_get_edges": (C.c_int, [C.c_void_p, C.c_int, c_int32_p, c_int32_p, c_int64_p, C.c_int64,
                                 c_int64_p]),
    "snsw_get_removed_edges": (C.c_int, [C.c_void_p, C.c_int, c_int32_p, c_int32_p, C.c_int64,
                                         c_int64_p]),
    "snsw_get_levels": (C.c_int, [C.c_void_p, C.c_int, c_int32_p]),
    "snsw_get_face_integrals": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, c_int32_p, c_double_p, c_double_p,
                                          c_double_p, c_double_p]),
    "snsw_sweep": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "snsw_reset": (C.c_int, [C.c_void_p]),
    "snsw_synchronize": (C.c_int, [C.c_void_p]),
    "snsw_set_wait_limit": (C.c_int, [C.c_void_p, C.c_int32]),
    "snsw_solve": (C.c_int, [C.c_void_p, C.POINTER(SnswSolveOpts), C.c_void_p, C.c_void_p,
                             C.POINTER(SnswSolveReport)]),
    "snsw_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, c_double_p]),
    "snsw_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "snsw_profile_read": (C.c_int, [C.c_void_p, c_int64_p, c_double_p]),
    "snsw_state_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "snsw_state_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "snsw_state_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "snsw_net_create": (C.c_int, [C.c_void_p, C.POINTER(SnswNetDesc), C.POINTER(C.c_void_p)]),
    "snsw_net_destroy": (None, [C.c_void_p]),
    "snsw_net_n_params": (C.c_int, [C.c_void_p, c_int64_p]),
    "snsw_net_get_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "snsw_net_set_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "snsw_net_get_grads": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "snsw_net_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_int32]),
    "snsw_net_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, c_double_p]),
    "snsw_net_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "snsw_net_step": (C.c_int, [C.c_void_p, C.POINTER(SnswAdam)]),
    "snsw_learn_pair": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "snsw_learn_pair_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
    "snsw_batch_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(SnswBatchOpts),
                                    C.POINTER(C.c_void_p)]),
    "snsw_batch_destroy": (None, [C.c_void_p]),
    "snsw_batch_sweep": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "snsw_batch_synchronize": (C.c_int, [C.c_void_p]),
    "snsw_batch_n_classes": (C.c_int, [C.c_void_p, c_int32_p]),
    "snsw_batch_class_get": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(SnswBatchClassInfo)]),
}

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "SHAPE", -3: "NONFINITE", -4: "BAD_JACOBIAN",
          -5: "NOT_CONVERGED", -6: "DIVERGED", -7: "HIP", -8: "OOM", -9: "UNSUPPORTED",
          -10: "STATE"}


def _q_kind(qa, E: int, n: int) -> int:
    """Layout code of a source array: 0 [E], 1 [E][n], 2 [D][E][n]."""
    if qa.size == E:
        return 0
    if qa.size == E * n:
        return 1
    if qa.size % (E * n) == 0:
        return 2
    raise ValueError(f"source has {qa.size} entries: expected E, E*n or D*E*n")


class SnswError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"snsweep error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


def library_path() -> str:
    return os.environ.get("SNSWEEP_LIB", os.path.join(_HERE, "libsnsweep.so"))


def lib():
    """Load libsnsweep.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_1810_11080_amd.build`")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != 0:
        raise SnswError(rc, lib().snsw_last_error().decode())


def _dptr(a: np.ndarray, dtype):
    return a.ctypes.data_as(C.POINTER(dtype))


def _tensor_ptr(t, numel: int, device: int, name: str):
    """Data pointer of a float64 contiguous device tensor of numel entries."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise TypeError(f"{name} must be a contiguous float64 device tensor")
    if t.device.index != device:
        raise ValueError(f"{name} is on device {t.device.index}, context uses {device}")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _f32_ptr(t, numel: int, device: int, name: str):
    """Data pointer of a float32 contiguous device tensor of numel entries."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    if t.device.index != device:
        raise ValueError(f"{name} is on device {t.device.index}, context uses {device}")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0, stream=None):
        """device = -1: host-only (setup and introspection only)."""
        self.device = device
        if stream is None and device >= 0:
            import torch
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        sp = C.c_void_p(stream.cuda_stream) if stream is not None else C.c_void_p()
        _check(lib().snsw_ctx_create(device, sp, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().snsw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A discretised S_N problem with its sweep schedule."""

    def __init__(self, ctx: Context, *, dim, nx, geom_order, dg_order, lattice, sn_order,
                 sigma_t, sigma_s, q, bc_kind=0, psi_inc=0.0, weighting=1, exact_scc_max=10,
                 precision=0, n_threads=0, omega=None, w=None, schedule=0, cache_inverse=0,
                 psi_inc_tab=None, nodes=None, elem_nodes=None, element=0, face_rule=0, face_tol=0.0,
                 cache_budget=0.0):
        """q: [E] or [E][n] isotropic, or [D][E][n] per direction (nodal
        values); psi_inc_tab: [D][E][n] incident flux for bc_kind 2.  With
        elem_nodes ([E][nv] control-point indices into nodes [n_nodes][dim])
        the mesh is unstructured: nx = (E, 1[, 1]) and lattice is ignored;
        element 0: Q_r quads / hexes, nv = (r+1)^dim; 1: P_r triangles
        (nv = (r+1)(r+2)/2, n = (p+1)(p+2)/2) or tetrahedra (nv =
        (r+1)(r+2)(r+3)/6, n = (p+1)(p+2)(p+3)/6).  face_rule 1: adaptive Romberg
        on faces where Omega . n changes sign, relative tolerance face_tol
        (<= 0: 1e-10).  cache_budget: bytes the cached inverses may take
        under cache_inverse AUTO (<= 0: half the free device memory); on the
        level schedule a smaller budget caches the first directions that
        fit."""
        self.ctx = ctx
        if dim not in (2, 3):
            raise SnswError(-1, "dim must be 2 or 3")
        E = int(np.prod(nx[:dim]))
        simplex = element == 1

        def count(k):   # nodes of order k on the element
            if not simplex:
                return (k + 1) ** dim
            return (k + 1) * (k + 2) // 2 if dim == 2 else (k + 1) * (k + 2) * (k + 3) // 6
        n, nv = count(dg_order), count(geom_order)
        self._keep = []

        def arr(x, size=None):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            if size is not None and a.size != size:
                raise ValueError(f"array has {a.size} entries, expected {size}")
            self._keep.append(a)
            return _dptr(a, C.c_double)

        desc = SnswProblemDesc()
        desc.dim = dim
        for a in range(3):
            desc.nx[a] = int(nx[a]) if a < len(nx) else 1
        desc.geom_order = geom_order
        desc.dg_order = dg_order
        if elem_nodes is None:
            L = int(np.prod([geom_order * int(nx[a]) + 1 for a in range(dim)]))
            desc.lattice = arr(lattice, L * dim)
        else:
            en = np.ascontiguousarray(np.asarray(elem_nodes, dtype=np.int64))
            if en.size != E * nv:
                raise ValueError(f"elem_nodes must have E*{nv} entries")
            self._keep.append(en)
            nd = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
            desc.n_nodes = nd.size // dim
            desc.nodes = arr(nd)
            desc.elem_nodes = en.ctypes.data_as(C.POINTER(C.c_int64))
        desc.sn_order = sn_order if omega is None else 0
        if omega is not None:
            desc.n_dirs = len(w)
            desc.omega = arr(omega, 3 * len(w))
            desc.w = arr(w, len(w))
        desc.sigma_t = arr(sigma_t, E)
        desc.sigma_s = arr(sigma_s, E)
        qa = np.asarray(q, dtype=np.float64)
        desc.q_per_dof = _q_kind(qa, E, n)
        desc.q = arr(qa)
        desc.bc_kind = bc_kind
        desc.psi_inc = psi_inc
        if psi_inc_tab is not None:
            desc.psi_inc_tab = arr(psi_inc_tab)
        desc.weighting = weighting
        desc.exact_scc_max = exact_scc_max
        desc.precision = precision
        desc.n_threads = n_threads
        desc.schedule = schedule
        desc.cache_inverse = cache_inverse
        desc.element = element
        desc.face_rule = face_rule
        desc.face_tol = face_tol
        desc.cache_budget = cache_budget
        h = C.c_void_p()
        _check(lib().snsw_problem_create(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h
        self._keep = []
        info = self.info()
        self.E, self.n, self.D = info["n_elements"], info["n_dofs_per_element"], info["n_dirs"]
        self.dim = dim
        self.nx = tuple(int(v) for v in nx[:dim])

    @classmethod
    def from_workload(cls, ctx: Context, prob, precision=0, n_threads=0, weighting=None,
                      exact_scc_max=None, schedule=0, cache_inverse=0, cache_budget=0.0):
        """Build from a ``workloads.Problem`` (seeded synthetic inputs)."""
        q_dir = getattr(prob, "q_dir", None)
        return cls(ctx, dim=prob.dim, nx=tuple(prob.nx), geom_order=prob.r, dg_order=prob.p,
                   lattice=prob.lattice, sn_order=prob.sn_order, sigma_t=prob.sigma_t,
                   sigma_s=prob.sigma_s, q=prob.q if q_dir is None else q_dir, bc_kind=prob.bc_kind,
                   psi_inc=prob.psi_inc, psi_inc_tab=getattr(prob, "psi_inc_tab", None),
                   weighting=prob.weighting if weighting is None else weighting,
                   exact_scc_max=prob.exact_scc_max if exact_scc_max is None else exact_scc_max,
                   precision=precision, n_threads=n_threads, schedule=schedule,
                   cache_inverse=cache_inverse, nodes=getattr(prob, "nodes", None),
                   elem_nodes=getattr(prob, "elem_nodes", None),
                   element=1 if getattr(prob, "element", "tensor") == "simplex" else 0,
                   face_rule=1 if getattr(prob, "face_rule", "exact") == "romberg" else 0,
                   face_tol=getattr(prob, "face_tol", 1e-10), cache_budget=cache_budget)

    def set_source(self, q, bc_kind=0, psi_inc=0.0, psi_inc_tab=None):
        """Replace the volume source and boundary condition (snsw_problem_set_source)."""
        qa = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
        kind = _q_kind(qa, self.E, self.n)
        tab = None if psi_inc_tab is None else np.ascontiguousarray(np.asarray(psi_inc_tab, dtype=np.float64))
        if tab is not None and tab.size != self.D * self.E * self.n:
            raise ValueError("psi_inc_tab must have D*E*n entries")
        if kind == 2 and qa.size != self.D * self.E * self.n:
            raise ValueError("a per-direction source must have D*E*n entries")
        _check(lib().snsw_problem_set_source(self.handle, kind, _dptr(qa, C.c_double), bc_kind, psi_inc,
                                             _dptr(tab, C.c_double) if tab is not None else None))

    def node_coordinates(self):
        """(E, n, dim) physical coordinates of the DG nodes."""
        out = np.zeros((self.E, self.n, self.dim))
        _check(lib().snsw_get_node_coordinates(self.handle, 0, self.E, _dptr(out, C.c_double)))
        return out

    def volume_rule(self, extra=0):
        """(x (E, Q, dim), wdet (E, Q), basis (Q, n)) of the tensor Gauss rule
        with `extra` points per axis beyond the element-matrix rule."""
        Q = C.c_int32()
        _check(lib().snsw_get_volume_rule(self.handle, extra, 0, self.E, C.byref(Q), None, None, None))
        x = np.zeros((self.E, Q.value, self.dim))
        wd = np.zeros((self.E, Q.value))
        basis = np.zeros((Q.value, self.n))
        _check(lib().snsw_get_volume_rule(self.handle, extra, 0, self.E, C.byref(Q), _dptr(x, C.c_double),
                                          _dptr(wd, C.c_double), _dptr(basis, C.c_double)))
        return x, wd, basis

    def close(self):
        if getattr(self, "handle", None):
            lib().snsw_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ introspection
    def info(self) -> dict:
        i = SnswProblemInfo()
        _check(lib().snsw_problem_get_info(self.handle, C.byref(i)))
        return {k: getattr(i, k) for k, _ in SnswProblemInfo._fields_}

    def quadrature(self):
        om = np.zeros((self.D, 3))
        w = np.zeros(self.D)
        _check(lib().snsw_get_quadrature(self.handle, _dptr(om, C.c_double), _dptr(w, C.c_double)))
        return om, w

    def element_matrices(self, e0=0, count=None):
        count = self.E - e0 if count is None else count
        M = np.zeros((count, self.n, self.n))
        K = np.zeros((count, self.dim, self.n, self.n))
        _check(lib().snsw_get_element_matrices(self.handle, e0, count, _dptr(M, C.c_double),
                                               _dptr(K, C.c_double)))
        return M, K

    def graph_stats(self, d: int) -> dict:
        s = SnswGraphStats()
        _check(lib().snsw_graph_stats_get(self.handle, d, C.byref(s)))
        return {k: getattr(s, k) for k, _ in SnswGraphStats._fields_}

    def edges(self, d: int):
        cnt = C.c_int64()
        _check(lib().snsw_get_edges(self.handle, d, None, None, None, 0, C.byref(cnt)))
        m = cnt.value
        up = np.zeros(m, dtype=np.int32)
        down = np.zeros(m, dtype=np.int32)
        w = np.zeros(m, dtype=np.int64)
        _check(lib().snsw_get_edges(self.handle, d, _dptr(up, C.c_int32), _dptr(down, C.c_int32),
                                    _dptr(w, C.c_int64), m, C.byref(cnt)))
        return up, down, w

    def removed_edges(self, d: int):
        cnt = C.c_int64()
        _check(lib().snsw_get_removed_edges(self.handle, d, None, None, 0, C.byref(cnt)))
        m = cnt.value
        down = np.zeros(m, dtype=np.int32)
        up = np.zeros(m, dtype=np.int32)
        _check(lib().snsw_get_removed_edges(self.handle, d, _dptr(down, C.c_int32),
                                            _dptr(up, C.c_int32), m, C.byref(cnt)))
        return down, up

    def levels(self, d: int):
        lev = np.zeros(self.E, dtype=np.int32)
        _check(lib().snsw_get_levels(self.handle, d, _dptr(lev, C.c_int32)))
        return lev

    def face_integrals(self, d: int, f: int, nf: int):
        """(class, m_plus, m_minus, P_plus, P_minus) of face f, direction d."""
        cls = np.zeros(1, dtype=np.int32)
        m = np.zeros(2)
        Pp, Pm = np.zeros((nf, nf)), np.zeros((nf, nf))
        _check(lib().snsw_get_face_integrals(self.handle, d, f, _dptr(cls, C.c_int32), _dptr(m[0:], C.c_double),
                                             _dptr(m[1:], C.c_double), _dptr(Pp, C.c_double),
                                             _dptr(Pm, C.c_double)))
        return int(cls[0]), float(m[0]), float(m[1]), Pp, Pm

    # ------------------------------------------------------------------ device
    def sweep(self, phi_in, phi_out, psi_out=None):
        dev = self.ctx.device
        a = _tensor_ptr(phi_in, self.E * self.n, dev, "phi_in")
        b = _tensor_ptr(phi_out, self.E * self.n, dev, "phi_out")
        c = _tensor_ptr(psi_out, self.D * self.E * self.n, dev, "psi_out") if psi_out is not None \
            else C.c_void_p()
        _check(lib().snsw_sweep(self.handle, a, b, c))

    def reset(self):
        _check(lib().snsw_reset(self.handle))

    def synchronize(self):
        """Wait for the stream; raises if a device-side dependency wait failed."""
        _check(lib().snsw_synchronize(self.handle))

    def set_wait_limit(self, polls: int):
        """Polls per dependency wait of persistent sweeps before giving up."""
        _check(lib().snsw_set_wait_limit(self.handle, int(polls)))

    def residual(self, a, b) -> float:
        out = C.c_double()
        dev = self.ctx.device
        _check(lib().snsw_residual(self.handle, _tensor_ptr(a, self.E * self.n, dev, "a"),
                                   _tensor_ptr(b, self.E * self.n, dev, "b"), C.byref(out)))
        return out.value

    def solve(self, phi, tol=1e-8, max_iters=1000, check_every=1, psi=None, history_cap=0,
              raise_on_not_converged=True, precond=None, precond_every=1):
        dev = self.ctx.device
        opts = SnswSolveOpts(tol=tol, max_iters=max_iters, check_every=check_every,
                             precond=precond.handle if precond is not None else None,
                             precond_every=precond_every)
        hist = np.zeros(max(history_cap, 1))
        rep = SnswSolveReport()
        rep.history = _dptr(hist, C.c_double) if history_cap else None
        rep.history_cap = history_cap
        pp = _tensor_ptr(psi, self.D * self.E * self.n, dev, "psi") if psi is not None else C.c_void_p()
        rc = lib().snsw_solve(self.handle, C.byref(opts), _tensor_ptr(phi, self.E * self.n, dev, "phi"),
                              pp, C.byref(rep))
        if rc != 0 and (raise_on_not_converged or rc != -5):
            _check(rc)
        n_hist = min(history_cap, rep.iterations)
        return {"iterations": rep.iterations, "residual": rep.residual, "seconds": rep.seconds,
                "history": hist[:n_hist].copy() if history_cap else None, "status": rc,
                "n_corrected": rep.n_corrected, "n_rejected": rep.n_rejected}

    def learn_pair(self, phi_prev, phi_swept, phi_star, x, t):
        """Network input x (float32 [3][E]) and target t (float32 [E], or None)."""
        dev = self.ctx.device
        En = self.E * self.n
        star = _tensor_ptr(phi_star, En, dev, "phi_star") if phi_star is not None else C.c_void_p()
        tp = _f32_ptr(t, self.E, dev, "t") if t is not None else C.c_void_p()
        _check(lib().snsw_learn_pair(self.handle, _tensor_ptr(phi_prev, En, dev, "phi_prev"),
                                     _tensor_ptr(phi_swept, En, dev, "phi_swept"), star,
                                     _f32_ptr(x, 3 * self.E, dev, "x"), tp))

    def learn_pair_noalloc(self, phi_prev, phi_swept, phi_star, x, t):
        """As learn_pair, through the entry point that allocates nothing
        (static device scratch; enqueued only, not synchronous)."""
        dev = self.ctx.device
        En = self.E * self.n
        star = _tensor_ptr(phi_star, En, dev, "phi_star") if phi_star is not None else C.c_void_p()
        tp = _f32_ptr(t, self.E, dev, "t") if t is not None else C.c_void_p()
        _check(lib().snsw_learn_pair_noalloc(self.handle, _tensor_ptr(phi_prev, En, dev, "phi_prev"),
                                             _tensor_ptr(phi_swept, En, dev, "phi_swept"), star,
                                             _f32_ptr(x, 3 * self.E, dev, "x"), tp))

    def profile_enable(self, enable: bool = True):
        _check(lib().snsw_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self):
        """(level launches, summed kernel milliseconds) since the last read."""
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().snsw_profile_read(self.handle, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def state_save(self) -> bytes:
        size = C.c_size_t()
        _check(lib().snsw_state_size(self.handle, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        _check(lib().snsw_state_save(self.handle, buf, size.value))
        return buf.raw

    def state_load(self, data):
        """Restore from bytes or any contiguous buffer (e.g. a numpy array),
        read in place."""
        buf = np.frombuffer(data, dtype=np.uint8)
        _check(lib().snsw_state_load(self.handle, buf.ctypes.data_as(C.c_void_p), buf.nbytes))


class Batch:
    """Independent problems swept together (merged per-class schedules,
    autotuned schedule choice, hipGraph replay).  Keep the problems alive
    while the batch exists."""

    def __init__(self, ctx: Context, problems, schedule: int = 0, use_graph: bool = True,
                 tune_reps: int = 0):
        self.ctx = ctx
        self.problems = list(problems)
        handles = (C.c_void_p * len(self.problems))(*[p.handle.value for p in self.problems])
        opts = SnswBatchOpts(schedule=schedule, use_graph=1 if use_graph else 0, tune_reps=tune_reps)
        h = C.c_void_p()
        _check(lib().snsw_batch_create(ctx.handle, handles, len(self.problems), C.byref(opts), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().snsw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, phi_in, phi_out):
        """One sweep of every problem: phi_in[k] -> phi_out[k] (device tensors)."""
        n = len(self.problems)
        if len(phi_in) != n or len(phi_out) != n:
            raise ValueError(f"expected {n} input and output tensors")
        dev = self.ctx.device
        a = (C.c_void_p * n)(*[_tensor_ptr(t, p.E * p.n, dev, f"phi_in[{k}]").value
                               for k, (t, p) in enumerate(zip(phi_in, self.problems))])
        b = (C.c_void_p * n)(*[_tensor_ptr(t, p.E * p.n, dev, f"phi_out[{k}]").value
                               for k, (t, p) in enumerate(zip(phi_out, self.problems))])
        _check(lib().snsw_batch_sweep(self.handle, a, b))

    def synchronize(self):
        _check(lib().snsw_batch_synchronize(self.handle))

    def classes(self):
        n = C.c_int32()
        _check(lib().snsw_batch_n_classes(self.handle, C.byref(n)))
        out = []
        for c in range(n.value):
            info = SnswBatchClassInfo()
            _check(lib().snsw_batch_class_get(self.handle, c, C.byref(info)))
            d = {k: getattr(info, k) for k, _ in info._fields_ if k != "tuned_ms"}
            d["tuned_ms"] = list(info.tuned_ms)
            out.append(d)
        return out


class Net:
    """The learned source-iteration correction (3D U-Net on the element grid)."""

    def __init__(self, ctx: Context, widths=(16, 32, 32), seed: int = 0):
        self.ctx = ctx
        self.widths = tuple(int(w) for w in widths)
        desc = SnswNetDesc(widths=(C.c_int32 * 3)(*self.widths), seed=seed)
        h = C.c_void_p()
        _check(lib().snsw_net_create(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h
        n = C.c_int64()
        _check(lib().snsw_net_n_params(h, C.byref(n)))
        self.n_params = n.value
        self._shape = None

    def close(self):
        if getattr(self, "handle", None):
            lib().snsw_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().snsw_net_get_params(self.handle, _dptr(out, C.c_float)))
        return out

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().snsw_net_set_params(self.handle, _dptr(a, C.c_float)))

    def get_grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().snsw_net_get_grads(self.handle, _dptr(out, C.c_float)))
        return out

    def forward(self, x, y, batch, nz, ny, nx):
        n = batch * nz * ny * nx
        dev = self.ctx.device
        _check(lib().snsw_net_forward(self.handle, _f32_ptr(x, 3 * n, dev, "x"), _f32_ptr(y, n, dev, "y"),
                                      batch, nz, ny, nx))
        self._shape = (batch, nz, ny, nx)

    def loss(self, y, t, dy) -> float:
        n = y.numel()
        dev = self.ctx.device
        out = C.c_double()
        _check(lib().snsw_net_loss(self.handle, _f32_ptr(y, n, dev, "y"), _f32_ptr(t, n, dev, "t"), n,
                                   _f32_ptr(dy, n, dev, "dy"), C.byref(out)))
        return out.value

    def backward(self, dy, dx=None):
        b, z, y, x = self._shape
        n = b * z * y * x
        dev = self.ctx.device
        dxp = _f32_ptr(dx, 3 * n, dev, "dx") if dx is not None else C.c_void_p()
        _check(lib().snsw_net_backward(self.handle, _f32_ptr(dy, n, dev, "dy"), dxp))

    def step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        opt = SnswAdam(lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        _check(lib().snsw_net_step(self.handle, C.byref(opt)))
