"""ctypes binding of libcutcell.so (include/cutcell.h): argument marshalling only.

Device arrays are torch tensors (float64, contiguous, on the GPU); every step of
the solve runs in the library's HIP kernels.  There is no fallback: if the
shared library is missing, `load()` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcutcell.so")

CC_OK, CC_EINVAL, CC_ENOMEM, CC_EDEVICE, CC_EGEOM, CC_EPLG, CC_ESINGULAR, CC_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
CC_FIELD = {"zero": 0, "poly": 1, "sinprod": 2, "expcos": 3, "gauss": 4, "xsinexp": 5}
CC_VALUE, CC_LAPLACIAN = 0, 1
CC_DIRICHLET, CC_NEUMANN, CC_ROBIN = 0, 1, 2
CC_ELLIPSOID, CC_TORUS = 0, 1
CC_FP64, CC_MIXED = 0, 1
HISTORY_MAX = 256
BATCH_MAX = 64
CC_TIME_SMO1, CC_TIME_SMO1_F32, CC_TIME_LU, CC_TIME_LU_F32, CC_TIME_COPY = 0, 1, 2, 3, 4

EXPORTED = [
    "cc_default_params", "cc_build", "cc_num_levels", "cc_get_level_info", "cc_assemble_rhs", "cc_solve",
    "cc_apply", "cc_residual", "cc_smo1", "cc_smo2", "cc_restrict", "cc_prolong_add", "cc_bottom_solve",
    "cc_vcycle", "cc_export_cells", "cc_export_plg", "cc_selfcheck_lu", "cc_export_lu_nodes", "cc_time_kernel",
    "cc_destroy", "cc_last_error", "cc_solve_batched", "cc_set_precision", "cc_set_krylov", "cc_solve_multi",
    "cc_set_lu_schedule", "cc_fmg", "cc_fmg_restrict", "cc_fmg_prolong", "cc_assemble_rhs_level",
    "cc_fmg_batched", "cc_set_stencil_schedule", "cc_get_stencil_schedule", "cc_fmg_noalloc", "cc_set_overlap", "cc_net_pairs",
    "cc_assemble_rhs_batched", "cc_fit_patches", "cc_solve_multi_graph",
    "cc_net_create", "cc_net_num_params", "cc_net_get_params", "cc_net_set_params", "cc_net_forward",
    "cc_net_loss_grad", "cc_net_adam_step", "cc_net_destroy", "cc_learned_guess", "cc_learned_fmg",
]


class CcObstacle(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("axes", C.c_double * 3), ("rot", C.c_double * 9), ("bc", C.c_int),
                ("robin", C.c_double * 2), ("kind", C.c_int), ("radii", C.c_double * 2)]


class CcDomain(C.Structure):
    _fields_ = [("n", C.c_int), ("origin", C.c_double * 3), ("h", C.c_double), ("wall_bc", C.c_int * 6),
                ("n_obst", C.c_int), ("obst", C.POINTER(CcObstacle)), ("inside", C.c_int),
                ("wall_robin", (C.c_double * 2) * 6)]


class CcParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("omega", C.c_double), ("nu1", C.c_int), ("nu2", C.c_int),
                ("n_min", C.c_int), ("max_iter", C.c_int), ("tol", C.c_double), ("precision", C.c_int),
                ("leaf_size", C.c_int), ("device", C.c_int), ("use_graph", C.c_int), ("krylov", C.c_int),
                ("pivot_tol", C.c_double), ("fit_on_device", C.c_int)]


class CcField(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_terms", C.c_int), ("data", C.POINTER(C.c_double))]


class CcSolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rel_residual", C.c_double), ("history_len", C.c_int),
                ("history", C.c_double * HISTORY_MAX), ("seconds", C.c_double)]


class CcLevelInfo(C.Structure):
    _fields_ = [("n", C.c_int), ("n_unknowns", C.c_longlong), ("n_phi2", C.c_longlong), ("n_cut", C.c_longlong),
                ("n_merged", C.c_longlong), ("lu_vars", C.c_longlong), ("lu_entries", C.c_longlong),
                ("lu_nodes", C.c_int), ("lu_depth", C.c_int), ("setup_seconds", C.c_double),
                ("lu_subtree_cut", C.c_int), ("lu_subtrees", C.c_int), ("lu_entries_per_lane", C.c_int),
                ("lu_tune_ms", C.c_double * 10), ("lu_waves_cap", C.c_int), ("stencil_march", C.c_int),
                ("stencil_planes", C.c_int), ("stencil_tune_us", C.c_double * 9), ("n_near", C.c_longlong),
                ("lu_seconds", C.c_double)]


class CutCellError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cutcell error {code}: {msg}")
        self.code = code


_LIB = None


def load() -> C.CDLL:
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_05865_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (same soname), so torch's streams and allocations are valid in it
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    P = C.POINTER
    lib.cc_default_params.argtypes = [P(CcParams)]
    lib.cc_default_params.restype = None
    lib.cc_build.argtypes = [P(CcDomain), P(CcParams), vp, P(vp)]
    lib.cc_num_levels.argtypes = [vp]
    lib.cc_get_level_info.argtypes = [vp, C.c_int, P(CcLevelInfo)]
    lib.cc_assemble_rhs.argtypes = [vp, P(CcField), C.c_int, P(CcField), vp]
    lib.cc_assemble_rhs_level.argtypes = [vp, C.c_int, P(CcField), C.c_int, P(CcField), vp]
    lib.cc_assemble_rhs_batched.argtypes = [vp, C.c_int, C.c_int, P(CcField), C.c_int, P(CcField), C.c_int, vp]
    lib.cc_solve.argtypes = [vp, vp, vp, P(CcSolveInfo)]
    lib.cc_apply.argtypes = [vp, C.c_int, vp, vp]
    lib.cc_residual.argtypes = [vp, C.c_int, vp, vp, vp, P(C.c_double)]
    for name in ("cc_smo1", "cc_smo2", "cc_prolong_add", "cc_vcycle"):
        getattr(lib, name).argtypes = [vp, C.c_int, vp, vp]
    lib.cc_restrict.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.cc_bottom_solve.argtypes = [vp, vp, vp]
    lib.cc_export_cells.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.cc_export_plg.argtypes = [vp, C.c_int, vp, vp, vp]
    lib.cc_selfcheck_lu.argtypes = [vp, C.c_int, P(C.c_double)]
    lib.cc_export_lu_nodes.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    lib.cc_set_precision.argtypes = [vp, C.c_int]
    lib.cc_set_krylov.argtypes = [vp, C.c_int]
    lib.cc_set_overlap.argtypes = [vp, C.c_int]
    lib.cc_set_lu_schedule.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.cc_set_stencil_schedule.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    lib.cc_get_stencil_schedule.argtypes = [vp, C.c_int, P(C.c_int), P(C.c_int)]
    lib.cc_fmg.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.cc_fmg_batched.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int]
    lib.cc_fmg_noalloc.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.cc_fmg_restrict.argtypes = [vp, C.c_int, vp, vp]
    lib.cc_fmg_prolong.argtypes = [vp, C.c_int, vp, vp]
    lib.cc_solve_multi.argtypes = [C.c_int, P(vp), P(vp), P(vp), P(CcSolveInfo)]
    lib.cc_solve_multi_graph.argtypes = [C.c_int, P(vp), P(vp), P(vp), P(CcSolveInfo)]
    lib.cc_fit_patches.argtypes = [vp, C.c_int, P(CcField), vp, vp, vp, vp, vp]
    lib.cc_net_create.argtypes = [C.c_int, C.c_int, C.c_ulonglong, vp, P(vp)]
    lib.cc_net_num_params.argtypes = [vp]
    lib.cc_net_num_params.restype = C.c_longlong
    lib.cc_net_get_params.argtypes = [vp, vp]
    lib.cc_net_set_params.argtypes = [vp, vp]
    lib.cc_net_forward.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    lib.cc_net_loss_grad.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, P(C.c_double), vp]
    lib.cc_net_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
    lib.cc_learned_guess.argtypes = [vp, vp, C.c_int, C.c_double, vp, vp]
    lib.cc_learned_fmg.argtypes = [vp, vp, C.c_int, C.c_double, vp, P(vp), vp, C.c_int]
    lib.cc_net_pairs.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_double, vp, vp, vp]
    lib.cc_net_destroy.argtypes = [vp]
    lib.cc_net_destroy.restype = None
    lib.cc_solve_batched.argtypes = [vp, C.c_int, vp, vp, P(CcSolveInfo)]
    lib.cc_time_kernel.argtypes = [vp, C.c_int, C.c_int, P(C.c_double), P(C.c_double)]
    lib.cc_destroy.argtypes = [vp]
    lib.cc_destroy.restype = None
    lib.cc_last_error.restype = C.c_char_p
    _LIB = lib
    return lib


def _check(rc):
    if rc != CC_OK:
        raise CutCellError(rc, load().cc_last_error().decode())


def default_params() -> CcParams:
    p = CcParams()
    load().cc_default_params(C.byref(p))
    return p


def _field(desc: Optional[dict]):
    """cc_field from an inputs.* field descriptor; returns (struct, keep-alive)."""
    if desc is None:
        desc = inputs.zero_field()
    k = desc["kind"]
    if k == "zero":
        data = np.zeros(1)
        nt = 0
    elif k == "poly":
        data = np.array(desc["terms"], dtype=np.float64).reshape(-1)
        nt = len(desc["terms"])
    elif k == "sinprod":
        data = np.array([desc["amp"], *desc["k"], *desc["p"]], dtype=np.float64)
        nt = 1
    elif k == "expcos":
        data = np.array([desc["amp"], desc["a"], desc["b"], desc["c"], desc["p"]], dtype=np.float64)
        nt = 1
    elif k == "gauss":
        data = np.array([[a, *m, s] for a, m, s in zip(desc["amp"], desc["mu"], desc["sigma"])],
                        dtype=np.float64).reshape(-1)
        nt = len(desc["amp"])
    elif k == "xsinexp":
        data = np.array([desc["amp"]], dtype=np.float64)
        nt = 1
    else:
        raise ValueError(k)
    data = np.ascontiguousarray(data)
    f = CcField(CC_FIELD[k], nt, data.ctypes.data_as(C.POINTER(C.c_double)))
    return f, data


def _ptr(t, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def solve_multi(problems, rs, phis) -> list:
    """Solve several problems concurrently (cc_solve_multi); rs[i], phis[i] are
    the n_i^3 float64 device tensors of problem i."""
    import torch
    torch.cuda.current_stream().synchronize()
    k = len(problems)
    hs = (C.c_void_p * k)(*[p._h.value for p in problems])
    rp = (C.c_void_p * k)(*[_ptr(r, p.n() ** 3).value for p, r in zip(problems, rs)])
    pp = (C.c_void_p * k)(*[_ptr(x, p.n() ** 3).value for p, x in zip(problems, phis)])
    infos = (CcSolveInfo * k)()
    rc = load().cc_solve_multi(k, hs, rp, pp, infos)
    if rc not in (CC_OK, CC_ENOCONV):
        _check(rc)
    return [dict(Problem._info(infos[i], CC_OK), converged=infos[i].rel_residual < problems[i].params.tol)
            for i in range(k)]


def solve_multi_graph(problems, rs, phis) -> list:
    """The plain multigrid iterations of several problems in lockstep from the
    calling thread: per iteration each problem's captured step on its own
    stream (cc_solve_multi_graph)."""
    import torch
    torch.cuda.current_stream().synchronize()
    k = len(problems)
    hs = (C.c_void_p * k)(*[p._h.value for p in problems])
    rp = (C.c_void_p * k)(*[_ptr(r, p.n() ** 3).value for p, r in zip(problems, rs)])
    pp = (C.c_void_p * k)(*[_ptr(x, p.n() ** 3).value for p, x in zip(problems, phis)])
    infos = (CcSolveInfo * k)()
    rc = load().cc_solve_multi_graph(k, hs, rp, pp, infos)
    if rc not in (CC_OK, CC_ENOCONV):
        _check(rc)
    return [dict(Problem._info(infos[i], CC_OK), converged=infos[i].rel_residual < problems[i].params.tol)
            for i in range(k)]


class Problem:
    """A built cut-cell problem (geometry, rows, factorizations, device data)."""

    def __init__(self, domain: inputs.Domain, params: Optional[CcParams] = None, stream=None,
                 device: int = 0, **overrides):
        lib = load()
        prm = params if params is not None else default_params()
        prm.n_min = domain.n_min
        prm.device = device
        for k, v in overrides.items():
            setattr(prm, k, v)
        obs = (CcObstacle * max(1, len(domain.obstacles)))()
        for t, o in enumerate(domain.obstacles):
            obs[t].center[:] = [float(v) for v in o.center]
            obs[t].axes[:] = [float(v) for v in o.axes]
            obs[t].rot[:] = [float(v) for v in np.asarray(o.rot).reshape(-1)]
            obs[t].bc = int(o.bc)
            obs[t].robin[:] = [float(v) for v in getattr(o, "robin", (1.0, 0.0))]
            obs[t].kind = int(getattr(o, "kind", 0))
            obs[t].radii[:] = [float(v) for v in getattr(o, "radii", (0.0, 0.0))]
        dom = CcDomain()
        dom.n = domain.n
        dom.origin[:] = [float(v) for v in domain.origin]
        dom.h = 1.0 / domain.n
        dom.wall_bc[:] = [int(v) for v in domain.wall_bc]
        dom.n_obst = len(domain.obstacles)
        dom.obst = obs
        dom.inside = int(bool(getattr(domain, "inside", False)))
        for w, ab in enumerate(getattr(domain, "wall_robin", ((1.0, 0.0),) * 6)):
            dom.wall_robin[w][0] = float(ab[0])
            dom.wall_robin[w][1] = float(ab[1])
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else None
        _check(lib.cc_build(C.byref(dom), C.byref(prm), st, C.byref(h)))
        self._h = h
        self._stream = stream
        self.params = prm
        self.domain = domain
        self.device = device

    def _order(self):
        """The library works on its own stream unless it was given torch's:
        wait for torch's pending work on the tensors passed in."""
        import torch
        cur = torch.cuda.current_stream()
        if self._stream is None or cur.cuda_stream != self._stream:
            cur.synchronize()

    def close(self):
        if getattr(self, "_h", None):
            load().cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- info
    @property
    def num_levels(self) -> int:
        return load().cc_num_levels(self._h)

    def level_info(self, level: int) -> dict:
        info = CcLevelInfo()
        _check(load().cc_get_level_info(self._h, level, C.byref(info)))
        out = {}
        for f, _ in CcLevelInfo._fields_:
            v = getattr(info, f)
            out[f] = list(v) if isinstance(v, C.Array) else v
        return out

    def n(self, level: int = 0) -> int:
        return self.level_info(level)["n"]

    def export_cells(self, level: int = 0):
        n = self.n(level)
        typ = np.zeros(n ** 3, dtype=np.uint8)
        host = np.zeros(n ** 3, dtype=np.int32)
        vf = np.zeros(n ** 3, dtype=np.float64)
        _check(load().cc_export_cells(self._h, level, typ.ctypes.data_as(C.c_void_p),
                                      host.ctypes.data_as(C.c_void_p), vf.ctypes.data_as(C.c_void_p)))
        return typ, host, vf

    def export_plg(self, level: int = 0):
        N2 = self.level_info(level)["n_phi2"]
        cell = np.zeros(N2, dtype=np.int32)
        cols = np.zeros(N2 * 35, dtype=np.int32)
        vals = np.zeros(N2 * 35, dtype=np.float64)
        _check(load().cc_export_plg(self._h, level, cell.ctypes.data_as(C.c_void_p),
                                    cols.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p)))
        return cell, cols.reshape(N2, 35), vals.reshape(N2, 35)

    def fit_patches(self, field: dict, level: int = 0):
        """The paper's boundary fitting on every cut cell (cc_fit_patches):
        (cell, axis, coef (n, 6), exact (n, 4), fitted (n, 4)); the last two
        hold volume, patch area and the averages of `field` over region and
        patch."""
        n = self.level_info(level)["n_cut"]
        cell = np.zeros(n, dtype=np.int32)
        axis = np.zeros(n, dtype=np.int32)
        coef = np.zeros(n * 6)
        exact = np.zeros(n * 4)
        fitted = np.zeros(n * 4)
        f, keep = _field(field)
        _check(load().cc_fit_patches(self._h, level, C.byref(f), cell.ctypes.data_as(C.c_void_p),
                                     axis.ctypes.data_as(C.c_void_p), coef.ctypes.data_as(C.c_void_p),
                                     exact.ctypes.data_as(C.c_void_p), fitted.ctypes.data_as(C.c_void_p)))
        return cell, axis, coef.reshape(n, 6), exact.reshape(n, 4), fitted.reshape(n, 4)

    def export_lu_nodes(self, level: int = 0):
        k = self.level_info(level)["lu_nodes"]
        arr = {name: np.zeros(k, dtype=np.int32) for name in ("base", "p", "q", "height", "parent")}
        _check(load().cc_export_lu_nodes(self._h, level, *[arr[nm].ctypes.data_as(C.c_void_p)
                                                            for nm in ("base", "p", "q", "height", "parent")]))
        return arr

    def selfcheck_lu(self, level: int) -> float:
        v = C.c_double()
        _check(load().cc_selfcheck_lu(self._h, level, C.byref(v)))
        return v.value

    # -------------------------------------------------------------- device
    def assemble_rhs(self, f: dict, g: Optional[dict], r, f_mode: int = CC_VALUE, level: int = 0):
        self._order()
        fs, fk = _field(f)
        gs, gk = _field(g)
        _check(load().cc_assemble_rhs_level(self._h, level, C.byref(fs), f_mode, C.byref(gs),
                                            _ptr(r, self.n(level) ** 3)))

    def assemble_rhs_batched(self, fs, gs, r, f_mode: int = CC_VALUE, level: int = 0):
        """r (nf, n_m^3) <- the right-hand sides of the fields fs (list of
        descriptors) with boundary data gs (one descriptor for all, or a list of
        nf, or None for zero data), each cut cell's quadrature rule built once."""
        self._order()
        nf = len(fs)
        fa = (CcField * nf)()
        keep = []
        for k, f in enumerate(fs):
            st, data = _field(f)
            fa[k] = st
            keep.append(data)
        per = isinstance(gs, (list, tuple))
        glist = list(gs) if per else [gs]
        if per and len(glist) != nf:
            raise ValueError("one boundary field per right-hand side expected")
        ga = (CcField * len(glist))()
        for k, g in enumerate(glist):
            st, data = _field(g)
            ga[k] = st
            keep.append(data)
        _check(load().cc_assemble_rhs_batched(self._h, level, nf, fa, f_mode, ga, 1 if per else 0,
                                              _ptr(r, nf * self.n(level) ** 3)))

    @staticmethod
    def _info(info: CcSolveInfo, rc: int) -> dict:
        return {"iterations": info.iterations, "rel_residual": info.rel_residual,
                "history": list(info.history[:info.history_len]), "seconds": info.seconds,
                "converged": rc == CC_OK}

    def set_precision(self, precision: int):
        _check(load().cc_set_precision(self._h, precision))
        self.params.precision = precision

    def set_krylov(self, k: int):
        _check(load().cc_set_krylov(self._h, k))
        self.params.krylov = k

    def set_lu_schedule(self, level: int, entries_per_lane: int, subtree: int = 0, waves_cap: int = 0):
        """Override the build-time sweep schedule of one level's factorization."""
        _check(load().cc_set_lu_schedule(self._h, level, entries_per_lane, subtree, waves_cap))

    def set_overlap(self, on: int):
        """Far SMO-1 sweeps beside the LU-correction (1) or whole sweeps (0, default)."""
        _check(load().cc_set_overlap(self._h, on))

    def set_stencil_schedule(self, level: int = -1, march: int = -1, planes: int = 0):
        """Override the regular-row kernel schedule (z-marching or one cell per
        thread, planes per workgroup) of one level (-1: all)."""
        _check(load().cc_set_stencil_schedule(self._h, level, march, planes))

    def stencil_schedule(self, level: int):
        """(march, planes) in force on `level`."""
        m, k = C.c_int(), C.c_int()
        _check(load().cc_get_stencil_schedule(self._h, level, C.byref(m), C.byref(k)))
        return m.value, k.value

    def solve(self, r, phi) -> dict:
        self._order()
        n3 = self.n() ** 3
        info = CcSolveInfo()
        rc = load().cc_solve(self._h, _ptr(r, n3), _ptr(phi, n3), C.byref(info))
        if rc not in (CC_OK, CC_ENOCONV):
            _check(rc)
        return self._info(info, rc)

    def solve_batched(self, r, phi) -> list:
        """r, phi: (nrhs, n^3) contiguous float64 device tensors (batch-major)."""
        self._order()
        n3 = self.n() ** 3
        if r.dim() != 2 or r.shape[1] != n3 or phi.shape != r.shape:
            raise ValueError("expected (nrhs, n^3) tensors of equal shape")
        nrhs = r.shape[0]
        infos = (CcSolveInfo * nrhs)()
        rc = load().cc_solve_batched(self._h, nrhs, _ptr(r), _ptr(phi), infos)
        if rc not in (CC_OK, CC_ENOCONV):
            _check(rc)
        out = []
        for b in range(nrhs):
            d = self._info(infos[b], CC_OK)
            d["converged"] = infos[b].rel_residual < self.params.tol
            out.append(d)
        return out

    def apply(self, level, x, y):
        self._order()
        n3 = self.n(level) ** 3
        _check(load().cc_apply(self._h, level, _ptr(x, n3), _ptr(y, n3)))

    def residual(self, level, r, x, s) -> float:
        self._order()
        n3 = self.n(level) ** 3
        m = C.c_double()
        _check(load().cc_residual(self._h, level, _ptr(r, n3), _ptr(x, n3), _ptr(s, n3), C.byref(m)))
        return m.value

    def smo1(self, level, s, e):
        self._order()
        n3 = self.n(level) ** 3
        _check(load().cc_smo1(self._h, level, _ptr(s, n3), _ptr(e, n3)))

    def smo2(self, level, s, e):
        self._order()
        n3 = self.n(level) ** 3
        _check(load().cc_smo2(self._h, level, _ptr(s, n3), _ptr(e, n3)))

    def restrict(self, level, s, e, sc):
        self._order()
        n3 = self.n(level) ** 3
        _check(load().cc_restrict(self._h, level, _ptr(s, n3), _ptr(e, n3), _ptr(sc, self.n(level + 1) ** 3)))

    def prolong_add(self, level, ec, ef):
        self._order()
        _check(load().cc_prolong_add(self._h, level, _ptr(ec, self.n(level + 1) ** 3), _ptr(ef, self.n(level) ** 3)))

    def fmg(self, r, phi, cycles: int = 2, coarse_rhs=None):
        """Full multigrid approximation of L phi = r into phi (FP64).
        coarse_rhs: the right-hand sides of levels 1..M (assemble_rhs with
        level=m), or None to restrict r."""
        self._order()
        n3 = self.n() ** 3
        arr = None
        if coarse_rhs is not None:
            if len(coarse_rhs) != self.num_levels - 1:
                raise ValueError("one right-hand side per coarser level expected")
            arr = (C.c_void_p * len(coarse_rhs))(*[_ptr(t, self.n(m + 1) ** 3) for m, t in enumerate(coarse_rhs)])
        _check(load().cc_fmg(self._h, _ptr(r, n3), arr, _ptr(phi, n3), cycles))

    def fmg_noalloc(self, r, phi, cycles: int = 2, coarse_rhs=None):
        """fmg() through cc_fmg_noalloc: no device allocation, the coarse arrays in
        the library's fixed per-GPU scratch (calls on one GPU must not overlap)."""
        self._order()
        n3 = self.n() ** 3
        arr = None
        if coarse_rhs is not None:
            if len(coarse_rhs) != self.num_levels - 1:
                raise ValueError("one right-hand side per coarser level expected")
            arr = (C.c_void_p * len(coarse_rhs))(*[_ptr(t, self.n(m + 1) ** 3) for m, t in enumerate(coarse_rhs)])
        _check(load().cc_fmg_noalloc(self._h, _ptr(r, n3), arr, _ptr(phi, n3), cycles))

    def fmg_batched(self, r, phi, cycles: int = 2, coarse_rhs=None):
        """FMG for r of shape (nrhs, n^3) into phi of the same shape; coarse_rhs:
        per coarser level a (nrhs, n_m^3) tensor, or None to restrict r."""
        self._order()
        nrhs = r.shape[0]
        n3 = self.n() ** 3
        arr = None
        if coarse_rhs is not None:
            if len(coarse_rhs) != self.num_levels - 1:
                raise ValueError("one right-hand side array per coarser level expected")
            arr = (C.c_void_p * len(coarse_rhs))(*[_ptr(t, nrhs * self.n(m + 1) ** 3)
                                                  for m, t in enumerate(coarse_rhs)])
        _check(load().cc_fmg_batched(self._h, nrhs, _ptr(r, nrhs * n3), arr, _ptr(phi, nrhs * n3), cycles))

    def fmg_restrict(self, level, s, sc):
        self._order()
        _check(load().cc_fmg_restrict(self._h, level, _ptr(s, self.n(level) ** 3), _ptr(sc, self.n(level + 1) ** 3)))

    def fmg_prolong(self, level, xc, xf):
        self._order()
        _check(load().cc_fmg_prolong(self._h, level, _ptr(xc, self.n(level + 1) ** 3), _ptr(xf, self.n(level) ** 3)))

    def bottom_solve(self, s, e):
        self._order()
        M = self.num_levels - 1
        n3 = self.n(M) ** 3
        _check(load().cc_bottom_solve(self._h, _ptr(s, n3), _ptr(e, n3)))

    def vcycle(self, level, s, e):
        self._order()
        n3 = self.n(level) ** 3
        _check(load().cc_vcycle(self._h, level, _ptr(s, n3), _ptr(e, n3)))

    def net_pairs(self, level: int, r, phi, phi_scale: float):
        """Training pairs (x (nrhs, m^3, 2) float32, t (nrhs, m^3) float32,
        mask (nrhs, m^3) uint8, device tensors) of the solved problems
        r, phi (nrhs, n^3) on level `level` (cc_net_pairs)."""
        import torch
        self._order()
        nrhs = r.shape[0]
        n3 = self.n() ** 3
        m3 = self.n(level) ** 3
        x = torch.empty(nrhs, m3, 2, dtype=torch.float32, device=r.device)
        t = torch.empty(nrhs, m3, dtype=torch.float32, device=r.device)
        mask = torch.empty(nrhs, m3, dtype=torch.uint8, device=r.device)
        _check(load().cc_net_pairs(self._h, level, nrhs, _ptr(r, nrhs * n3), _ptr(phi, nrhs * n3), phi_scale,
                                   C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), C.c_void_p(mask.data_ptr())))
        return x, t, mask

    def learned_guess(self, net: "Net", level: int, phi_scale: float, r, phi):
        """phi <- the network's guess (see cc_learned_guess)."""
        self._order()
        n3 = self.n() ** 3
        _check(load().cc_learned_guess(self._h, net._h, level, phi_scale, _ptr(r, n3), _ptr(phi, n3)))

    def learned_fmg(self, net: "Net", level: int, phi_scale: float, r, phi, cycles: int = 2, coarse_rhs=None):
        """phi <- the full multigrid ascent from the network's prediction on
        `level` (see cc_learned_fmg); coarse_rhs as for fmg()."""
        self._order()
        n3 = self.n() ** 3
        arr = None
        if coarse_rhs is not None:
            if len(coarse_rhs) != self.num_levels - 1:
                raise ValueError("one right-hand side per coarser level expected")
            arr = (C.c_void_p * len(coarse_rhs))(*[_ptr(t, self.n(m + 1) ** 3) for m, t in enumerate(coarse_rhs)])
        _check(load().cc_learned_fmg(self._h, net._h, level, phi_scale, _ptr(r, n3), arr, _ptr(phi, n3), cycles))

    def time_kernel(self, which: int, reps: int = 20):
        """(ms per launch, algorithmic bytes per launch) of a timing hook."""
        v = C.c_double()
        b = C.c_double()
        _check(load().cc_time_kernel(self._h, which, reps, C.byref(v), C.byref(b)))
        return v.value, b.value


def _dptr(t, dtype, numel):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    if t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Net:
    """The learned-guess U-Net of the library (cc_net_*)."""

    def __init__(self, base_channels: int = 16, seed: int = 0, stream=None, depth: int = 3):
        h = C.c_void_p()
        _check(load().cc_net_create(base_channels, depth, seed, C.c_void_p(stream) if stream is not None else None,
                                    C.byref(h)))
        self._h = h
        self.C = base_channels
        self.depth = depth

    def close(self):
        if getattr(self, "_h", None):
            load().cc_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def num_params(self) -> int:
        return int(load().cc_net_num_params(self._h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        _check(load().cc_net_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError("wrong parameter count")
        _check(load().cc_net_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def forward(self, x, y, n: int, nb: int):
        """x: float32 (nb, n^3, 2) device tensor; y: float32 (nb, n^3)."""
        import torch
        torch.cuda.current_stream().synchronize()
        v = nb * n ** 3
        _check(load().cc_net_forward(self._h, n, nb, _dptr(x, torch.float32, 2 * v), _dptr(y, torch.float32, v)))

    def loss_grad(self, x, t, mask, n: int, nb: int, want_grad: bool = False):
        import torch
        torch.cuda.current_stream().synchronize()
        v = nb * n ** 3
        loss = C.c_double()
        g = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        _check(load().cc_net_loss_grad(self._h, n, nb, _dptr(x, torch.float32, 2 * v), _dptr(t, torch.float32, v),
                                       _dptr(mask, torch.uint8, v), C.byref(loss),
                                       g.ctypes.data_as(C.c_void_p) if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(load().cc_net_adam_step(self._h, lr, beta1, beta2, eps))
