"""Thin ctypes binding of libafe (the C ABI declared in include/afe.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device buffers are torch tensors (float64, on the GPU); their
data pointers and the current HIP stream are handed to the C calls.  There is
no fallback: a missing or unloadable library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafe.so")

AFE_OK = 0
STATUS_NAMES = {
    0: "AFE_OK", -1: "AFE_E_ARG", -2: "AFE_E_BAD_MESH", -3: "AFE_E_DEGENERATE_SUBTET",
    -4: "AFE_E_NO_CONVERGENCE", -5: "AFE_E_POSITIVITY", -6: "AFE_E_HBM_BUDGET", -7: "AFE_E_HIP",
    -8: "AFE_E_NONFINITE",
}
AFE_FP64, AFE_MIXED = 0, 1

EXPORTED = [
    "build_afe_cell_data", "afe_query", "afe_cell_dof_ptr", "afe_dof_coords", "afe_connectivity",
    "afe_prim_to_cons", "ader_cfl_dt", "ader_predict", "ader_correct", "ader_step",
    "afe_predictor_state", "afe_cell_diagnostics", "afe_free", "afe_last_error", "afe_subgrid_sizes",
    "afe_subgrid_host", "afe_profile_enable", "afe_profile_read", "afe_estimate_bytes",
    "afe_batch_create", "afe_batch_free", "afe_batch_attach", "afe_batch_detach", "afe_batch_step",
    "afe_batch_set_shape", "afe_batch_get_shape", "afe_batch_tune", "afe_batch_profile_enable",
    "afe_batch_profile_read", "ader_step_noalloc", "afe_l2_points", "afe_l2_error",
    "afe_boundary_nodes", "afe_set_boundary_states", "afe_set_boundary_gradients",
]
BATCH_SLOTS = 64


class AfeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS_NAMES.get(code, str(code))


class _Mesh(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int32), ("xyz", ctypes.c_void_p),
        ("n_faces", ctypes.c_int32), ("face_ptr", ctypes.c_void_p), ("face_vtx", ctypes.c_void_p),
        ("face_vshift", ctypes.c_void_p), ("face_cell", ctypes.c_void_p), ("nbr_shift", ctypes.c_void_p),
        ("n_cells", ctypes.c_int32), ("box", ctypes.c_double),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("m1", ctypes.c_double), ("av", ctypes.c_int32),
        ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("accel_depth", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t), ("predictor_guess", ctypes.c_int32),
        ("history_cells", ctypes.c_int32), ("kappa", ctypes.c_double), ("cv", ctypes.c_double),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("ndof", ctypes.c_int64), ("n_cells", ctypes.c_int32), ("n_subtets", ctypes.c_int64), ("N", ctypes.c_int32),
        ("max_cell_dofs", ctypes.c_int32), ("max_cell_subtets", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
        ("h_min", ctypes.c_double),
    ]


class _Report(ctypes.Structure):
    _fields_ = [
        ("iters_min", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("iters_mean", ctypes.c_double),
        ("n_troubled", ctypes.c_int32), ("status_cell", ctypes.c_int32),
    ]


class _Shape(ctypes.Structure):
    _fields_ = [
        ("sub", ctypes.c_double), ("minv", ctypes.c_double), ("anderson", ctypes.c_double),
        ("rounds", ctypes.c_int32), ("graph", ctypes.c_int32),
    ]


class _BatchReport(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iters_min", ctypes.c_int32), ("iters_max", ctypes.c_int32),
        ("iters_mean", ctypes.c_double), ("n_troubled", ctypes.c_int32), ("status_cell", ctypes.c_int32),
        ("dt", ctypes.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libafe.so (built in place by paper_2605_00619_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2605_00619_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sigs = {
        "build_afe_cell_data": ([ctypes.POINTER(_Mesh), i32, ctypes.POINTER(_Params), vp, ctypes.POINTER(vp)], i32),
        "afe_query": ([vp, ctypes.POINTER(_Info)], i32),
        "afe_cell_dof_ptr": ([vp, vp], i32),
        "afe_dof_coords": ([vp, vp, vp], i32),
        "afe_connectivity": ([vp, vp, vp, vp, vp], i32),
        "afe_prim_to_cons": ([vp, vp, vp, vp], i32),
        "ader_cfl_dt": ([vp, vp, dbl, ctypes.POINTER(dbl), vp], i32),
        "ader_predict": ([vp, vp, dbl, vp], i32),
        "ader_correct": ([vp, vp, dbl, vp], i32),
        "ader_step": ([vp, vp, dbl, ctypes.POINTER(_Report), vp], i32),
        "ader_step_noalloc": ([vp, vp, dbl, ctypes.POINTER(_Report), vp], i32),
        "afe_predictor_state": ([vp, vp, vp], i32),
        "afe_cell_diagnostics": ([vp, vp, vp, vp], i32),
        "afe_free": ([vp], None),
        "afe_l2_points": ([vp, vp, vp, ctypes.POINTER(i32), vp], i32),
        "afe_l2_error": ([vp, vp, i32, vp, ctypes.POINTER(dbl), vp], i32),
        "afe_boundary_nodes": ([vp, ctypes.POINTER(ctypes.c_int64), vp, vp], i32),
        "afe_set_boundary_states": ([vp, vp], i32),
        "afe_set_boundary_gradients": ([vp, vp], i32),
        "afe_subgrid_sizes": ([ctypes.POINTER(_Mesh), i32, vp], i32),
        "afe_subgrid_host": ([ctypes.POINTER(_Mesh), i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "afe_last_error": ([], ctypes.c_char_p),
        "afe_profile_enable": ([vp, i32], i32),
        "afe_profile_read": ([vp, vp, vp, vp, vp], i32),
        "afe_estimate_bytes": ([ctypes.POINTER(_Mesh), i32, ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_size_t)],
                               i32),
        "afe_batch_create": ([ctypes.POINTER(vp)], i32),
        "afe_batch_free": ([vp], None),
        "afe_batch_attach": ([vp, vp, vp, dbl, ctypes.POINTER(i32)], i32),
        "afe_batch_detach": ([vp, vp], i32),
        "afe_batch_step": ([vp, ctypes.POINTER(_BatchReport), i32, vp], i32),
        "afe_batch_set_shape": ([vp, ctypes.POINTER(_Shape)], i32),
        "afe_batch_get_shape": ([vp, ctypes.POINTER(_Shape)], i32),
        "afe_batch_tune": ([vp, vp, ctypes.POINTER(_Shape)], i32),
        "afe_batch_profile_enable": ([vp, i32], i32),
        "afe_batch_profile_read": ([vp, vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(code: int) -> None:
    if code != AFE_OK:
        msg = _lib.afe_last_error().decode(errors="replace")
        raise AfeError(code, msg)


@dataclass
class Params:
    gamma: float = 1.4
    mu: float = 0.0
    m1: float = 0.1
    av: bool = False
    max_iter: int = 300
    tol: float = 1e-12
    accel_depth: int = 63
    precision: int = AFE_FP64
    hbm_budget: int = 0
    predictor_guess: bool = True
    history_cells: int = 0
    kappa: float = 0.0
    cv: float = 2.5

    def c(self) -> _Params:
        return _Params(self.gamma, self.mu, self.m1, int(self.av), self.max_iter, self.tol, self.accel_depth,
                       self.precision, self.hbm_budget, int(self.predictor_guess), self.history_cells, self.kappa,
                       self.cv)


@dataclass
class StepReport:
    iters_min: int
    iters_max: int
    iters_mean: float
    n_troubled: int
    status_cell: int


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _dev(t) -> ctypes.c_void_p:
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _c_mesh(mesh: dict):
    arrs = dict(
            xyz=np.ascontiguousarray(mesh["xyz"], dtype=np.float64),
            face_ptr=np.ascontiguousarray(mesh["face_ptr"], dtype=np.int32),
            face_vtx=np.ascontiguousarray(mesh["face_vtx"], dtype=np.int32),
            face_vshift=np.ascontiguousarray(mesh["face_vshift"], dtype=np.int8),
            face_cell=np.ascontiguousarray(mesh["face_cell"], dtype=np.int32),
            nbr_shift=np.ascontiguousarray(mesh["nbr_shift"], dtype=np.int8),
    )
    cm = _Mesh(len(arrs["xyz"]), arrs["xyz"].ctypes.data, len(arrs["face_cell"]), arrs["face_ptr"].ctypes.data,
               arrs["face_vtx"].ctypes.data, arrs["face_vshift"].ctypes.data, arrs["face_cell"].ctypes.data,
               arrs["nbr_shift"].ctypes.data, int(mesh["n_cells"]), float(mesh["box"]))
    return cm, arrs


def estimate_bytes(mesh: dict, N: int, params: Params | None = None) -> int:
    """Device bytes a CellData of this mesh, degree and parameters would hold
    (host-only closed form over the mesh's cell counts)."""
    lib = load()
    cm, keep = _c_mesh(mesh)
    cp = (params or Params()).c()
    out = ctypes.c_size_t()
    _check(lib.afe_estimate_bytes(ctypes.byref(cm), N, ctypes.byref(cp), ctypes.byref(out)))
    return int(out.value)


def subgrid_host(mesh: dict, N: int) -> dict:
    """The library's host-only sub-grid construction (no GPU needed)."""
    lib = load()
    cm, keep = _c_mesh(mesh)
    sizes = np.zeros(2, dtype=np.int64)
    _check(lib.afe_subgrid_sizes(ctypes.byref(cm), N, sizes.ctypes.data))
    nsub, ndof = int(sizes[0]), int(sizes[1])
    npn = (N + 1) * (N + 2) * (N + 3) // 6
    nf = (N + 1) * (N + 2) // 2
    nc = int(mesh["n_cells"])
    out = dict(subtet_ptr=np.zeros(nc + 1, np.int64), dof_ptr=np.zeros(nc + 1, np.int64),
               conn=np.zeros((nsub, npn), np.int32), nbr_subtet=np.zeros(nsub, np.int32),
               nbr_perm=np.zeros((nsub, nf), np.int32), geo=np.zeros((nsub, 10)), tri=np.zeros((nsub, 4)))
    _check(lib.afe_subgrid_host(ctypes.byref(cm), N, *(out[k].ctypes.data for k in
                                                       ("subtet_ptr", "dof_ptr", "conn", "nbr_subtet", "nbr_perm",
                                                        "geo", "tri"))))
    out["ndof"] = ndof
    return out


class CellData:
    """A built afe_cell_data object for one mesh and degree N."""

    def __init__(self, mesh: dict, N: int, params: Params | None = None, stream=None):
        lib = load()
        self.params = params or Params()
        cm, self._keep = _c_mesh(mesh)
        handle = ctypes.c_void_p()
        cp = self.params.c()
        _check(lib.build_afe_cell_data(ctypes.byref(cm), N, ctypes.byref(cp), _stream(stream), ctypes.byref(handle)))
        self._h = handle
        self.N = N
        info = _Info()
        _check(lib.afe_query(self._h, ctypes.byref(info)))
        self.ndof = int(info.ndof)
        self.n_cells = int(info.n_cells)
        self.n_subtets = int(info.n_subtets)
        self.max_cell_dofs = int(info.max_cell_dofs)
        self.max_cell_subtets = int(info.max_cell_subtets)
        self.device_bytes = int(info.device_bytes)
        self.h_min = float(info.h_min)
        ptr = np.zeros(self.n_cells + 1, dtype=np.int64)
        _check(lib.afe_cell_dof_ptr(self._h, ptr.ctypes.data))
        self.dof_ptr = ptr
        self.np = (N + 1) * (N + 2) * (N + 3) // 6
        self.nf = (N + 1) * (N + 2) // 2

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.afe_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- queries
    def connectivity(self):
        """(subtet_ptr, conn [nsub, np], nbr_subtet [nsub], nbr_perm [nsub, nf]) as numpy."""
        sp = np.zeros(self.n_cells + 1, dtype=np.int64)
        conn = np.zeros((self.n_subtets, self.np), dtype=np.int32)
        nb = np.zeros(self.n_subtets, dtype=np.int32)
        perm = np.zeros((self.n_subtets, self.nf), dtype=np.int32)
        _check(_lib.afe_connectivity(self._h, sp.ctypes.data, conn.ctypes.data, nb.ctypes.data, perm.ctypes.data))
        return sp, conn, nb, perm

    def dof_coords(self, stream=None):
        import torch
        x = torch.empty((3, self.ndof), dtype=torch.float64, device="cuda")
        _check(_lib.afe_dof_coords(self._h, _dev(x), _stream(stream)))
        return x

    def prim_to_cons(self, prim, out=None, stream=None):
        import torch
        out = torch.empty_like(prim) if out is None else out
        _check(_lib.afe_prim_to_cons(self._h, _dev(prim), _dev(out), _stream(stream)))
        return out

    # ------------------------------------------------------------------ steps
    def cfl_dt(self, u, cfl: float, stream=None) -> float:
        dt = ctypes.c_double()
        _check(_lib.ader_cfl_dt(self._h, _dev(u), float(cfl), ctypes.byref(dt), _stream(stream)))
        return float(dt.value)

    def predict(self, u, dt: float, stream=None) -> None:
        _check(_lib.ader_predict(self._h, _dev(u), float(dt), _stream(stream)))

    def correct(self, u, dt: float, stream=None) -> None:
        _check(_lib.ader_correct(self._h, _dev(u), float(dt), _stream(stream)))

    def step(self, u, dt: float, stream=None, report: bool = True) -> StepReport | None:
        rep = _Report()
        _check(_lib.ader_step(self._h, _dev(u), float(dt), ctypes.byref(rep) if report else None, _stream(stream)))
        if not report:
            return None
        return StepReport(rep.iters_min, rep.iters_max, rep.iters_mean, rep.n_troubled, rep.status_cell)

    def step_noalloc(self, u, dt: float, stream=None) -> StepReport:
        """ader_step_noalloc: the same step without any device allocation."""
        rep = _Report()
        _check(_lib.ader_step_noalloc(self._h, _dev(u), float(dt), ctypes.byref(rep), _stream(stream)))
        return StepReport(rep.iters_min, rep.iters_max, rep.iters_mean, rep.n_troubled, rep.status_cell)

    def l2_points(self, stream=None):
        """Error-norm quadrature points [n_subtets * nq, 3] (device), each
        cell's frame; nq = (N + 3)^3 points per sub-tet."""
        import torch
        nq = ctypes.c_int32()
        _check(_lib.afe_l2_points(self._h, None, None, ctypes.byref(nq), _stream(stream)))
        x = self.dof_coords(stream)
        xq = torch.empty((self.n_subtets * nq.value, 3), dtype=torch.float64, device="cuda")
        _check(_lib.afe_l2_points(self._h, _dev(x), _dev(xq), ctypes.byref(nq), _stream(stream)))
        return xq

    def l2_error(self, u, var: int, ref, stream=None) -> float:
        """(sum over cells of int |u_h[var] - u_e|^2)^(1/2) with ref = u_e at
        the points of l2_points (device, [n_subtets * nq])."""
        out = ctypes.c_double()
        _check(_lib.afe_l2_error(self._h, _dev(u), int(var), _dev(ref), ctypes.byref(out), _stream(stream)))
        return float(out.value)

    # ------------------------------------------------- Dirichlet boundaries
    def boundary_nodes(self):
        """(xyz [count, 3], tau [N + 1]) as numpy: the boundary face nodes of a
        bounded mesh (count = 0 for a periodic one) and the predictor's time
        nodes in (0, 1); the Dirichlet data of a step from t with time step
        dt is the solution at (xyz[i], t + tau[a] dt)."""
        count = ctypes.c_int64()
        _check(_lib.afe_boundary_nodes(self._h, ctypes.byref(count), None, None))
        xyz = np.zeros((count.value, 3))
        tau = np.zeros(self.N + 1)
        _check(_lib.afe_boundary_nodes(self._h, ctypes.byref(count), xyz.ctypes.data, tau.ctypes.data))
        return xyz, tau

    def set_boundary_states(self, prim) -> None:
        """Register the Dirichlet data, primitive (rho, u, v, w, p) device
        [count, N + 1, 5] (None unregisters).  The tensor is read by every
        following step: keep it alive and refill it before each step."""
        if prim is not None:
            count = ctypes.c_int64()
            _check(_lib.afe_boundary_nodes(self._h, ctypes.byref(count), None, None))
            if tuple(prim.shape) != (count.value, self.N + 1, 5):
                raise ValueError(f"boundary states must have shape ({count.value}, {self.N + 1}, 5)")
        self._bstate = prim
        _check(_lib.afe_set_boundary_states(self._h, None if prim is None else _dev(prim)))

    def set_boundary_gradients(self, grad) -> None:
        """Register the gradients of the Dirichlet data, d prim_k / d x_d,
        device [count, N + 1, 3, 5] (needed with viscosity or heat
        conduction; None unregisters); kept and refilled like the states."""
        if grad is not None:
            count = ctypes.c_int64()
            _check(_lib.afe_boundary_nodes(self._h, ctypes.byref(count), None, None))
            if tuple(grad.shape) != (count.value, self.N + 1, 3, 5):
                raise ValueError(f"boundary gradients must have shape ({count.value}, {self.N + 1}, 3, 5)")
        self._bgrad = grad
        _check(_lib.afe_set_boundary_gradients(self._h, None if grad is None else _dev(grad)))

    def predictor_state(self, stream=None):
        import torch
        q = torch.empty((self.ndof, 5 * (self.N + 1)), dtype=torch.float64, device="cuda")
        _check(_lib.afe_predictor_state(self._h, _dev(q), _stream(stream)))
        return q

    def profile_enable(self, on: bool = True) -> None:
        _check(_lib.afe_profile_enable(self._h, int(on)))

    def profile_read(self):
        """(milliseconds, launches, algorithmic bytes, bytes as stored) of the
        predictor's M^-1 kernel."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        b = ctypes.c_double()
        bs = ctypes.c_double()
        _check(_lib.afe_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b), ctypes.byref(bs)))
        return float(ms.value), int(n.value), float(b.value), float(bs.value)

    def diagnostics(self, stream=None):
        it = np.zeros(self.n_cells, dtype=np.int32)
        mu = np.zeros(self.n_cells, dtype=np.float64)
        _check(_lib.afe_cell_diagnostics(self._h, it.ctypes.data, mu.ctypes.data, _stream(stream)))
        return it, mu


@dataclass
class LaunchShape:
    """Predictor launch shape: persistent grid multiples (0 = one workgroup
    per work item), iterations between reads of the list lengths, graph replay."""
    sub: float = 1.0
    minv: float = 0.0
    anderson: float = 0.0
    rounds: int = 2
    graph: bool = False

    def c(self) -> _Shape:
        return _Shape(self.sub, self.minv, self.anderson, self.rounds, int(self.graph))

    @staticmethod
    def of(c: _Shape) -> "LaunchShape":
        return LaunchShape(c.sub, c.minv, c.anderson, int(c.rounds), bool(c.graph))


@dataclass
class BatchReport:
    status: str
    iters_min: int
    iters_max: int
    iters_mean: float
    n_troubled: int
    status_cell: int
    dt: float


class Batch:
    """Several simulations stepped together (afe_batch): one ADER step of
    every attached CellData per step(), predictor launches shared by the
    simulations of one degree and precision, each with its own CFL time step."""

    def __init__(self):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.afe_batch_create(ctypes.byref(h)))
        self._h = h
        self._members = {}  # slot -> (CellData, state tensor), kept alive while attached

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.afe_batch_free(self._h)
            self._h = None
            self._members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def attach(self, cd: CellData, u, cfl: float) -> int:
        slot = ctypes.c_int32()
        _check(_lib.afe_batch_attach(self._h, cd._h, _dev(u), float(cfl), ctypes.byref(slot)))
        self._members[int(slot.value)] = (cd, u)
        return int(slot.value)

    def detach(self, cd: CellData) -> None:
        _check(_lib.afe_batch_detach(self._h, cd._h))
        for k in [k for k, (c, _) in self._members.items() if c is cd]:
            del self._members[k]

    def step(self, stream=None, check: bool = True) -> dict:
        """One step of every attached simulation; {slot: BatchReport}.  With
        check, a failed simulation raises AfeError after the reports are filled."""
        reps = (_BatchReport * BATCH_SLOTS)()
        code = _lib.afe_batch_step(self._h, reps, BATCH_SLOTS, _stream(stream))
        out = {k: BatchReport(STATUS_NAMES.get(reps[k].status, str(reps[k].status)), reps[k].iters_min,
                              reps[k].iters_max, reps[k].iters_mean, reps[k].n_troubled, reps[k].status_cell,
                              reps[k].dt) for k in self._members}
        if code != AFE_OK and all(r.status == "AFE_OK" for r in out.values()):
            # no member reported the failure: the step did not complete for any of them
            for r in out.values():
                r.status = STATUS_NAMES.get(code, str(code))
        if check:
            _check(code)
        return out

    @property
    def shape(self) -> LaunchShape:
        c = _Shape()
        _check(_lib.afe_batch_get_shape(self._h, ctypes.byref(c)))
        return LaunchShape.of(c)

    @shape.setter
    def shape(self, sh: LaunchShape) -> None:
        c = sh.c()
        _check(_lib.afe_batch_set_shape(self._h, ctypes.byref(c)))

    def tune(self, stream=None) -> LaunchShape:
        c = _Shape()
        _check(_lib.afe_batch_tune(self._h, _stream(stream), ctypes.byref(c)))
        return LaunchShape.of(c)

    def profile_enable(self, on: bool = True) -> None:
        _check(_lib.afe_batch_profile_enable(self._h, int(on)))

    def profile_read(self):
        """(milliseconds, launches, algorithmic bytes, bytes as stored) of the
        predictor's M^-1 kernel of the first group."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        b = ctypes.c_double()
        bs = ctypes.c_double()
        _check(_lib.afe_batch_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                           ctypes.byref(bs)))
        return float(ms.value), int(n.value), float(b.value), float(bs.value)
