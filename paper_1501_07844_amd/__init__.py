"""MI355X (gfx950) pseudo-flow continuous max-flow solvers.

Thin Python binding over the C ABI of ``_lib/libpseudoflow.so`` (declared in
``include/pseudoflow.h``): it checks tensor shapes and dtypes, allocates the
caller-owned outputs and workspace with PyTorch, and passes raw device
pointers and torch's current HIP stream.  Every step of the solve runs in the
library's HIP kernels; there is no CPU fallback, and a missing library raises.

Entry points mirror the C names: ``solve_potts``, ``solve_hmf``,
``solve_dagmf``, ``solve_ishikawa``, ``workspace_bytes``, ``tape_bytes``.
``potts_layer`` and ``dagmf_layer`` wrap a recorded solve and the C backward
entry points in a ``torch.autograd.Function``: the loss gradient on the final
log-labels flows back to the data terms and the capacities.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Union

import numpy as np

__all__ = [
    "solve_potts", "solve_hmf", "solve_dagmf", "solve_dagmf_static", "solve_ishikawa",
    "solve_potts_fullflow", "fullflow_workspace_bytes",
    "workspace_bytes", "auto_kernel",
    "potts_layer", "dagmf_layer", "tape_bytes", "PottsFn", "DagFn",
    "SolveResult", "PseudoflowError", "library", "lib_path", "EXPORTED",
    "PF_OK", "PF_EINVAL", "PF_EGRAPH", "PF_ENOMEM", "PF_EHIP", "PF_ENONFINITE",
    "PF_EUNSUPPORTED", "MAX_LEAVES", "MAX_NODES",
]

PF_OK, PF_EINVAL, PF_EGRAPH, PF_ENOMEM, PF_EHIP, PF_ENONFINITE, PF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAX_LEAVES, MAX_NODES = 16, 32
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2}
KERNEL = {"auto": 0, "two_pass": 1, "fused": 2, "fused2": 3, "lds": 4}
S_MODE = {"node_scalar": 0, "shared_field": 1, "node_field": 2}

# every symbol include/pseudoflow.h declares
EXPORTED = ["pf_workspace_bytes", "solve_potts", "solve_dagmf", "solve_hmf",
            "solve_ishikawa", "pf_last_error", "pf_abi_version", "pf_tape_bytes",
            "pf_backward_workspace_bytes", "pf_potts_backward", "pf_dagmf_backward",
            "pf_auto_kernel", "solve_dagmf_static", "solve_potts_fullflow",
            "pf_fullflow_workspace_bytes"]
ABI_VERSION = 3

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "_lib", "libpseudoflow.so")


class PseudoflowError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pseudoflow error {code}: {msg}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("batch", C.c_int32), ("ndim", C.c_int32), ("nz", C.c_int32),
                ("ny", C.c_int32), ("nx", C.c_int32)]


class _Graph(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_edges", C.c_int32),
                ("parent", C.POINTER(C.c_int32)), ("child", C.POINTER(C.c_int32)),
                ("weight", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("c", C.c_float), ("tau", C.c_float),
                ("storage", C.c_int32), ("kernel", C.c_int32), ("warm_start", C.c_int32),
                ("gap_every", C.c_int32), ("gap_tol", C.c_double),
                ("final_energy", C.c_int32), ("check_inputs", C.c_int32),
                ("timing_stride", C.c_int32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("ckpt_every", C.c_int32),
                ("tape", C.c_void_p), ("tape_bytes", C.c_size_t)]


class _Result(C.Structure):
    _fields_ = [("u", C.c_void_p), ("labels", C.c_void_p), ("q", C.c_void_p), ("ell", C.c_void_p),
                ("gap_history", C.POINTER(C.c_double)), ("gap_history_cap", C.c_int32),
                ("gap_history_len", C.c_int32), ("iters_done", C.c_int32),
                ("energy", C.c_double), ("dual", C.c_double), ("gap", C.c_double),
                ("max_simplex_err", C.c_double), ("max_flow_excess", C.c_double),
                ("kernel_ms", C.c_double), ("kernel_timed", C.c_int32)]


_LIB = None


def library() -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is missing: build it first (python -m paper_1501_07844_amd.build); "
                "there is no CPU fallback")
        lib = C.CDLL(path)
        lib.pf_workspace_bytes.restype = C.c_size_t
        lib.pf_workspace_bytes.argtypes = [C.POINTER(_Grid), C.c_int32, C.c_int32, C.POINTER(_Params)]
        lib.pf_fullflow_workspace_bytes.restype = C.c_size_t
        lib.pf_fullflow_workspace_bytes.argtypes = [C.POINTER(_Grid), C.c_int32]
        lib.pf_auto_kernel.restype = C.c_int32
        lib.pf_auto_kernel.argtypes = [C.POINTER(_Grid), C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        sig = [C.POINTER(_Grid), C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
               C.POINTER(_Params), C.POINTER(_Result), C.c_void_p]
        gsig = [C.POINTER(_Grid), C.POINTER(_Graph), C.c_void_p, C.c_void_p, C.c_int32,
                C.POINTER(_Params), C.POINTER(_Result), C.c_void_p]
        for name, argt in (("solve_potts", sig), ("solve_ishikawa", sig),
                           ("solve_dagmf", gsig), ("solve_hmf", gsig),
                           ("solve_dagmf_static", gsig), ("solve_potts_fullflow", sig)):
            f = getattr(lib, name)
            f.restype = C.c_int
            f.argtypes = argt
        lib.pf_last_error.restype = C.c_char_p
        lib.pf_abi_version.restype = C.c_int32
        lib.pf_tape_bytes.restype = C.c_size_t
        lib.pf_tape_bytes.argtypes = [C.POINTER(_Grid), C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        lib.pf_backward_workspace_bytes.restype = C.c_size_t
        lib.pf_backward_workspace_bytes.argtypes = [C.POINTER(_Grid), C.c_int32, C.c_int32, C.c_int32]
        bsig = [C.POINTER(_Grid), C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(_Params),
                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        bgsig = [C.POINTER(_Grid), C.POINTER(_Graph), C.c_void_p, C.c_void_p, C.c_int32,
                 C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.pf_potts_backward.restype = C.c_int
        lib.pf_potts_backward.argtypes = bsig
        lib.pf_dagmf_backward.restype = C.c_int
        lib.pf_dagmf_backward.argtypes = bgsig
        if lib.pf_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{path}: ABI {lib.pf_abi_version()} != {ABI_VERSION}; rebuild it")
        _LIB = lib
    return _LIB


@dataclass
class SolveResult:
    u: Optional[object]            # torch float32 [B][n_leaf][Z][Y][X]
    ell: Optional[object]          # torch float32 [B][n_leaf][Z][Y][X], ln u
    labels: Optional[object]       # torch int32 [B][Z][Y][X]
    q: Optional[object]            # torch float32 [B][n_node][ndim][Z][Y][X]
    iters_done: int
    energy: float
    dual: float
    gap: float
    max_simplex_err: float
    max_flow_excess: float
    kernel_ms: float
    kernel_timed: int
    gap_history: List[float] = field(default_factory=list)
    workspace: Optional[object] = None


def _torch():
    import torch
    return torch


def _grid_of(D, ndim: Optional[int]) -> _Grid:
    if D.dim() != 5:
        raise ValueError("D must be [B][L][Z][Y][X]")
    B, _, Z, Y, X = D.shape
    nd = ndim if ndim is not None else (3 if Z > 1 else 2)
    return _Grid(B, nd, Z, Y, X)


def _check_dev(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")


def workspace_bytes(shape, n_leaf: int, n_node: int, ndim: int, storage: str = "fp32",
                    kernel: str = "auto") -> int:
    """Bytes of workspace for a [B, Z, Y, X] problem."""
    B, Z, Y, X = shape
    g = _Grid(B, ndim, Z, Y, X)
    p = _Params()
    p.storage = STORAGE[storage]
    p.kernel = KERNEL[kernel]
    return int(library().pf_workspace_bytes(C.byref(g), n_leaf, n_node, C.byref(p)))


def auto_kernel(shape, n_leaf: int, n_node: int, ndim: int, storage: str = "fp32",
                identity: bool = True) -> str:
    """The kernel ``kernel="auto"`` runs for an unrecorded solve of a
    [B, Z, Y, X] problem ("two_pass", "fused", "fused2" or "lds")."""
    B, Z, Y, X = shape
    k = int(library().pf_auto_kernel(C.byref(_Grid(B, ndim, Z, Y, X)), n_leaf, n_node,
                                     int(bool(identity)), STORAGE[storage]))
    if k < 0:
        raise ValueError("no solver accepts this problem")
    return {v: n for n, v in KERNEL.items()}[k]


def _s_args(S, s_mode, B, nn, Z, Y, X, keep):
    """Returns (pointer, mode) for S given as a scalar / host sequence
    (one value per flow) or a device field."""
    torch = _torch()
    if isinstance(S, torch.Tensor) and S.is_cuda:
        if s_mode is None:
            s_mode = "shared_field" if S.dim() == 4 else "node_field"
        want = (B, Z, Y, X) if s_mode == "shared_field" else (B, nn, Z, Y, X)
        if s_mode not in ("shared_field", "node_field") or tuple(S.shape) != want:
            raise ValueError(f"S field must be {want} for {s_mode}")
        _check_dev(S, "S", torch.float32)
        return S.data_ptr(), S_MODE[s_mode]
    arr = np.broadcast_to(np.asarray(S, np.float32), (nn,)).copy()
    keep.append(arr)
    return arr.ctypes.data, S_MODE["node_scalar"]


def _graph_struct(graph, keep) -> _Graph:
    par = np.ascontiguousarray(np.asarray(graph.parent, np.int32))
    chi = np.ascontiguousarray(np.asarray(graph.child, np.int32))
    keep += [par, chi]
    g = _Graph(int(graph.n_nodes), int(par.shape[0]),
               par.ctypes.data_as(C.POINTER(C.c_int32)), chi.ctypes.data_as(C.POINTER(C.c_int32)),
               None)
    if getattr(graph, "weight", None) is not None:
        w = np.ascontiguousarray(np.asarray(graph.weight, np.float64))
        keep.append(w)
        g.weight = w.ctypes.data_as(C.POINTER(C.c_double))
    return g


def _solve(entry, D, S, n_leaf, n_node, *, graph=None, n_labels=None, c, tau, iters,
           s_mode=None, ndim=None, storage="fp32", kernel="auto", gap_every=0, gap_tol=0.0,
           final_energy=True, check_inputs=False, timing_stride=0, return_u=True,
           return_labels=True, return_q=False, return_ell=False, workspace=None,
           warm_start=False, gap_history_cap=0, tape=None, ckpt_every=0,
           static_scratch=False, fullflow=False) -> SolveResult:
    torch = _torch()
    lib = library()
    _check_dev(D, "D", torch.float32)
    grid = _grid_of(D, ndim)
    B, Z, Y, X = grid.batch, grid.nz, grid.ny, grid.nx
    keep: list = []
    s_ptr, s_code = _s_args(S, s_mode, B, n_node, Z, Y, X, keep)
    p = _Params()
    p.iters, p.c, p.tau = int(iters), float(c), float(tau)
    p.storage, p.kernel = STORAGE[storage], KERNEL[kernel]
    p.warm_start, p.gap_every, p.gap_tol = int(bool(warm_start)), int(gap_every), float(gap_tol)
    p.final_energy, p.check_inputs = int(bool(final_energy)), int(bool(check_inputs))
    p.timing_stride = int(timing_stride)
    if tape is not None:
        p.ckpt_every, p.tape, p.tape_bytes = int(ckpt_every), tape.data_ptr(), tape.numel()
    if static_scratch:
        # the library's static device scratch: no workspace at all
        if workspace is not None:
            raise ValueError("the static-scratch solve takes no workspace")
        p.workspace, p.workspace_bytes = None, 0
    else:
        need = (lib.pf_fullflow_workspace_bytes(C.byref(grid), n_leaf) if fullflow
                else lib.pf_workspace_bytes(C.byref(grid), n_leaf, n_node, C.byref(p)))
        if need == 0:
            # let the solver report the precise reason
            need = 256
        if workspace is None or workspace.numel() < need:
            if warm_start:
                raise ValueError("warm_start needs the workspace of an earlier call")
            workspace = torch.empty(need, dtype=torch.uint8, device=D.device)
        p.workspace, p.workspace_bytes = workspace.data_ptr(), workspace.numel()
    r = _Result()
    u = labels = q = ell = None
    if return_ell:
        ell = torch.empty((B, n_leaf, Z, Y, X), dtype=torch.float32, device=D.device)
        r.ell = ell.data_ptr()
    if return_u:
        u = torch.empty((B, n_leaf, Z, Y, X), dtype=torch.float32, device=D.device)
        r.u = u.data_ptr()
    if return_labels:
        labels = torch.empty((B, Z, Y, X), dtype=torch.int32, device=D.device)
        r.labels = labels.data_ptr()
    if return_q:
        q = torch.empty((B, n_node, grid.ndim, Z, Y, X), dtype=torch.float32, device=D.device)
        r.q = q.data_ptr()
    hist = None
    if gap_history_cap > 0:
        hist = (C.c_double * gap_history_cap)()
        r.gap_history = C.cast(hist, C.POINTER(C.c_double))
        r.gap_history_cap = gap_history_cap
    stream = torch.cuda.current_stream(D.device).cuda_stream
    if graph is not None:
        gs = _graph_struct(graph, keep)
        st = entry(C.byref(grid), C.byref(gs), C.c_void_p(D.data_ptr()), C.c_void_p(s_ptr),
                   s_code, C.byref(p), C.byref(r), C.c_void_p(stream))
    else:
        st = entry(C.byref(grid), int(n_labels), C.c_void_p(D.data_ptr()), C.c_void_p(s_ptr),
                   s_code, C.byref(p), C.byref(r), C.c_void_p(stream))
    if st != PF_OK:
        raise PseudoflowError(st, lib.pf_last_error().decode())
    return SolveResult(u, ell, labels, q, r.iters_done, r.energy, r.dual, r.gap,
                       r.max_simplex_err, r.max_flow_excess, r.kernel_ms, r.kernel_timed,
                       [hist[i] for i in range(r.gap_history_len)] if hist is not None else [],
                       workspace)


def solve_potts(D, S, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """Pseudo-flow Potts model.  D: device float32 [B][n][Z][Y][X].
    S: scalar or host sequence of n per-label constants, or a device field
    [B][Z][Y][X] (shared) or [B][n][Z][Y][X] (per label).  ``kernel``:
    "auto" (see ``auto_kernel``), "two_pass", "fused" (one pass per
    iteration), "fused2" (one pass per two iterations; 3-D, n <= 8) or
    "lds" (2-D, n <= 8: iterations in LDS, whole problems per block for
    batches of 8 or more that fit, tiles with ghost zones otherwise); all
    give the same result bit for bit.  ``final_energy=True`` (the default)
    reads the energy back and synchronises the stream; with it off and no
    gap checks the call is asynchronous."""
    n = int(D.shape[1])
    return _solve(library().solve_potts, D, S, n, n, n_labels=n, c=c, tau=tau, iters=iters, **kw)


def _graph_sizes(graph):
    has_child = set(int(p) for p in np.asarray(graph.parent))
    nl = sum(1 for a in range(1, int(graph.n_nodes)) if a not in has_child)
    return nl, int(graph.n_nodes) - 1


def solve_dagmf(D, S, graph, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """Pseudo-flow DAGMF model on a label DAG (``graph`` has n_nodes, parent,
    child and optional weight; node 0 is the source).  D holds one field per
    leaf in ascending node id; S one value (or field) per non-source node."""
    nl, nn = _graph_sizes(graph)
    return _solve(library().solve_dagmf, D, S, nl, nn, graph=graph, c=c, tau=tau, iters=iters, **kw)


def solve_dagmf_static(D, S, graph, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """``solve_dagmf`` on the library's static device scratch (the C entry
    point ``solve_dagmf_static``): no workspace is allocated or passed; the
    outputs (u, labels, q, ell) are still allocated here.  For callers that
    cannot allocate device memory; calls overlapping on one GPU race."""
    nl, nn = _graph_sizes(graph)
    return _solve(library().solve_dagmf_static, D, S, nl, nn, graph=graph, c=c, tau=tau,
                  iters=iters, static_scratch=True, **kw)


def fullflow_workspace_bytes(shape, n_labels: int, ndim: int) -> int:
    """Bytes of workspace of the full-flow Potts solver for a [B, Z, Y, X] problem."""
    B, Z, Y, X = shape
    return int(library().pf_fullflow_workspace_bytes(C.byref(_Grid(B, ndim, Z, Y, X)), n_labels))


def solve_potts_fullflow(D, S, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """Full-flow counterpart of ``solve_potts`` (explicit source, sink and
    spatial flows, the labels as multipliers; ``c`` the penalty of the
    augmented Lagrangian, ``tau`` the spatial-flow step).  float32 state;
    ``u`` holds the multipliers as they are."""
    n = int(D.shape[1])
    return _solve(library().solve_potts_fullflow, D, S, n, n, n_labels=n, c=c, tau=tau,
                  iters=iters, fullflow=True, **kw)


def solve_hmf(D, S, graph, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """Hierarchical max-flow: ``solve_dagmf`` restricted to trees."""
    nl, nn = _graph_sizes(graph)
    return _solve(library().solve_hmf, D, S, nl, nn, graph=graph, c=c, tau=tau, iters=iters, **kw)


def solve_ishikawa(D, S, *, c: float, tau: float, iters: int, **kw) -> SolveResult:
    """Pseudo-flow Ishikawa chain: D [B][N+1][Z][Y][X], S for the N flows."""
    n = int(D.shape[1])
    return _solve(library().solve_ishikawa, D, S, n, n - 1, n_labels=n, c=c, tau=tau,
                  iters=iters, **kw)


# ------------------------------------------------------- differentiable ---

def tape_bytes(shape, n_leaf: int, n_node: int, ndim: int, iters: int, ckpt_every: int) -> int:
    B, Z, Y, X = shape
    return int(library().pf_tape_bytes(C.byref(_Grid(B, ndim, Z, Y, X)), n_leaf, n_node,
                                       iters, ckpt_every))


class _Spec:
    """Static arguments of a differentiable solve."""

    def __init__(self, kind, graph, c, tau, iters, ckpt_every, s_mode, ndim, backward_kernel):
        self.kind, self.graph, self.c, self.tau = kind, graph, c, tau
        self.iters, self.ckpt_every, self.s_mode, self.ndim = iters, ckpt_every, s_mode, ndim
        self.backward_kernel = KERNEL[backward_kernel]


def _host_or_dev_S(S, s_mode):
    if s_mode == "node_scalar":
        return S.detach().float().cpu().numpy()
    return S.detach().float().contiguous()


class _PseudoflowFn:
    """Holder of the torch.autograd.Function (built lazily: torch import)."""
    cls = None


def _autograd_fn():
    if _PseudoflowFn.cls is not None:
        return _PseudoflowFn.cls
    torch = _torch()

    class PseudoflowSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, D, S, spec):
            lib = library()
            D = D.detach().float().contiguous()
            grid = _grid_of(D, spec.ndim)
            B, Z, Y, X = grid.batch, grid.nz, grid.ny, grid.nx
            if spec.kind == "potts":
                nl = nn = int(D.shape[1])
            else:
                nl, nn = _graph_sizes(spec.graph)
            tb = lib.pf_tape_bytes(C.byref(grid), nl, nn, spec.iters, spec.ckpt_every)
            tape = torch.empty(max(tb, 256), dtype=torch.uint8, device=D.device)
            Sx = _host_or_dev_S(S, spec.s_mode)
            kw = dict(c=spec.c, tau=spec.tau, iters=spec.iters, s_mode=spec.s_mode,
                      ndim=spec.ndim, kernel="two_pass", final_energy=False, return_u=False,
                      return_labels=False, return_ell=True, tape=tape,
                      ckpt_every=spec.ckpt_every)
            if spec.kind == "potts":
                res = _solve(lib.solve_potts, D, Sx, nl, nn, n_labels=nl, **kw)
            else:
                res = _solve(lib.solve_dagmf, D, Sx, nl, nn, graph=spec.graph, **kw)
            ctx.save_for_backward(D, S)
            ctx.spec, ctx.tape, ctx.sizes = spec, tape, (nl, nn)
            return res.ell

        @staticmethod
        def backward(ctx, grad_ell):
            lib = library()
            D, S = ctx.saved_tensors
            spec, (nl, nn) = ctx.spec, ctx.sizes
            grid = _grid_of(D, spec.ndim)
            gl = grad_ell.detach().float().contiguous()
            gD = torch.empty_like(D)
            gS = torch.empty(S.shape, dtype=torch.float32, device=D.device)
            ws_bytes = lib.pf_backward_workspace_bytes(C.byref(grid), nl, nn, spec.ckpt_every)
            ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=D.device)
            p = _Params()
            p.iters, p.c, p.tau = spec.iters, float(spec.c), float(spec.tau)
            p.storage, p.kernel = STORAGE["fp32"], spec.backward_kernel
            p.workspace, p.workspace_bytes = ws.data_ptr(), ws.numel()
            p.ckpt_every, p.tape, p.tape_bytes = spec.ckpt_every, ctx.tape.data_ptr(), ctx.tape.numel()
            keep: list = []
            Sx = _host_or_dev_S(S, spec.s_mode)
            s_ptr, s_code = _s_args(Sx, spec.s_mode, grid.batch, nn, grid.nz, grid.ny, grid.nx, keep)
            stream = C.c_void_p(torch.cuda.current_stream(D.device).cuda_stream)
            if spec.kind == "potts":
                st = lib.pf_potts_backward(C.byref(grid), nl, C.c_void_p(D.data_ptr()),
                                              C.c_void_p(s_ptr), s_code, C.byref(p),
                                              C.c_void_p(gl.data_ptr()), C.c_void_p(gD.data_ptr()),
                                              C.c_void_p(gS.data_ptr()), stream)
            else:
                gs = _graph_struct(spec.graph, keep)
                st = lib.pf_dagmf_backward(C.byref(grid), C.byref(gs), C.c_void_p(D.data_ptr()),
                                              C.c_void_p(s_ptr), s_code, C.byref(p),
                                              C.c_void_p(gl.data_ptr()), C.c_void_p(gD.data_ptr()),
                                              C.c_void_p(gS.data_ptr()), stream)
            if st != PF_OK:
                raise PseudoflowError(st, lib.pf_last_error().decode())
            return gD, gS.to(S.dtype), None

    _PseudoflowFn.cls = PseudoflowSolve
    return PseudoflowSolve


def potts_layer(D, S, *, c: float, tau: float, iters: int, ckpt_every: int = 10,
                s_mode: Optional[str] = None, ndim: Optional[int] = None,
                backward_kernel: str = "auto"):
    """Differentiable pseudo-flow Potts solve: returns the final log-labels
    ell_K = ln u_K (float32, [B][n][Z][Y][X]); gradients flow to D and S.
    S: device tensor [n] (per-label constants), [B][Z][Y][X] (shared field) or
    [B][n][Z][Y][X] (per-label field).  The forward records a checkpoint
    every ``ckpt_every`` iterations; ``backward_kernel`` picks the reverse
    step ("fused", "two_pass" or "auto")."""
    if s_mode is None:
        s_mode = {1: "node_scalar", 4: "shared_field", 5: "node_field"}[S.dim()]
    nd = ndim if ndim is not None else (3 if D.shape[2] > 1 else 2)
    spec = _Spec("potts", None, c, tau, iters, max(1, min(ckpt_every, iters)), s_mode, nd,
                 backward_kernel)
    return _autograd_fn().apply(D, S, spec)


def dagmf_layer(D, S, graph, *, c: float, tau: float, iters: int, ckpt_every: int = 10,
                s_mode: Optional[str] = None, ndim: Optional[int] = None,
                backward_kernel: str = "auto"):
    """Differentiable pseudo-flow DAGMF (or HMF) solve on ``graph``; as
    ``potts_layer`` with one S value or field per non-source node."""
    if s_mode is None:
        s_mode = {1: "node_scalar", 4: "shared_field", 5: "node_field"}[S.dim()]
    nd = ndim if ndim is not None else (3 if D.shape[2] > 1 else 2)
    spec = _Spec("dagmf", graph, c, tau, iters, max(1, min(ckpt_every, iters)), s_mode, nd,
                 backward_kernel)
    return _autograd_fn().apply(D, S, spec)


class PottsFn:
    """Function-style spelling of ``potts_layer``: ``PottsFn.apply(D, S, params)``
    with ``params`` a dict of its keyword arguments (c, tau, iters, ...)."""

    @staticmethod
    def apply(D, S, params):
        return potts_layer(D, S, **params)


class DagFn:
    """Function-style spelling of ``dagmf_layer``:
    ``DagFn.apply(D, S, graph, params)``."""

    @staticmethod
    def apply(D, S, graph, params):
        return dagmf_layer(D, S, graph, **params)
