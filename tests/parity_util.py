"""Shared helpers of the GPU parity tests: run the reference CPU
implementation and the HIP library on the same seeded float32 inputs and
compare them.

Tolerances (float32 state and arithmetic against the float64 reference):
  * u: max |u_gpu - u_ref| <= 1e-4 (the float32 target of the solver).
  * labels: identical wherever the reference's top-two margin exceeds
    2e-4, twice the u tolerance (closer margins may flip legitimately);
    ties go to the lowest label on both sides.
  * energy and dual: relative 1e-4.  |dE| <= sum |D| |du| + sum S |grad du|
    with |du| <= 1e-4 and D, S, |grad u| of order one per voxel bounds the
    relative change well below that.
"""
from __future__ import annotations

import numpy as np
import torch

import paper_1501_07844_amd as pf
from oracle import pseudoflow_oracle as O

U_TOL = 1e-4
LABEL_MARGIN = 2e-4
E_RTOL = 1e-4


def oracle_graph(p):
    return O.OracleGraph(p.graph.n_nodes, p.graph.parent, p.graph.child, p.graph.weight)


def oracle_solve(p, iters=None, history=False):
    iters = p.iters if iters is None else iters
    if p.kind == "potts":
        r = O.solve_potts(p.D, p.S, p.s_mode, p.c, p.tau, iters, p.ndim, history=history)
    elif p.kind == "ishikawa":
        r = O.solve_ishikawa(p.D, p.S, p.s_mode, p.c, p.tau, iters, p.ndim, history=history)
    else:
        r = O.solve_dagmf(p.D, p.S, p.s_mode, oracle_graph(p), p.c, p.tau, iters, p.ndim,
                          history=history)
    return r


def oracle_energy_dual(p, u, q):
    B, Z, Y, X = p.shape
    D = torch.tensor(p.D, dtype=torch.float64)
    if p.kind == "potts":
        S = O.expand_S(p.S, p.s_mode, B, p.n_leaf, Z, Y, X)
        return float(O.energy_potts(u, D, S, p.ndim).sum()), float(O.dual_potts(q, D, p.ndim).sum())
    if p.kind == "ishikawa":
        S = O.expand_S(p.S, p.s_mode, B, p.n_leaf - 1, Z, Y, X)
        return float(O.energy_ishikawa(u, D, S, p.ndim).sum()), float(O.dual_ishikawa(q, D, p.ndim).sum())
    g = oracle_graph(p)
    S = O.expand_S(p.S, p.s_mode, B, g.n_node, Z, Y, X)
    return float(O.energy_dag(u, D, S, g, p.ndim).sum()), float(O.dual_dag(q, D, g, p.ndim).sum())


def device_inputs(p, device="cuda"):
    D = torch.from_numpy(np.ascontiguousarray(p.D)).to(device)
    if p.s_mode == "node_scalar":
        S = np.asarray(p.S, np.float32)
    else:
        S = torch.from_numpy(np.ascontiguousarray(p.S)).to(device)
    return D, S


def supported_kernels(p):
    """The kernels the library documents for problem p (include/pseudoflow.h):
    the table of expected PF_EUNSUPPORTED cases.  A test asking for a kernel
    outside it is skipped; inside it, every error propagates."""
    ks = ["auto", "two_pass"]
    if p.kind == "potts" and p.n_leaf <= 16:
        ks.append("fused")
    if p.kind in ("hmf", "dagmf") and p.n_leaf <= 16 and p.n_node <= 16:
        ks.append("fused")
    if p.kind == "ishikawa" and p.ndim == 3 and p.n_leaf <= 16:
        ks.append("fused")
    if p.kind == "potts" and p.ndim == 3 and p.n_leaf <= 8:
        ks.append("fused2")
    if p.ndim == 2 and p.n_leaf <= 8 and p.n_node <= 16:
        ks.append("lds")
    return ks


def gpu_solve(p, iters=None, **kw):
    import pytest
    iters = p.iters if iters is None else iters
    kernel = kw.get("kernel", "auto")
    if kernel not in supported_kernels(p):
        pytest.skip(f"no {kernel} kernel for {p.name} (documented as unsupported)")
    D, S = device_inputs(p)
    args = dict(c=p.c, tau=p.tau, iters=iters, ndim=p.ndim, s_mode=p.s_mode)
    args.update(kw)
    if p.kind == "potts":
        return pf.solve_potts(D, S, **args)
    if p.kind == "ishikawa":
        return pf.solve_ishikawa(D, S, **args)
    if p.kind == "hmf":
        return pf.solve_hmf(D, S, p.graph, **args)
    return pf.solve_dagmf(D, S, p.graph, **args)


def top2_margin(u: np.ndarray) -> np.ndarray:
    s = np.sort(u, axis=1)
    if u.shape[1] < 2:
        return np.full(s[:, 0].shape, np.inf)
    return s[:, -1] - s[:, -2]


def compare_labels(u_ref: np.ndarray, labels_gpu: np.ndarray):
    """Returns (mismatches, mismatches where the margin is decisive)."""
    ref = np.argmax(u_ref, axis=1)
    bad = ref != labels_gpu
    decisive = bad & (top2_margin(u_ref) > LABEL_MARGIN)
    return int(bad.sum()), int(decisive.sum())


def check_parity(p, ref, res, u_tol=U_TOL, e_rtol=E_RTOL, check_q=True):
    u_ref = ref["u"].numpy()
    u_gpu = res.u.cpu().numpy()
    du = float(np.abs(u_ref - u_gpu).max()) if u_ref.size else 0.0
    n_bad, n_decisive = compare_labels(u_ref, res.labels.cpu().numpy())
    msg = f"{p.name}: max|du|={du:.3e} label mismatches={n_bad} decisive={n_decisive}"
    print(msg, flush=True)
    assert du <= u_tol, msg
    assert n_decisive == 0, msg
    if res.q is not None and check_q:
        q_ref = ref["q"].numpy()
        dq = float(np.abs(q_ref - res.q.cpu().numpy()).max())
        assert dq <= 10 * u_tol, f"{p.name}: max|dq|={dq:.3e}"
    if np.isfinite(res.energy):
        E, P = oracle_energy_dual(p, ref["u"], ref["q"])
        assert abs(res.energy - E) <= e_rtol * abs(E), (res.energy, E)
        assert abs(res.dual - P) <= e_rtol * abs(E), (res.dual, P)
    return du
