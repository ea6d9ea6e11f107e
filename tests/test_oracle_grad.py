"""Pins of the reference gradient (autograd through the float64 oracle) that
the differentiable solver is compared with.

The paper defines no gradients: the differentiated map is K unrolled
iterations of Algorithm 1 / Algorithm 2 from the initial state, and the pins
here check its reverse-mode derivative against what does not depend on
autograd: float64 central finite differences, the transpose identity
<J v, w> = <v, J^T w> with J v from finite differences, and the closed form
of the S = 0 case (no flow ever moves, so the final labels are a softmax of
-K D / c).
"""
import math

import numpy as np
import pytest
import torch

from oracle import pseudoflow_oracle as O
from paper_1501_07844_amd import synth

torch.set_num_threads(min(8, torch.get_num_threads()))
F64 = torch.float64
H = 1e-6


def _graph(g):
    return O.OracleGraph(g.n_nodes, g.parent, g.child, g.weight)


def _final_ell(p, D, S, iters):
    if p.kind == "potts":
        return O.solve_potts(D, S, p.s_mode, p.c, p.tau, iters, p.ndim, history=False)["ell"]
    return O.solve_dagmf(D, S, p.s_mode, _graph(p.graph), p.c, p.tau, iters, p.ndim,
                         history=False)["ell"]


def _cross_entropy(ell, gt):
    """Mean over voxels of -ln u_{gt(x)}(x)."""
    return -torch.gather(ell, 1, gt.unsqueeze(1)).mean()


def _fd_check(p, iters, n_entries, seed):
    D0 = torch.tensor(p.D, dtype=F64)
    S0 = torch.tensor(np.asarray(p.S), dtype=F64)
    gt = torch.tensor(p.gt, dtype=torch.int64)
    D = D0.clone().requires_grad_(True)
    S = S0.clone().requires_grad_(True)
    _cross_entropy(_final_ell(p, D, S, iters), gt).backward()
    rng = np.random.default_rng(seed)
    checked = 0
    for name, base, g in (("D", D0, D.grad), ("S", S0, S.grad)):
        flat = base.reshape(-1)
        idx = rng.choice(flat.numel(), size=min(n_entries, flat.numel()), replace=False)
        for i in idx:
            plus, minus = flat.clone(), flat.clone()
            plus[i] += H
            minus[i] -= H
            args = {"D": D0, "S": S0}
            args[name] = plus.view_as(base)
            lp = float(_cross_entropy(_final_ell(p, args["D"], args["S"], iters), gt))
            args[name] = minus.view_as(base)
            lm = float(_cross_entropy(_final_ell(p, args["D"], args["S"], iters), gt))
            fd = (lp - lm) / (2 * H)
            ad = float(g.reshape(-1)[i])
            assert abs(fd - ad) <= 1e-6 * (abs(ad) + 1e-3), (name, int(i), fd, ad)
            checked += 1
    return checked


def test_potts_gradient_matches_central_differences():
    """Cross-entropy loss of K = 12 unrolled Potts iterations (shared
    capacity field): 8 entries of D and 8 of S against central differences."""
    p = synth.random_potts(21, (1, 8, 9), 2, 5, s_mode="shared_field", c=2.0, tau=0.125)
    assert _fd_check(p, 12, 8, 0) == 16


def test_dag_gradient_matches_central_differences():
    """Same on a label DAG with per-node constant capacities (Algorithm 2)."""
    g = synth.random_dag(np.random.default_rng(3), 3, 4)
    p = synth.random_problem(22, (2, 4, 5), 3, g, s_mode="node_scalar", c=4.0, tau=0.0625)
    assert _fd_check(p, 8, 8, 1) == 8 + min(8, g.n_nodes - 1)


def test_tree_gradient_matches_central_differences():
    """Same on a hierarchical (tree) model with per-node capacity fields."""
    g = synth.random_tree(np.random.default_rng(4), 2, 4)
    p = synth.random_problem(23, (1, 6, 6), 2, g, s_mode="node_field", c=4.0, tau=0.0625,
                             kind="hmf")
    assert _fd_check(p, 8, 8, 2) == 16


def test_transpose_identity():
    """<J v, w> = <v, J^T w> for the map D -> ell_K; J v by central
    differences along v, J^T w by reverse mode."""
    p = synth.random_potts(24, (2, 4, 5), 3, 3, s_mode="node_field", c=1.0, tau=0.125)
    g = torch.Generator().manual_seed(5)
    D0 = torch.tensor(p.D, dtype=F64)
    S = torch.tensor(np.asarray(p.S), dtype=F64)
    v = torch.randn(D0.shape, generator=g, dtype=F64)
    w = torch.randn(D0.shape, generator=g, dtype=F64)
    Jv = (_final_ell(p, D0 + H * v, S, 9) - _final_ell(p, D0 - H * v, S, 9)) / (2 * H)
    D = D0.clone().requires_grad_(True)
    (_final_ell(p, D, S, 9) * w).sum().backward()
    lhs, rhs = float((Jv * w).sum()), float((v * D.grad).sum())
    assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(lhs))


@pytest.mark.parametrize("iters", [1, 7])
def test_zero_capacity_closed_form(iters):
    """With S = 0 every flow stays 0, so ell_K = log softmax(-K D / c) and
    d(sum w ell_K)/dD = -(K / c) (w - u sum_L w_L)."""
    p = synth.random_potts(25, (1, 5, 6), 2, 4, s_mode="node_scalar", c=3.0, tau=0.125)
    D = torch.tensor(p.D, dtype=F64).requires_grad_(True)
    S = torch.zeros(4, dtype=F64)
    w = torch.randn(D.shape, generator=torch.Generator().manual_seed(6), dtype=F64)
    ell = _final_ell(p, D, S, iters)
    (ell * w).sum().backward()
    t = -iters * D.detach() / p.c
    u = torch.softmax(t, dim=1)
    assert torch.allclose(ell.detach(), torch.log_softmax(t, dim=1), atol=1e-13)
    expect = -(iters / p.c) * (w - u * w.sum(dim=1, keepdim=True))
    assert torch.allclose(D.grad, expect, atol=1e-13)
