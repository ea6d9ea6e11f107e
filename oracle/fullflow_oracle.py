"""Reference CPU implementation ("oracle") of the full-flow continuous
max-flow method for the Potts model: the counterpart the pseudo-flow method is
measured against (Baxter, Rajchl, Yuan, Peters: "A Proximal Bregman
Projection Approach to Continuous Max-Flow Problems Using Entropic
Distances", section "Pseudo-Flow Approach to the Potts Model": the primal
max-flow model and the primal-dual model).

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
tests, the package smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU library and the GPU library never imports
it; it uses the grid operators of the pseudo-flow oracle (same package).

Plain PyTorch on the CPU in float64.

The full-flow method keeps every variable of the primal-dual model explicit:
the source flow p_S(x), one sink flow p_L(x) per label (p_L <= D_L), one
spatial flow q_L(x) per label (|q_L| <= S_L) and the labels u_L(x), which are
the multipliers of the flow-conservation constraints
div q_L - p_S + p_L = 0.  The paper names the method but prints no algorithm
for it.  Reading taken here: the augmented Lagrangian of the primal-dual model
with penalty c,

    L_c = int p_S + sum_L u_L R_L - (c/2) sum_L R_L^2,   R_L = div q_L - p_S + p_L,

maximised over the flows one block at a time (Gauss-Seidel), then one
multiplier step on the labels:

  1. spatial flows, one projected gradient ascent step of size tau:
         q_L <- Proj_{|q_L| <= S_L}(q_L + tau grad(div q_L - p_S + p_L - u_L / c))
     (dL_c / d q_L = grad(c R_L - u_L), since div = -grad^T);
  2. sink flows, exact maximiser under p_L <= D_L:
         p_L <- min(D_L, p_S - div q_L + u_L / c);
  3. source flow, exact (unconstrained) maximiser:
         p_S <- (1/n) sum_L (div q_L + p_L - u_L / c) + 1 / (n c);
  4. labels:  u_L <- u_L - c (div q_L - p_S + p_L).

Step 3 makes sum_L u_L = 1 hold exactly after every iteration; u_L >= 0 is
not enforced (the labelling constraints are implicit in the primal-dual
model and hold only at convergence).  Initial state: q = 0,
p_S = p_L = min_L D_L (a feasible source and sink flow), u_L = 1/n.

Energy and dual of an iterate, for comparison with the pseudo-flow method:
E of the labelling u clipped at 0 and renormalised per voxel (a point of the
simplex, so E is an upper bound of the relaxed optimum), and the pseudo-flow
dual P(q) = int min_L (D_L + div q_L) of the spatial flows (a lower bound for
any |q_L| <= S_L).  The grid operators, the norm and the projection are those
of the pseudo-flow oracle.
"""
from __future__ import annotations

from typing import Dict

import torch

from oracle.pseudoflow_oracle import (F64, _t, _zero_last, div, dual_potts, energy_potts,
                                      expand_S, grad, project)

__all__ = ["init_state", "fullflow_iteration", "feasible_labels", "solve_potts_fullflow"]


def init_state(D: torch.Tensor, ndim: int) -> Dict[str, torch.Tensor]:
    """q = 0, p_S = p_L = min_L D_L, u = 1/n.  D [B][n][Z][Y][X] float64."""
    B, n, Z, Y, X = D.shape
    pS = D.min(dim=1, keepdim=True).values
    return {"q": torch.zeros(B, n, ndim, Z, Y, X, dtype=F64), "pS": pS.clone(),
            "pL": pS.expand_as(D).clone(), "u": torch.full_like(D, 1.0 / n)}


def fullflow_iteration(st: Dict[str, torch.Tensor], D, S, c: float, tau: float,
                       ndim: int) -> Dict[str, torch.Tensor]:
    """One iteration (steps 1-4 of the module docstring).  st holds q
    [B][n][nd][...], pS [B][1][...], pL and u [B][n][...]; S broadcastable to
    [B][n][Z][Y][X]."""
    q, pS, pL, u = st["q"], st["pS"], st["pL"], st["u"]
    n = D.shape[1]
    # 1. spatial flows: gradient ascent on the augmented Lagrangian, projected
    r = div(q, ndim) - pS + pL - u / c
    q = project(_zero_last(q + tau * grad(r, ndim), ndim), S)
    dq = div(q, ndim)
    # 2. sink flows, capped by the data terms
    pL = torch.minimum(D, pS - dq + u / c)
    # 3. source flow
    pS = (dq + pL - u / c).sum(dim=1, keepdim=True) / n + 1.0 / (n * c)
    # 4. multipliers of the flow conservation constraints
    u = u - c * (dq - pS + pL)
    return {"q": q, "pS": pS, "pL": pL, "u": u}


def feasible_labels(u: torch.Tensor) -> torch.Tensor:
    """u clipped at 0 and renormalised over the labels (the uniform labelling
    where every label clips to 0)."""
    v = u.clamp(min=0.0)
    s = v.sum(dim=1, keepdim=True)
    n = u.shape[1]
    return torch.where(s > 0, v / torch.where(s > 0, s, torch.ones_like(s)),
                       torch.full_like(v, 1.0 / n))


def solve_potts_fullflow(D, S, s_mode: str, c: float, tau: float, iters: int, ndim: int,
                         history: bool = True, state=None) -> Dict[str, object]:
    """Run the full-flow method for ``iters`` iterations from the initial
    state (or from ``state``).  Returns the final state, the argmax labels,
    and per iteration the energy E of the feasible labelling, the dual P(q)
    and the maximal flow-conservation residual."""
    D = _t(D)
    B, n, Z, Y, X = D.shape
    Sx = expand_S(S, s_mode, B, n, Z, Y, X)
    st = init_state(D, ndim) if state is None else {k: _t(v) for k, v in state.items()}
    E, P, R = [], [], []
    for _ in range(iters):
        st = fullflow_iteration(st, D, Sx, c, tau, ndim)
        if history:
            E.append(float(energy_potts(feasible_labels(st["u"]), D, Sx, ndim).sum()))
            P.append(float(dual_potts(st["q"], D, ndim).sum()))
            res = div(st["q"], ndim) - st["pS"] + st["pL"]
            R.append(float(res.abs().max()))
    out = dict(st)
    out.update({"E": E, "P": P, "residual": R, "labels": torch.argmax(st["u"], dim=1)})
    return out
