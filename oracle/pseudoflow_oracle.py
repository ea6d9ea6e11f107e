"""Reference CPU implementation ("oracle") of entropic pseudo-flow continuous
max-flow (Baxter, Rajchl, Yuan, Peters: "A Proximal Bregman Projection
Approach to Continuous Max-Flow Problems Using Entropic Distances").

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
tests, the package smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU library (no kernels, headers, helpers,
tables or pre/post-processing) and the GPU library never imports it.

Everything is plain PyTorch on the CPU in float64, slow and direct.  Inputs
given as float32 arrays are widened to float64, so input rounding never counts
as a parity error.  Autograd through these functions provides the reference
gradient for the differentiable solver.

Readings of the paper taken here (where the text is silent, ambiguous or
garbled):
  * Grid operators: unit spacing, forward differences with a zero gradient
    on the last index of each axis (Neumann), div = -grad^T (so the
    divergence uses backward differences), Euclidean norm over the spatial
    components of a flow at a point.  Component k of a flow is the axis
    x, y, z for k = 0, 1, 2; arrays are [..., Z, Y, X] with x fastest.
  * Proj_{|q| <= S}(p) = p * min(1, S/|p|): p itself when |p| <= S, 0 when
    S = 0.  Component k of every flow is kept at 0 on the last index of
    axis k (the divergence never reads it there).
  * Label step, flow step order (Algorithm 1 / Algorithm 2): the flow step
    uses the gradient of the NORMALISED label field (for DAGs: the normalised
    leaf labels aggregated bottom-up).  This is the gradient of the proximal
    objective with the closed-form labelling substituted (Section on the
    Potts model, flow update derivation); the equation printed beside it
    differentiates the un-normalised product instead.  ``literal=True``
    selects the printed form for documentation; it is not what the GPU
    library computes.
  * Labels are carried as ell = ln u and the proximal update
    u <- v exp(-d/c) / sum(v exp(-d/c)) is evaluated as a max-subtracted
    log-sum-exp; this is the same map in exact arithmetic.
  * Initial state: u = 1/(number of end-labels), q = 0.
  * Internal (non-end) labels carry no data term.  Source children receive
    nothing from the source (its flow excess is 0).
  * Energy, dual and gap after an iteration: E(u^k) with u after the label
    step, P(q^k) with q after the flow step; both are feasible so P <= E.
"""
from __future__ import annotations

import heapq
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

F64 = torch.float64

__all__ = [
    "OracleGraph", "grad", "div", "project", "expand_S",
    "potts_iteration", "solve_potts", "energy_potts", "dual_potts",
    "dag_iteration", "solve_dagmf", "energy_dag", "dual_dag", "dag_upward",
    "brute_force_min_energy", "ishikawa_iteration", "solve_ishikawa",
    "energy_ishikawa", "dual_ishikawa",
]


def _t(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(F64)
    return torch.from_numpy(np.ascontiguousarray(a)).to(F64)


# ------------------------------------------------------ grid operators ---

def grad(f: torch.Tensor, ndim: int) -> torch.Tensor:
    """Forward-difference gradient with a zero last row per axis.

    f [..., Z, Y, X] -> [..., ndim, Z, Y, X]; component k is axis -1-k.
    """
    comps = []
    for k in range(ndim):
        ax = f.dim() - 1 - k
        n = f.shape[ax]
        zero = torch.zeros_like(f.narrow(ax, 0, 1))
        if n > 1:
            g = torch.cat([f.narrow(ax, 1, n - 1) - f.narrow(ax, 0, n - 1), zero], dim=ax)
        else:
            g = zero
        comps.append(g)
    return torch.stack(comps, dim=-4)


def div(q: torch.Tensor, ndim: int) -> torch.Tensor:
    """Divergence, the negative adjoint of ``grad``.

    q [..., ndim, Z, Y, X] -> [..., Z, Y, X]:
    div q(x) = sum_k q_k(x) [x_k < N_k - 1] - q_k(x - e_k) [x_k > 0].
    """
    out = None
    for k in range(ndim):
        qk = q.select(-4, k)
        ax = qk.dim() - 1 - k
        n = qk.shape[ax]
        zero = torch.zeros_like(qk.narrow(ax, 0, 1))
        if n > 1:
            inner = qk.narrow(ax, 0, n - 1)
            term = torch.cat([inner, zero], dim=ax) - torch.cat([zero, inner], dim=ax)
        else:
            term = torch.zeros_like(qk)
        out = term if out is None else out + term
    return out


def _zero_last(p: torch.Tensor, ndim: int) -> torch.Tensor:
    """Set flow component k to 0 on the last index of axis k."""
    comps = []
    for k in range(ndim):
        pk = p.select(-4, k)
        ax = pk.dim() - 1 - k
        n = pk.shape[ax]
        zero = torch.zeros_like(pk.narrow(ax, 0, 1))
        comps.append(torch.cat([pk.narrow(ax, 0, n - 1), zero], dim=ax) if n > 1 else zero)
    return torch.stack(comps, dim=-4)


def project(p: torch.Tensor, S: torch.Tensor) -> torch.Tensor:
    """Projection onto the pointwise ball |q(x)| <= S(x).

    p [..., nd, Z, Y, X]; S broadcastable to [..., Z, Y, X], S >= 0.
    """
    ss = (p * p).sum(dim=-4)
    S = S.expand_as(ss)
    out = ss > S * S                     # outside the ball (implies |p| > 0)
    safe = torch.where(out, ss, torch.ones_like(ss))
    scale = torch.where(out, S / torch.sqrt(safe), torch.ones_like(ss))
    return p * scale.unsqueeze(-4)


def expand_S(S, s_mode: str, B: int, n_node: int, Z: int, Y: int, X: int) -> torch.Tensor:
    """Smoothness term as float64 broadcastable to [B][n_node][Z][Y][X]."""
    S = _t(S)
    if s_mode == "node_scalar":
        assert S.shape == (n_node,)
        return S.view(1, n_node, 1, 1, 1)
    if s_mode == "shared_field":
        assert S.shape == (B, Z, Y, X)
        return S.view(B, 1, Z, Y, X)
    if s_mode == "node_field":
        assert S.shape == (B, n_node, Z, Y, X)
        return S
    raise ValueError(s_mode)


# -------------------------------------------------------- Potts model ---

def potts_iteration(ell, q, D, S, c: float, tau: float, ndim: int, literal: bool = False):
    """One pass of the loop of Algorithm 1 (pseudo-flow Potts).

    ell [B][n][Z][Y][X] (ln u), q [B][n][nd][Z][Y][X], D [B][n][...],
    S broadcastable to [B][n][Z][Y][X].  Returns (ell, q, d) where d is the
    flow excess D + div q used by the label step.
    """
    d = D + div(q, ndim)                                   # D_L + div q_L
    if literal:
        # printed form: multiply, take the flow step on the un-normalised
        # product, then normalise
        w = torch.exp(ell) * torch.exp(-d / c)
        q = project(_zero_last(q - c * tau * grad(w, ndim), ndim), S)
        ell = torch.log(w / w.sum(dim=1, keepdim=True))
        return ell, q, d
    t = ell - d / c                                        # ln(v exp(-d/c))
    ell = t - torch.logsumexp(t, dim=1, keepdim=True)      # normalise (a = sum)
    u = torch.exp(ell)
    q = project(_zero_last(q - c * tau * grad(u, ndim), ndim), S)
    return ell, q, d


def energy_potts(u, D, S, ndim: int) -> torch.Tensor:
    """Relaxed Potts energy per problem: sum_x sum_L D_L u_L + S_L |grad u_L|."""
    g = grad(u, ndim)
    tv = torch.sqrt((g * g).sum(dim=2))
    return (D * u + S * tv).sum(dim=(1, 2, 3, 4))


def dual_potts(q, D, ndim: int) -> torch.Tensor:
    """Pseudo-flow dual per problem: sum_x min_L (D_L + div q_L)."""
    d = D + div(q, ndim)
    return d.min(dim=1).values.sum(dim=(1, 2, 3))


def solve_potts(D, S, s_mode: str, c: float, tau: float, iters: int, ndim: int,
                history: bool = True, literal: bool = False, ell0=None, q0=None,
                callback=None) -> Dict[str, object]:
    """Run Algorithm 1 for ``iters`` iterations from u = 1/n, q = 0."""
    D = _t(D)
    B, n, Z, Y, X = D.shape
    Sx = expand_S(S, s_mode, B, n, Z, Y, X)
    ell = torch.full_like(D, -math.log(n)) if ell0 is None else _t(ell0)
    q = torch.zeros(B, n, ndim, Z, Y, X, dtype=F64) if q0 is None else _t(q0)
    E, P = [], []
    for k in range(iters):
        ell, q, _ = potts_iteration(ell, q, D, Sx, c, tau, ndim, literal)
        if history:
            u = torch.exp(ell)
            E.append(float(energy_potts(u, D, Sx, ndim).sum()))
            P.append(float(dual_potts(q, D, ndim).sum()))
        if callback is not None:
            callback(k, ell, q)
    u = torch.exp(ell)
    return {"ell": ell, "u": u, "q": q, "E": E, "P": P,
            "labels": torch.argmax(u, dim=1)}


# ----------------------------------------------------- label graphs ------

class OracleGraph:
    """Label DAG with the source as node 0 (the paper's S).

    Built from edge lists; weights default to w_(A,B) = 1/|B.P|.  Leaves
    (end-labels, the paper's blackboard L) are the non-source nodes without
    children, in ascending node id.  ``order`` is a top-down topological
    order starting with the source (smallest id first among ready nodes).
    """

    def __init__(self, n_nodes: int, parent: Sequence[int], child: Sequence[int],
                 weight: Optional[Sequence[float]] = None, check: bool = True):
        self.n_nodes = int(n_nodes)
        parent = [int(p) for p in parent]
        child = [int(c) for c in child]
        if len(parent) != len(child):
            raise ValueError("edge arrays differ in length")
        self.parents: List[List[int]] = [[] for _ in range(self.n_nodes)]
        self.children: List[List[int]] = [[] for _ in range(self.n_nodes)]
        for p, c in zip(parent, child):
            if not (0 <= p < self.n_nodes and 0 <= c < self.n_nodes) or p == c:
                raise ValueError(f"bad edge {p}->{c}")
            if c in self.children[p]:
                raise ValueError(f"duplicate edge {p}->{c}")
            self.children[p].append(c)
            self.parents[c].append(p)
        self.w: Dict[tuple, float] = {}
        for i, (p, c) in enumerate(zip(parent, child)):
            if weight is None:
                self.w[(p, c)] = 1.0 / len(self.parents[c])
            else:
                self.w[(p, c)] = float(weight[i])
        for a in range(self.n_nodes):
            self.children[a].sort()
            self.parents[a].sort()
        self.leaves = [a for a in range(1, self.n_nodes) if not self.children[a]]
        self.leaf_index = {a: i for i, a in enumerate(self.leaves)}
        self.order = self._topological()
        if check:
            self.validate()

    @property
    def n_leaf(self) -> int:
        return len(self.leaves)

    @property
    def n_node(self) -> int:
        return self.n_nodes - 1

    def _topological(self) -> List[int]:
        indeg = [len(self.parents[a]) for a in range(self.n_nodes)]
        ready = [a for a in range(self.n_nodes) if indeg[a] == 0]
        heapq.heapify(ready)
        order = []
        while ready:
            a = heapq.heappop(ready)
            order.append(a)
            for c in self.children[a]:
                indeg[c] -= 1
                if indeg[c] == 0:
                    heapq.heappush(ready, c)
        return order

    def validate(self) -> None:
        if len(self.order) != self.n_nodes:
            raise ValueError("label graph has a cycle")
        if self.parents[0]:
            raise ValueError("the source has a parent")
        if self.order[0] != 0:
            raise ValueError("a non-source node has no parent")
        if not self.leaves:
            raise ValueError("no end-labels")
        for (p, c), w in self.w.items():
            if not (w > 0.0):
                raise ValueError(f"non-positive weight on {p}->{c}")
        W = self.path_weights()
        for L in self.leaves:
            if abs(W[0][L] - 1.0) > 1e-12:
                raise ValueError(f"W(S,{L}) = {W[0][L]} != 1")

    def path_weights(self) -> List[List[float]]:
        """W[A][B] = sum over paths A -> B of the product of edge weights."""
        n = self.n_nodes
        W = [[0.0] * n for _ in range(n)]
        for A in reversed(self.order):            # children before parents
            W[A][A] = 1.0
            for C in self.children[A]:
                for B in range(n):
                    if W[C][B] != 0.0:
                        W[A][B] += self.w[(A, C)] * W[C][B]
        return W

    def is_tree(self) -> bool:
        return all(len(self.parents[a]) <= 1 for a in range(1, self.n_nodes))


def _flow_excess(q, D, graph: OracleGraph, ndim: int) -> Dict[int, torch.Tensor]:
    """Flow excess d_A of every non-source node, from its definition in the
    DAGMF section: d_S = 0, and for A != S
        d_A = div q_A + sum_{P in A.P} w_(P,A) d_P   (+ D_A when A is an end-label).
    Evaluated as a memoised recursion over the parents (the source term is
    0), so the value of a node is read straight off the definition."""
    dq = div(q, ndim)                                     # [B][n_node][Z][Y][X]
    memo: Dict[int, torch.Tensor] = {}

    def d_of(A: int) -> Optional[torch.Tensor]:
        if A == 0:
            return None                                   # d_S = 0
        if A not in memo:
            val = dq[:, A - 1]
            if A in graph.leaf_index:
                val = val + D[:, graph.leaf_index[A]]
            for P in graph.parents[A]:
                dP = d_of(P)
                if dP is not None:
                    val = val + graph.w[(P, A)] * dP
            memo[A] = val
        return memo[A]

    return {A: d_of(A) for A in range(1, graph.n_nodes)}


def dag_upward(u, graph: OracleGraph) -> Dict[int, torch.Tensor]:
    """Implicit labels from the labelling constraint of the DAGMF model:
    U_L = u_L on end-labels and U_A = sum_{C in A.C} w_(A,C) U_C otherwise,
    as a memoised recursion over the children."""
    memo: Dict[int, torch.Tensor] = {}

    def U_of(A: int) -> torch.Tensor:
        if A not in memo:
            if A in graph.leaf_index:
                memo[A] = u[:, graph.leaf_index[A]]
            else:
                memo[A] = sum(graph.w[(A, C)] * U_of(C) for C in graph.children[A])
        return memo[A]

    return {A: U_of(A) for A in range(1, graph.n_nodes)}


def dag_iteration(ell, q, D, S, graph: OracleGraph, c: float, tau: float, ndim: int):
    """One iteration of the pseudo-flow DAGMF method (Algorithm 2): the flow
    excess of every end-label, the closed-form entropic label update over the
    end-labels, then the Chambolle flow update of every non-source node A
    driven by the implicit label U_A of the normalised end-labels.

    ell [B][n_leaf][...], q [B][n_node][nd][...] (node A at index A-1),
    D [B][n_leaf][...], S broadcastable to [B][n_node][Z][Y][X].
    """
    d = _flow_excess(q, D, graph, ndim)
    dl = torch.stack([d[L] for L in graph.leaves], dim=1)
    t = ell - dl / c
    ell = t - torch.logsumexp(t, dim=1, keepdim=True)
    U = dag_upward(torch.exp(ell), graph)
    newq = []
    for A in range(1, graph.n_nodes):
        SA = S[:, A - 1] if S.shape[1] > 1 else S[:, 0]
        newq.append(project(_zero_last(q[:, A - 1] - c * tau * grad(U[A], ndim), ndim), SA))
    return ell, torch.stack(newq, dim=1), dl


def energy_dag(u, D, S, graph: OracleGraph, ndim: int) -> torch.Tensor:
    """DAGMF energy per problem: sum_x sum_{L leaf} D_L u_L
    + sum_{A != S} S_A |grad U_A| with U from the labelling constraint."""
    U = dag_upward(u, graph)
    e = (D * u).sum(dim=(1, 2, 3, 4))
    for A in range(1, graph.n_nodes):
        g = grad(U[A], ndim)
        SA = S[:, A - 1] if S.shape[1] > 1 else S[:, 0]
        e = e + (SA * torch.sqrt((g * g).sum(dim=1))).sum(dim=(1, 2, 3))
    return e


def dual_dag(q, D, graph: OracleGraph, ndim: int) -> torch.Tensor:
    """Pseudo-flow dual per problem: sum_x min over end-labels of d_L."""
    d = _flow_excess(q, D, graph, ndim)
    dl = torch.stack([d[L] for L in graph.leaves], dim=1)
    return dl.min(dim=1).values.sum(dim=(1, 2, 3))


def solve_dagmf(D, S, s_mode: str, graph: OracleGraph, c: float, tau: float, iters: int,
                ndim: int, history: bool = True, ell0=None, q0=None,
                callback=None) -> Dict[str, object]:
    """Run Algorithm 2 for ``iters`` iterations from u = 1/|leaves|, q = 0.
    A tree graph is the HMF model."""
    D = _t(D)
    B, nl, Z, Y, X = D.shape
    assert nl == graph.n_leaf
    Sx = expand_S(S, s_mode, B, graph.n_node, Z, Y, X)
    ell = torch.full_like(D, -math.log(nl)) if ell0 is None else _t(ell0)
    q = torch.zeros(B, graph.n_node, ndim, Z, Y, X, dtype=F64) if q0 is None else _t(q0)
    E, P = [], []
    for k in range(iters):
        ell, q, _ = dag_iteration(ell, q, D, Sx, graph, c, tau, ndim)
        if history:
            u = torch.exp(ell)
            E.append(float(energy_dag(u, D, Sx, graph, ndim).sum()))
            P.append(float(dual_dag(q, D, graph, ndim).sum()))
        if callback is not None:
            callback(k, ell, q)
    u = torch.exp(ell)
    return {"ell": ell, "u": u, "q": q, "E": E, "P": P,
            "labels": torch.argmax(u, dim=1)}


# ------------------------------------------------------ brute force ------

def brute_force_min_energy(D, S, s_mode: str, graph: OracleGraph, ndim: int,
                           chunk: int = 1 << 16) -> float:
    """Smallest energy over all integral labellings (every voxel takes one
    end-label), by enumeration.  Only for tiny grids: |leaves|^voxels cases.
    D [1][n_leaf][Z][Y][X]."""
    D = _t(D)
    _, nl, Z, Y, X = D.shape
    V = Z * Y * X
    total = nl ** V
    Sx = expand_S(S, s_mode, 1, graph.n_node, Z, Y, X)
    best = math.inf
    powers = torch.tensor([nl ** i for i in range(V)], dtype=torch.int64)
    for start in range(0, total, chunk):
        idx = torch.arange(start, min(total, start + chunk), dtype=torch.int64)
        lab = (idx[:, None] // powers[None, :]) % nl          # [M][V]
        u = torch.nn.functional.one_hot(lab, nl).to(F64)      # [M][V][nl]
        u = u.permute(0, 2, 1).reshape(-1, nl, Z, Y, X)
        Db = D.expand(u.shape[0], -1, -1, -1, -1)
        Sb = Sx.expand(u.shape[0], -1, -1, -1, -1) if Sx.shape[0] == 1 else Sx
        e = energy_dag(u, Db, Sb, graph, ndim)
        best = min(best, float(e.min()))
    return best


# --------------------------------------------------- Ishikawa model ------

def _ishikawa_excess(q, D, ndim: int) -> torch.Tensor:
    """Flow excess of the chain labels L_0..L_N (Algorithm 3): d_{L_0} = D_0
    and d_{L_i} = D_i + sum_{j=1..i} div q_j, i.e. L_i receives the flow of
    every level at or below it."""
    dq = div(q, ndim)                                      # [B][N][...]
    zero = torch.zeros_like(dq[:, :1])
    return torch.cumsum(torch.cat([zero, dq], dim=1), dim=1) + D


def ishikawa_iteration(ell, q, D, S, c: float, tau: float, ndim: int):
    """One iteration of the pseudo-flow Ishikawa chain (Algorithm 3), labels
    L_0..L_N and flows q_1..q_N: the chain's flow excess, the entropic label
    update, and the Chambolle step of q_i driven by the accumulated label
    U_i = sum_{j >= i} u_j (the super-object made of L_i and every label
    above it in the chain).

    ell [B][N+1][...], q [B][N][nd][...] (flow of L_i at index i-1),
    S broadcastable to [B][N][Z][Y][X]."""
    n = ell.shape[1]
    dl = _ishikawa_excess(q, D, ndim)
    t = ell - dl / c
    ell = t - torch.logsumexp(t, dim=1, keepdim=True)
    u = torch.exp(ell)
    newq = []
    for i in range(1, n):
        Ui = u[:, i:].sum(dim=1)
        Si = S[:, i - 1] if S.shape[1] > 1 else S[:, 0]
        newq.append(project(_zero_last(q[:, i - 1] - c * tau * grad(Ui, ndim), ndim), Si))
    return ell, torch.stack(newq, dim=1), dl


def energy_ishikawa(u, D, S, ndim: int) -> torch.Tensor:
    """sum_x sum_i D_i u_i + sum_{i>=1} S_i |grad U_i|, U_i = sum_{j>=i} u_j."""
    n = u.shape[1]
    e = (D * u).sum(dim=(1, 2, 3, 4))
    for i in range(1, n):
        Ui = u[:, i:].sum(dim=1)
        g = grad(Ui, ndim)
        Si = S[:, i - 1] if S.shape[1] > 1 else S[:, 0]
        e = e + (Si * torch.sqrt((g * g).sum(dim=1))).sum(dim=(1, 2, 3))
    return e


def dual_ishikawa(q, D, ndim: int) -> torch.Tensor:
    """Pseudo-flow dual per problem: sum_x min_i d_{L_i}."""
    return _ishikawa_excess(q, D, ndim).min(dim=1).values.sum(dim=(1, 2, 3))


def solve_ishikawa(D, S, s_mode: str, c: float, tau: float, iters: int, ndim: int,
                   history: bool = True) -> Dict[str, object]:
    """Run Algorithm 3 from u = 1/(N+1), q = 0."""
    D = _t(D)
    B, n, Z, Y, X = D.shape
    Sx = expand_S(S, s_mode, B, n - 1, Z, Y, X)
    ell = torch.full_like(D, -math.log(n))
    q = torch.zeros(B, n - 1, ndim, Z, Y, X, dtype=F64)
    E, P = [], []
    for _ in range(iters):
        ell, q, _ = ishikawa_iteration(ell, q, D, Sx, c, tau, ndim)
        if history:
            E.append(float(energy_ishikawa(torch.exp(ell), D, Sx, ndim).sum()))
            P.append(float(dual_ishikawa(q, D, ndim).sum()))
    u = torch.exp(ell)
    return {"ell": ell, "u": u, "q": q, "E": E, "P": P, "labels": torch.argmax(u, dim=1)}
