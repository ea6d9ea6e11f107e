"""Closed-form pins of one and two iterations of the oracle, written out with
plain loops over voxels, labels and nodes (no call into the oracle's own
operators).

From the initial state (u = 1/n, q = 0) every flow divergence is 0, so the
first label update of the Potts section (and of the DAGMF section) is the
softmax of -D/c, independent of the flows.  The first flow update is then
the projected Chambolle step q_1 = Proj_{|q| <= S}(-c tau grad U_1) of the
flow-update equations, with U the normalised label of the node (Potts: u_L;
DAGMF: sum_L W_(A,L) u_L; Ishikawa chain: sum_{j >= i} u_j).  The second
label update is the softmax of ln u_1 - (D + excess of q_1)/c with the
excess as the DAGMF section defines it (d_A = div q_A + sum over parents
P of w_(P,A) d_P, d_S = 0; the chain's d_i = D_i + sum_{j <= i} div q_j).

The cases use c != 1 and tau != 1 so that the flow-step size c*tau is
distinguished from c, tau and 1, and capacities both above the largest step
(projection inactive) and below the typical one (projection active on some
voxels), in 1-D (where the ball is an interval, so the projection is a clip)
and on a 2 x 2 x 2 grid (the Euclidean ball of R^3, written out by hand).
"""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import pseudoflow_oracle as O

F64 = torch.float64
C_, TAU = 2.5, 0.1         # c * tau = 0.25, distinct from c, tau and 1


def _softmax_vox(a):
    m = max(a)
    e = [math.exp(x - m) for x in a]
    s = sum(e)
    return [x / s for x in e]


def _grid_points(shape):
    Z, Y, X = shape
    return list(itertools.product(range(Z), range(Y), range(X)))


def _step_by_hand(U, S, shape, nd):
    """Proj_{|p| <= S}(-c tau grad U) at every voxel, with loops.
    U: dict (z, y, x) -> value; S: dict (z, y, x) -> capacity.
    Returns dict (z, y, x) -> list of nd components (x, y, z order)."""
    Z, Y, X = shape
    ext = (X, Y, Z)
    out = {}
    for (z, y, x) in _grid_points(shape):
        pos = (x, y, z)
        p = []
        for k in range(nd):
            if pos[k] < ext[k] - 1:
                nb = list(pos)
                nb[k] += 1
                g = U[(nb[2], nb[1], nb[0])] - U[(z, y, x)]
                p.append(-C_ * TAU * g)
            else:
                p.append(0.0)
        n = math.sqrt(sum(c * c for c in p))
        s = S[(z, y, x)]
        if n > s:
            p = [c * s / n for c in p]
        out[(z, y, x)] = p
    return out


def _clip_1d(U, S, X):
    """1-D case with a library routine: the ball of R^1 is an interval."""
    g = np.zeros(X)
    g[:-1] = np.diff(U)
    return np.clip(-C_ * TAU * g, -S, S)


def _div_by_hand(q, shape, nd):
    """div q(x) = sum_k q_k(x)[x_k < N_k - 1] - q_k(x - e_k)[x_k > 0]."""
    Z, Y, X = shape
    ext = (X, Y, Z)
    out = {}
    for (z, y, x) in _grid_points(shape):
        pos = (x, y, z)
        v = 0.0
        for k in range(nd):
            if pos[k] < ext[k] - 1:
                v += q[(z, y, x)][k]
            if pos[k] > 0:
                pb = list(pos)
                pb[k] -= 1
                v -= q[(pb[2], pb[1], pb[0])][k]
        out[(z, y, x)] = v
    return out


def _to_field(d, shape):
    Z, Y, X = shape
    a = np.zeros((Z, Y, X))
    for key, v in d.items():
        a[key] = v
    return a


def _flow_tensor(qs, shape, nd):
    """list over flows of dicts -> tensor [1][n][nd][Z][Y][X]."""
    Z, Y, X = shape
    t = np.zeros((1, len(qs), nd, Z, Y, X))
    for A, qa in enumerate(qs):
        for key, comps in qa.items():
            for k in range(nd):
                t[(0, A, k) + key] = comps[k]
    return torch.tensor(t, dtype=F64)


# ------------------------------------------------------- Potts section ---

@pytest.mark.parametrize("s_level", ["inactive", "active"])
def test_potts_one_dimensional_first_steps(s_level):
    """Potts on a 1 x 1 x 7 chain, three labels: the first flow step is the
    clipped -c tau grad u_1 and the second label step uses D + div q_1."""
    rng = np.random.default_rng(5)
    X, n = 7, 3
    D = rng.uniform(0.0, 2.0, size=(1, n, 1, 1, X))
    S = np.array([10.0, 10.0, 10.0]) if s_level == "inactive" else np.array([0.02, 0.05, 0.03])
    ell0 = torch.full((1, n, 1, 1, X), -math.log(n), dtype=F64)
    q0 = torch.zeros(1, n, 2, 1, 1, X, dtype=F64)
    St = torch.tensor(S).view(1, n, 1, 1, 1)
    ell1, q1, _ = O.potts_iteration(ell0, q0, torch.tensor(D), St, C_, TAU, 2)
    ell2, _, _ = O.potts_iteration(ell1, q1, torch.tensor(D), St, C_, TAU, 2)

    u1 = np.array([_softmax_vox([-D[0, L, 0, 0, i] / C_ for L in range(n)]) for i in range(X)]).T
    assert np.abs(np.exp(ell1.numpy()[0, :, 0, 0]) - u1).max() < 1e-15
    q1x = np.stack([_clip_1d(u1[L], S[L], X) for L in range(n)])
    assert np.abs(q1.numpy()[0, :, 0, 0, 0] - q1x).max() < 1e-15
    assert float(q1[0, :, 1].abs().max()) == 0.0          # no y extent, no y flow
    if s_level == "active":
        clipped = np.isclose(np.abs(q1x), S[:, None], rtol=0, atol=0)
        assert clipped.any() and not clipped.all()
    # second label step: ell_1 - (D + div q_1)/c, normalised
    dv = np.zeros((n, X))
    for L in range(n):
        for i in range(X):
            dv[L, i] = (q1x[L, i] if i < X - 1 else 0.0) - (q1x[L, i - 1] if i > 0 else 0.0)
    for i in range(X):
        t = [math.log(u1[L, i]) - (D[0, L, 0, 0, i] + dv[L, i]) / C_ for L in range(n)]
        u2 = _softmax_vox(t)
        for L in range(n):
            assert abs(math.exp(float(ell2[0, L, 0, 0, i])) - u2[L]) < 1e-15


@pytest.mark.parametrize("s_level", ["inactive", "active"])
def test_potts_cube_first_steps(s_level):
    """Potts on a 2 x 2 x 2 grid, four labels, a capacity field: the first
    flow step is the Euclidean-ball projection of -c tau grad u_1 in R^3."""
    rng = np.random.default_rng(6)
    shape, n, nd = (2, 2, 2), 4, 3
    D = rng.uniform(0.0, 3.0, size=(1, n) + shape)
    hi = 10.0 if s_level == "inactive" else 0.04
    S = rng.uniform(0.5 * hi, hi, size=(1, n) + shape)
    ell0 = torch.full((1, n) + shape, -math.log(n), dtype=F64)
    q0 = torch.zeros((1, n, nd) + shape, dtype=F64)
    ell1, q1, _ = O.potts_iteration(ell0, q0, torch.tensor(D), torch.tensor(S), C_, TAU, nd)
    ell2, _, _ = O.potts_iteration(ell1, q1, torch.tensor(D), torch.tensor(S), C_, TAU, nd)
    pts = _grid_points(shape)
    u1 = {pt: _softmax_vox([-D[(0, L) + pt] / C_ for L in range(n)]) for pt in pts}
    qs = []
    for L in range(n):
        U = {pt: u1[pt][L] for pt in pts}
        qs.append(_step_by_hand(U, {pt: S[(0, L) + pt] for pt in pts}, shape, nd))
    assert float((q1 - _flow_tensor(qs, shape, nd)).abs().max()) < 1e-15
    if s_level == "active":
        norms = [math.sqrt(sum(c * c for c in qs[L][pt])) for L in range(n) for pt in pts]
        caps = [S[(0, L) + pt] for L in range(n) for pt in pts]
        on = [abs(a - b) < 1e-15 for a, b in zip(norms, caps)]
        assert any(on) and not all(on)
    divs = [_div_by_hand(qs[L], shape, nd) for L in range(n)]
    for pt in pts:
        t = [math.log(u1[pt][L]) - (D[(0, L) + pt] + divs[L][pt]) / C_ for L in range(n)]
        u2 = _softmax_vox(t)
        for L in range(n):
            assert abs(math.exp(float(ell2[(0, L) + pt])) - u2[L]) < 1e-15


# ------------------------------------------------------- DAGMF section ---

# two-level tree: S -> {1, 2}, 1 -> {3, 4}, 2 -> {5, 6}; and a DAG with a
# shared end-label: S -> {1, 2}, 1 -> {3, 4}, 2 -> {4, 5}, w(1,4) = w(2,4) = 1/2
GRAPHS = {
    "tree": (7, [0, 0, 1, 1, 2, 2], [1, 2, 3, 4, 5, 6], None),
    "dag": (6, [0, 0, 1, 1, 2, 2], [1, 2, 3, 4, 4, 5], None),
}


@pytest.mark.parametrize("s_level", ["inactive", "active"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_dag_cube_first_steps(name, s_level):
    """DAGMF on a 2 x 2 x 2 grid: the first flow step of every node A is the
    projection of -c tau grad U_A with U_A the weighted sum of the normalised
    end-labels under A; the second label step adds the top-down excess."""
    n_nodes, par, chi, w = GRAPHS[name]
    g = O.OracleGraph(n_nodes, par, chi, w)
    # weights and children written out for this test, not taken from g
    wt = {}
    for p_, c_ in zip(par, chi):
        wt[(p_, c_)] = 1.0 / sum(1 for x in chi if x == c_)
    kids = {a: [c_ for p_, c_ in zip(par, chi) if p_ == a] for a in range(n_nodes)}
    parents = {a: [p_ for p_, c_ in zip(par, chi) if c_ == a] for a in range(n_nodes)}
    leaves = [a for a in range(1, n_nodes) if not kids[a]]
    assert leaves == g.leaves
    rng = np.random.default_rng(7)
    shape, nd = (2, 2, 2), 3
    nl, nn = len(leaves), n_nodes - 1
    D = rng.uniform(0.0, 3.0, size=(1, nl) + shape)
    hi = 10.0 if s_level == "inactive" else 0.04
    S = rng.uniform(0.5 * hi, hi, size=(1, nn) + shape)
    ell0 = torch.full((1, nl) + shape, -math.log(nl), dtype=F64)
    q0 = torch.zeros((1, nn, nd) + shape, dtype=F64)
    ell1, q1, _ = O.dag_iteration(ell0, q0, torch.tensor(D), torch.tensor(S), g, C_, TAU, nd)
    ell2, _, _ = O.dag_iteration(ell1, q1, torch.tensor(D), torch.tensor(S), g, C_, TAU, nd)
    pts = _grid_points(shape)
    u1 = {pt: _softmax_vox([-D[(0, i) + pt] / C_ for i in range(nl)]) for pt in pts}

    def U_at(a, pt):
        if a in leaves:
            return u1[pt][leaves.index(a)]
        return sum(wt[(a, c_)] * U_at(c_, pt) for c_ in kids[a])
    qs = []
    for a in range(1, n_nodes):
        U = {pt: U_at(a, pt) for pt in pts}
        qs.append(_step_by_hand(U, {pt: S[(0, a - 1) + pt] for pt in pts}, shape, nd))
    assert float((q1 - _flow_tensor(qs, shape, nd)).abs().max()) < 1e-15
    divs = {a: _div_by_hand(qs[a - 1], shape, nd) for a in range(1, n_nodes)}

    def d_at(a, pt):
        if a == 0:
            return 0.0
        v = divs[a][pt] + sum(wt[(p_, a)] * d_at(p_, pt) for p_ in parents[a])
        if a in leaves:
            v += D[(0, leaves.index(a)) + pt]
        return v
    for pt in pts:
        t = [math.log(u1[pt][i]) - d_at(L, pt) / C_ for i, L in enumerate(leaves)]
        u2 = _softmax_vox(t)
        for i in range(nl):
            assert abs(math.exp(float(ell2[(0, i) + pt])) - u2[i]) < 1e-15


# --------------------------------------------------- Ishikawa section ----

@pytest.mark.parametrize("s_level", ["inactive", "active"])
def test_ishikawa_one_dimensional_first_steps(s_level):
    """Ishikawa chain of N = 3 levels (labels L_0..L_3) on a 1 x 1 x 6 line:
    q_i of the first iteration is the clipped -c tau grad of sum_{j >= i} u_j,
    and the second label step uses d_i = D_i + sum_{j <= i} div q_j."""
    rng = np.random.default_rng(8)
    X, N = 6, 3
    D = rng.uniform(0.0, 2.0, size=(1, N + 1, 1, 1, X))
    S = np.array([10.0] * N) if s_level == "inactive" else np.array([0.03, 0.05, 0.02])
    ell0 = torch.full((1, N + 1, 1, 1, X), -math.log(N + 1), dtype=F64)
    q0 = torch.zeros(1, N, 2, 1, 1, X, dtype=F64)
    St = torch.tensor(S).view(1, N, 1, 1, 1)
    ell1, q1, _ = O.ishikawa_iteration(ell0, q0, torch.tensor(D), St, C_, TAU, 2)
    ell2, _, _ = O.ishikawa_iteration(ell1, q1, torch.tensor(D), St, C_, TAU, 2)
    u1 = np.array([_softmax_vox([-D[0, L, 0, 0, i] / C_ for L in range(N + 1)])
                   for i in range(X)]).T                           # [N+1][X]
    qx = np.zeros((N, X))
    for i in range(1, N + 1):
        Ui = np.array([sum(u1[j, x] for j in range(i, N + 1)) for x in range(X)])
        qx[i - 1] = _clip_1d(Ui, S[i - 1], X)
    assert np.abs(q1.numpy()[0, :, 0, 0, 0] - qx).max() < 1e-15
    dv = np.zeros((N, X))
    for i in range(N):
        for x in range(X):
            dv[i, x] = (qx[i, x] if x < X - 1 else 0.0) - (qx[i, x - 1] if x > 0 else 0.0)
    for x in range(X):
        t = []
        for L in range(N + 1):
            d = D[0, L, 0, 0, x] + sum(dv[j - 1, x] for j in range(1, L + 1))
            t.append(math.log(u1[L, x]) - d / C_)
        u2 = _softmax_vox(t)
        for L in range(N + 1):
            assert abs(math.exp(float(ell2[0, L, 0, 0, x])) - u2[L]) < 1e-15
