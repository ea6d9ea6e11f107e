"""Pins of the full-flow reference implementation (the counterpart of the
pseudo-flow method; primal and primal-dual Potts models of the section
"Pseudo-Flow Approach to the Potts Model") against what the model and the
mathematics fix: closed forms of the first iteration from the initial flows,
the labelling constraint that the source-flow step restores exactly, the
pointwise problem when S = 0, weak duality, an independent LP solver on 1-D
chains (where the relaxation is a linear programme), flow conservation at
convergence, and agreement with the pseudo-flow optimum."""
import numpy as np
import pytest
import torch

from oracle import fullflow_oracle as F
from oracle import pseudoflow_oracle as O
from paper_1501_07844_amd import synth

from test_oracle_pins import _lp_optimum_chain

torch.set_num_threads(min(8, torch.get_num_threads()))


def test_first_iteration_from_the_initial_flows():
    """From q = 0, p_S = p_L = m = min_L D_L and u = 1/n the quantity whose
    gradient drives the spatial flows is the constant -1/(n c), so q stays 0;
    the sink flows are then min(D_L, m + 1/(n c)), the source flow their mean,
    and the labels 1/n + c (p_S - p_L)."""
    p = synth.random_potts(3, (1, 5, 6), 2, 4, s_mode="node_field", d_scale=3.0)
    c, tau = 0.7, 0.2
    r = F.solve_potts_fullflow(p.D, p.S, p.s_mode, c, tau, 1, 2, history=False)
    assert torch.all(r["q"] == 0)
    D = p.D.astype(np.float64)
    n = D.shape[1]
    for y in range(5):
        for x in range(6):
            d = [D[0, L, 0, y, x] for L in range(n)]
            m = min(d)
            pl = [min(dl, m + 1.0 / (n * c)) for dl in d]
            ps = sum(pl) / n
            assert abs(float(r["pS"][0, 0, 0, y, x]) - ps) < 1e-14
            for L in range(n):
                assert abs(float(r["pL"][0, L, 0, y, x]) - pl[L]) < 1e-14
                assert abs(float(r["u"][0, L, 0, y, x]) - (1.0 / n + c * (ps - pl[L]))) < 1e-14


def test_second_iteration_flow_step():
    """The second spatial-flow step is one projected ascent step from q = 0
    along the forward-difference gradient of div q - p_S + p_L - u/c, i.e. of
    p_L - p_S - u_L / c after the first iteration (loops, small and large S)."""
    for s_range in ((5.0, 6.0), (0.01, 0.02)):
        p = synth.random_potts(4, (1, 4, 5), 2, 3, s_mode="node_field", d_scale=3.0,
                               s_range=s_range)
        c, tau = 0.9, 0.15
        r1 = F.solve_potts_fullflow(p.D, p.S, p.s_mode, c, tau, 1, 2, history=False)
        r2 = F.solve_potts_fullflow(p.D, p.S, p.s_mode, c, tau, 2, 2, history=False)
        f = (r1["pL"] - r1["pS"] - r1["u"] / c).numpy()[0]         # [n][1][Y][X]
        S = p.S.astype(np.float64)[0]
        q2 = r2["q"].numpy()[0]                                      # [n][2][1][Y][X]
        for L in range(3):
            for y in range(4):
                for x in range(5):
                    gx = f[L, 0, y, x + 1] - f[L, 0, y, x] if x < 4 else 0.0
                    gy = f[L, 0, y + 1, x] - f[L, 0, y, x] if y < 3 else 0.0
                    px, py = tau * gx, tau * gy
                    nrm = (px * px + py * py) ** 0.5
                    s = S[L, 0, y, x]
                    if nrm > s:
                        px, py = px * s / nrm, py * s / nrm
                    assert abs(q2[L, 0, 0, y, x] - px) < 1e-14
                    assert abs(q2[L, 1, 0, y, x] - py) < 1e-14


def test_labels_sum_to_one_after_every_iteration():
    """The source-flow step is the exact maximiser of the augmented
    Lagrangian, whose optimality condition is 1 - sum_L u_L + c sum_L R_L = 0;
    after the multiplier step that is sum_L u_L = 1 at every voxel."""
    p = synth.potts3d_voronoi(shape=(5, 7, 9), iters=15)
    st = F.init_state(O._t(p.D), 3)
    Sx = O.expand_S(p.S, p.s_mode, 1, p.n_leaf, 5, 7, 9)
    for _ in range(15):
        st = F.fullflow_iteration(st, O._t(p.D), Sx, 1.0, 0.11, 3)
        assert float((st["u"].sum(dim=1) - 1).abs().max()) < 1e-12


def test_S_zero_gives_the_pointwise_argmin():
    """With S = 0 the spatial flows stay 0 and every voxel solves
    min_u sum_L u_L D_L on the simplex, whose solution is the indicator of
    argmin_L D_L (data terms a permutation of 0, 0.5, 1, 1.5 per voxel)."""
    p = synth.random_potts(5, (1, 6, 7), 2, 4, s_range=(0.0, 0.0))
    rng = np.random.default_rng(5)
    perm = np.argsort(rng.random((1, 1, 6, 7, 4)), axis=-1).transpose(0, 4, 1, 2, 3)
    p.D = (0.5 * perm).astype(np.float32)
    r = F.solve_potts_fullflow(p.D, p.S, p.s_mode, 0.5, 0.2, 400, 2, history=False)
    assert torch.all(r["q"] == 0)
    am = np.argmin(p.D, axis=1)
    onehot = np.eye(4)[am].transpose(0, 4, 1, 2, 3)
    assert np.abs(r["u"].numpy() - onehot).max() < 1e-6
    assert np.array_equal(r["labels"].numpy(), am)


@pytest.mark.parametrize("nd,shape", [(2, (1, 9, 11)), (3, (4, 5, 6))])
def test_weak_duality_and_feasible_flows_every_iteration(nd, shape):
    """P(q) = int min_L (D_L + div q_L) is a lower bound of the relaxed
    energy for every |q_L| <= S_L, and the clipped, renormalised labelling is a
    point of the simplex, so P <= E at every iteration."""
    p = synth.random_potts(6, shape, nd, 3, s_mode="shared_field", d_scale=3.0)
    r = F.solve_potts_fullflow(p.D, p.S, p.s_mode, 1.0, 0.1, 60, nd)
    E, P = np.array(r["E"]), np.array(r["P"])
    assert np.all(P <= E + 1e-12 * np.abs(E))
    nrm = torch.sqrt((r["q"] ** 2).sum(dim=2))
    assert float((nrm - O._t(p.S)[:, None]).max()) <= 1e-12


@pytest.mark.parametrize("c,tau", [(0.5, 0.2), (2.0, 0.3)])
def test_chain_matches_lp_optimum(c, tau):
    """On a 1-D chain the relaxed Potts energy is a linear programme (scipy
    HiGHS, independent of this code): E and P bracket its optimum at every
    iteration, the gap closes onto it, and flow conservation holds at the
    end."""
    N = 9
    p = synth.random_potts(33, (1, 1, N), 2, 3, d_scale=3.0, s_range=(0.3, 1.2),
                           s_mode="node_field")
    Dm = p.D[0, :, 0, 0, :].astype(np.float64)
    Smat = p.S[0, :, 0, 0, :].astype(np.float64)
    lp = _lp_optimum_chain(Dm, Smat, np.eye(3))
    r = F.solve_potts_fullflow(p.D, p.S, p.s_mode, c, tau, 3000, 2)
    E, P = np.array(r["E"]), np.array(r["P"])
    tol = 1e-9 * abs(lp)
    assert np.all(P <= lp + tol) and np.all(E >= lp - tol)
    assert E[-1] - P[-1] < 1e-6 * abs(lp)
    assert r["residual"][-1] < 1e-6


def test_same_optimum_as_the_pseudoflow_method():
    """Both methods solve the same relaxed Potts model: on the 64 x 64
    workload their certified intervals [P, E] after 200 iterations overlap
    and are each within 1e-4 of the energy."""
    p = synth.potts2d_rects()
    ff = F.solve_potts_fullflow(p.D, p.S, p.s_mode, 0.3, 0.16, 200, 2)
    ps = O.solve_potts(p.D, p.S, p.s_mode, p.c, p.tau, 200, 2)
    Ef, Pf, Ep, Pp = ff["E"][-1], ff["P"][-1], ps["E"][-1], ps["P"][-1]
    assert Ef - Pf < 1e-4 * Ef and Ep - Pp < 1e-4 * Ep
    assert max(Pf, Pp) <= min(Ef, Ep) + 1e-9 * Ef
