"""Parity of the HIP path (through the C ABI) with the float64 reference
implementation, on seeded synthetic workloads at reduced sizes that span many
thread blocks and end in ragged tails, plus edge cases of the method.
Every case compares element by element: u within 1e-4, labels exact where the
reference's top-two margin is decisive, energy/dual relative 1e-4."""
import numpy as np
import pytest
import torch

import paper_1501_07844_amd as pf
from paper_1501_07844_amd import synth
from oracle import pseudoflow_oracle as O

from parity_util import (check_parity, compare_labels, device_inputs, gpu_solve,
                         oracle_energy_dual, oracle_solve, supported_kernels)

pytestmark = pytest.mark.gpu
torch.set_num_threads(max(1, min(16, torch.get_num_threads())))

KERNELS = ["two_pass", "fused", "fused2", "lds"]


def _kernels_for(p):
    return [k for k in supported_kernels(p) if k != "auto"]


def _run_and_check(p, kernel, iters=None, **kw):
    ref = oracle_solve(p, iters)
    res = gpu_solve(p, iters, kernel=kernel, return_q=True, final_energy=True, **kw)
    check_parity(p, ref, res)
    return ref, res


# reduced-size workloads: (name, factory)
WORKLOADS = {
    "potts2d_rects_64x64": lambda: synth.potts2d_rects(),
    "potts3d_voronoi_36x40x44": lambda: synth.potts3d_voronoi(shape=(36, 40, 44), iters=200),
    "hmf_ellipsoids_20x36x44": lambda: synth.hmf_ellipsoids(shape=(20, 36, 44), iters=120),
    "dagmf_blobs_18x30x38": lambda: synth.dagmf_blobs(shape=(18, 30, 38), iters=120),
    "diff_batch_3x40x52": lambda: synth.diff_batch(batch=3, ny=40, nx=52, iters=100),
    "ishikawa_levels_48x61": lambda: synth.ishikawa_levels(shape=(1, 48, 61), iters=150),
    "ishikawa_levels_20x36x44_n7": lambda: synth.ishikawa_levels(shape=(20, 36, 44), n_levels=7,
                                                                 iters=120),
}


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_workload_parity(name, kernel):
    p = WORKLOADS[name]()
    if kernel not in _kernels_for(p):
        pytest.skip(f"no {kernel} kernel for this model")
    print(f"[parity] {name} kernel={kernel} shape={p.shape} iters={p.iters}", flush=True)
    _run_and_check(p, kernel)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("s_mode", ["node_scalar", "shared_field", "node_field"])
@pytest.mark.parametrize("nd,shape,nl", [(2, (1, 37, 29), 5), (3, (7, 11, 13), 3),
                                         (3, (5, 1, 9), 2), (2, (1, 1, 300), 4)])
def test_potts_ragged_shapes_and_s_modes(kernel, s_mode, nd, shape, nl):
    p = synth.random_potts(100 + nl, shape, nd, nl, batch=2, s_mode=s_mode, c=1.0,
                           tau=0.1, iters=30)
    print(f"[parity] potts nd={nd} {shape} nl={nl} {s_mode} {kernel}", flush=True)
    _run_and_check(p, kernel)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("kind", ["tree", "dag", "deep"])
def test_graph_models_random(kernel, kind):
    rng = np.random.default_rng(7)
    if kind == "tree":
        gr = synth.random_tree(rng, 4, 9)
    elif kind == "dag":
        gr = synth.random_dag(rng, 5, 11, max_parents=3)
    else:
        gr = synth.random_dag(rng, 15, 16, max_parents=2)     # 31 nodes, 16 leaves
    p = synth.random_problem(200, (6, 13, 17), 3, gr, batch=2, s_mode="node_field", c=2.0,
                             tau=0.05, iters=25, kind="hmf" if kind == "tree" else "dagmf")
    print(f"[parity] graph {kind} nodes={gr.n_nodes} leaves={gr.n_leaf} {kernel}", flush=True)
    _run_and_check(p, kernel)


def test_hmf_equals_dagmf_on_a_tree():
    p = synth.hmf_ellipsoids(shape=(9, 17, 21), iters=20)
    a = gpu_solve(p, kernel="two_pass", return_q=True)
    p.kind = "dagmf"
    b = gpu_solve(p, kernel="two_pass", return_q=True)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q)


def test_flat_dag_matches_potts():
    p = synth.random_potts(300, (5, 9, 11), 3, 4, s_mode="node_field", c=1.0, tau=0.1, iters=40)
    a = gpu_solve(p, kernel="two_pass", return_q=True)
    p.kind = "dagmf"
    b = gpu_solve(p, kernel="two_pass", return_q=True)
    assert float((a.u - b.u).abs().max()) < 1e-5


def test_degenerate_cases():
    # a single label: u = 1 everywhere and the flow never moves
    p = synth.random_potts(1, (3, 4, 5), 3, 1, iters=10)
    r = gpu_solve(p, return_q=True)
    assert torch.all(r.u == 1.0) and torch.all(r.q == 0.0) and torch.all(r.labels == 0)
    # a single voxel
    p = synth.random_potts(2, (1, 1, 1), 3, 4, iters=10)
    _run_and_check(p, "two_pass")
    # zero iterations: the initial labelling 1/n
    p = synth.random_potts(3, (2, 3, 4), 3, 5, iters=0)
    r = gpu_solve(p, return_q=True)
    assert torch.allclose(r.u, torch.full_like(r.u, 0.2), atol=1e-7) and torch.all(r.q == 0)
    # S = 0: labels are argmin D, flows stay 0
    p = synth.random_potts(4, (4, 6, 8), 3, 6, s_range=(0.0, 0.0), iters=40)
    r = gpu_solve(p, return_q=True)
    assert torch.all(r.q == 0)
    assert np.array_equal(r.labels.cpu().numpy(), np.argmin(p.D, axis=1))
    # equal data terms: stationary uniform labelling
    p = synth.random_potts(5, (4, 6, 8), 3, 4, iters=20)
    p.D[:] = p.D[:, :1]
    r = gpu_solve(p, return_q=True)
    assert float((r.u - 0.25).abs().max()) < 1e-6 and float(r.q.abs().max()) == 0.0
    # every voxel is an exact four-way tie: the export takes the lowest label
    assert torch.all(r.u[:, 1:] == r.u[:, :1]) and torch.all(r.labels == 0)


@pytest.mark.parametrize("kernel", KERNELS)
def test_warm_start_continues_exactly(kernel):
    p = synth.random_potts(11, (6, 10, 14), 3, 5, s_mode="shared_field", iters=12)
    full = gpu_solve(p, 12, kernel=kernel, return_q=True)
    first = gpu_solve(p, 7, kernel=kernel, return_q=True)
    second = gpu_solve(p, 5, kernel=kernel, return_q=True, warm_start=True,
                       workspace=first.workspace)
    assert torch.equal(full.u, second.u) and torch.equal(full.q, second.q)


@pytest.mark.parametrize("kernel", KERNELS)
def test_deterministic(kernel):
    p = synth.dagmf_blobs(shape=(10, 20, 24), iters=15)
    a = gpu_solve(p, kernel=kernel, return_q=True)
    b = gpu_solve(p, kernel=kernel, return_q=True)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q)
    assert a.energy == b.energy and a.dual == b.dual


def test_gap_history_and_tolerance_stop():
    p = synth.potts2d_rects()
    ref = oracle_solve(p, 60, history=True)
    r = gpu_solve(p, 60, gap_every=10, gap_history_cap=16)
    assert len(r.gap_history) == 6
    for k, g in enumerate(r.gap_history):
        i = 10 * (k + 1) - 1
        g_ref = ref["E"][i] - ref["P"][i]
        assert abs(g - g_ref) <= 1e-4 * abs(ref["E"][i]), (k, g, g_ref)
        assert g >= -1e-6 * abs(ref["E"][i])
    assert all(b <= a + 1e-6 * abs(ref["E"][-1]) for a, b in zip(r.gap_history, r.gap_history[1:]))
    # stop at a relative gap of 2e-3 (reached after 30 iterations, well clear
    # of the threshold at the evaluations before and after)
    rel = [(e - q) / e for e, q in zip(ref["E"], ref["P"])]
    first = next(i for i in range(9, 60, 10) if rel[i] <= 2e-3)
    r = gpu_solve(p, 60, gap_every=10, gap_tol=2e-3)
    assert r.iters_done == first + 1


def test_feasibility_reported():
    p = synth.hmf_ellipsoids(shape=(12, 20, 24), iters=40)
    r = gpu_solve(p)
    assert r.max_simplex_err < 1e-5
    assert r.max_flow_excess <= 1e-6
    assert r.gap >= -1e-6 * abs(r.energy)


def test_nonfinite_inputs_rejected():
    p = synth.random_potts(12, (3, 5, 7), 3, 3, s_mode="shared_field", iters=3)
    p.D[0, 1, 1, 2, 3] = np.nan
    with pytest.raises(pf.PseudoflowError) as e:
        gpu_solve(p, check_inputs=True)
    assert e.value.code == pf.PF_ENONFINITE
    p = synth.random_potts(13, (3, 5, 7), 3, 3, s_mode="shared_field", iters=3)
    p.S[0, 0, 0, 0] = -1.0
    with pytest.raises(pf.PseudoflowError) as e:
        gpu_solve(p, check_inputs=True)
    assert e.value.code == pf.PF_ENONFINITE


@pytest.mark.parametrize("storage", ["bf16", "fp16"])
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", ["potts3d_voronoi_36x40x44", "hmf_ellipsoids_20x36x44",
                                  "dagmf_blobs_18x30x38", "ishikawa_levels_20x36x44_n7"])
def test_low_precision_storage_energy(name, kernel, storage):
    """Flow and label state stored in 16 bits, float32 arithmetic: the energy
    stays within 1e-3 relative of the float64 reference."""
    p = WORKLOADS[name]()
    ref = oracle_solve(p)
    E, P = oracle_energy_dual(p, ref["u"], ref["q"])
    r = gpu_solve(p, kernel=kernel, storage=storage)
    rel = abs(r.energy - E) / abs(E)
    n_bad, n_dec = compare_labels(ref["u"].numpy(), r.labels.cpu().numpy())
    print(f"[storage] {name} {storage} {kernel}: rel energy err {rel:.2e}, "
          f"label mismatches {n_bad} ({n_dec} decisive) of {r.labels.numel()}", flush=True)
    assert rel <= 1e-3
    assert r.gap >= -1e-3 * abs(r.energy)


@pytest.mark.parametrize("name", ["potts3d_voronoi_36x40x44", "hmf_ellipsoids_20x36x44",
                                  "dagmf_blobs_18x30x38", "diff_batch_3x40x52"])
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_fused_equals_two_pass_bitwise(name, storage):
    """The fused single pass evaluates the two-pass expressions in the same
    order, so the states agree bit for bit."""
    p = WORKLOADS[name]()
    a = gpu_solve(p, 40, kernel="two_pass", storage=storage, return_q=True)
    b = gpu_solve(p, 40, kernel="fused", storage=storage, return_q=True)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and torch.equal(a.labels, b.labels)
    assert a.energy == b.energy and a.dual == b.dual


FLOW_LABEL_CASES = {
    "hmf_ellipsoids_20x36x44": (lambda: WORKLOADS["hmf_ellipsoids_20x36x44"](), 0),
    "dagmf_blobs_18x30x38_gap7": (lambda: WORKLOADS["dagmf_blobs_18x30x38"](), 7),
    "ishikawa_levels_20x36x44_n7": (lambda: WORKLOADS["ishikawa_levels_20x36x44_n7"](), 0),
    # chains in the chain builds of 4, 8, 12 and 16 labels, with padding labels
    "ishikawa_2_labels": (lambda: synth.ishikawa_levels(shape=(9, 15, 66), n_levels=1), 0),
    "ishikawa_3_labels_gap5": (lambda: synth.ishikawa_levels(shape=(21, 13, 70), n_levels=2), 5),
    "ishikawa_5_labels": (lambda: synth.ishikawa_levels(shape=(19, 17, 40), n_levels=4), 0),
    "ishikawa_12_labels": (lambda: synth.ishikawa_levels(shape=(7, 12, 67), n_levels=11), 0),
    "ishikawa_16_labels": (lambda: synth.ishikawa_levels(shape=(6, 9, 40), n_levels=15), 0),
    "dag_nl16_nn16_B2_field": (lambda: synth.random_problem(
        37, (9, 14, 70), 3, synth.random_dag(np.random.default_rng(37), 0, 16), batch=2,
        s_mode="node_field"), 0),
    "tree_nl2_nn3_shared_gap3": (lambda: synth.random_problem(
        38, (5, 7, 133), 3, synth.random_tree(np.random.default_rng(38), 1, 2),
        s_mode="shared_field", kind="hmf"), 3),
    "dagmf_blobs_40x70x130_chunks": (lambda: synth.dagmf_blobs(shape=(40, 70, 130)), 0),
    # graphs that fill every slot of a build with identity slots (the exact forms)
    "dag_nl4_nn8_B2_exact": (lambda: synth.random_problem(
        39, (11, 17, 75), 3, synth.random_dag(np.random.default_rng(39), 4, 4), batch=2,
        s_mode="node_field"), 5),
    "dag_nl8_nn12_exact": (lambda: synth.random_problem(
        40, (19, 9, 66), 3, synth.random_dag(np.random.default_rng(40), 4, 8),
        s_mode="shared_field"), 0),
}


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name", list(FLOW_LABEL_CASES))
def test_graph_fused_equals_two_pass_bitwise(name, storage):
    """3-D label graphs under the fused kernel run the flow step of one
    iteration and the label step of the next in one pass (entered with a
    label pass, left with a flow pass around every gap check): each voxel
    evaluates the two-pass expressions in the same order, so the states,
    energies and duals agree bit for bit (several z chunks, ragged tiles,
    batches, every capacity mode, odd iteration counts and gap checks)."""
    make, gap_every = FLOW_LABEL_CASES[name]
    p = make()
    iters = 23
    print(f"[flow-label] {name} {storage} gap_every={gap_every}", flush=True)
    a = gpu_solve(p, iters, kernel="two_pass", storage=storage, return_q=True, gap_every=gap_every,
                  gap_history_cap=8)
    b = gpu_solve(p, iters, kernel="fused", storage=storage, return_q=True, gap_every=gap_every,
                  gap_history_cap=8)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and torch.equal(a.labels, b.labels)
    assert a.energy == b.energy and a.dual == b.dual and a.gap_history == b.gap_history


LDS_CASES = {
    "potts2d_rects_64x64": lambda: WORKLOADS["potts2d_rects_64x64"](),
    "potts2d_nl5_B3_nodefield": lambda: synth.random_potts(31, (1, 37, 70), 2, 5, batch=3,
                                                           s_mode="node_field"),
    "dag2d_B2_shared": lambda: synth.random_problem(32, (1, 26, 37), 2,
                                                    synth.random_dag(np.random.default_rng(32), 3, 5),
                                                    batch=2, s_mode="shared_field"),
    "ishikawa_levels_48x61": lambda: WORKLOADS["ishikawa_levels_48x61"](),
    "diff_batch_3x40x52": lambda: WORKLOADS["diff_batch_3x40x52"](),
    "potts2d_one_row": lambda: synth.random_potts(33, (1, 1, 1000), 2, 3, s_mode="node_scalar"),
    "potts2d_B40_shared": lambda: synth.random_potts(34, (1, 33, 47), 2, 4, batch=40,
                                                     s_mode="shared_field"),
    # the label-graph builds of 9..12 and 13..16 flows
    "tree2d_nn11_B3": lambda: synth.random_problem(35, (1, 20, 30), 2,
                                                   synth.random_tree(np.random.default_rng(35), 3, 8),
                                                   batch=3, s_mode="node_field", kind="hmf"),
    "dag2d_nn15_B2": lambda: synth.random_problem(36, (1, 24, 40), 2,
                                                  synth.random_dag(np.random.default_rng(36), 7, 8),
                                                  batch=2, s_mode="node_scalar"),
    # tiles with ghost zones: 16 x 16 owned tiles with ragged edges, 8 x 8
    # owned tiles over a batch of 7, and a label graph over 16 x 16 tiles
    "potts2d_nl3_150x200_tiles": lambda: synth.random_potts(37, (1, 150, 200), 2, 3,
                                                            s_mode="node_field"),
    "potts2d_nl8_B7_shared": lambda: synth.random_potts(38, (1, 45, 38), 2, 8, batch=7,
                                                        s_mode="shared_field"),
    "dag2d_nn8_B3_70x90": lambda: synth.random_problem(39, (1, 70, 90), 2,
                                                       synth.random_dag(np.random.default_rng(39), 3, 5),
                                                       batch=3, s_mode="node_field"),
}


def test_lds_batch_of_256_images_equals_two_pass():
    """The benchmark's batch: 256 copies of the 64 x 64 workload, 200
    iterations, the LDS-resident solve AUTO takes against the two-pass
    kernels, bit for bit."""
    p = synth.potts2d_rects()
    D = torch.from_numpy(np.ascontiguousarray(np.repeat(p.D, 256, axis=0))).cuda()
    assert pf.auto_kernel((256,) + tuple(p.shape[1:]), 3, 3, 2) == "lds"
    kw = dict(c=p.c, tau=p.tau, iters=p.iters, ndim=2, s_mode=p.s_mode, return_q=True)
    a = pf.solve_potts(D, p.S, kernel="two_pass", **kw)
    b = pf.solve_potts(D, p.S, **kw)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and a.energy == b.energy
    assert torch.equal(b.u[0], b.u[255])          # identical problems, identical answers


def test_lds_warm_start_continues_exactly():
    """23 iterations in one LDS-resident solve equal 10 then 13 more from the
    state the first call left in the workspace."""
    p = LDS_CASES["potts2d_nl5_B3_nodefield"]()
    full = gpu_solve(p, 23, kernel="lds", return_q=True)
    first = gpu_solve(p, 10, kernel="lds", return_q=True)
    second = gpu_solve(p, 13, kernel="lds", return_q=True, warm_start=True, workspace=first.workspace)
    assert torch.equal(full.u, second.u) and torch.equal(full.q, second.q)


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name", list(LDS_CASES))
def test_lds_equals_two_pass_bitwise(name, storage):
    """The LDS-resident 2-D solve keeps each value as the storage type holds
    it and evaluates the two-pass expressions, so the states agree bit for
    bit; with gap checks every 7 iterations it runs one launch per chunk."""
    p = LDS_CASES[name]()
    for iters, gap_every in ((23, 0), (30, 7)):
        print(f"[lds] {name} {storage} iters={iters} gap_every={gap_every}", flush=True)
        a = gpu_solve(p, iters, kernel="two_pass", storage=storage, return_q=True, gap_every=gap_every)
        b = gpu_solve(p, iters, kernel="lds", storage=storage, return_q=True, gap_every=gap_every)
        assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and torch.equal(a.labels, b.labels)
        assert a.energy == b.energy and a.dual == b.dual and a.iters_done == b.iters_done


FUSED2_CASES = {
    "potts3d_voronoi_36x40x44": lambda: WORKLOADS["potts3d_voronoi_36x40x44"](),
    "potts3d_nl3_B2_nodefield": lambda: synth.random_potts(21, (37, 19, 131), 3, 3, batch=2,
                                                           s_mode="node_field"),
    "potts3d_nl5_shared": lambda: synth.random_potts(22, (33, 17, 70), 3, 5, s_mode="shared_field"),
    "potts3d_nl8_thin": lambda: synth.random_potts(23, (2, 9, 65), 3, 8, s_mode="node_scalar"),
}


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name", list(FUSED2_CASES))
def test_fused2_equals_fused_bitwise(name, storage):
    """Two iterations per pass evaluate each point's expressions of the
    one-iteration kernels, with the intermediate state rounded where those
    store it, so the states agree bit for bit; with an odd count and gap
    checks every 5 iterations, one-iteration passes mix in."""
    p = FUSED2_CASES[name]()
    for iters, gap_every in ((40, 0), (23, 5)):
        print(f"[fused2] {name} {storage} iters={iters} gap_every={gap_every}", flush=True)
        a = gpu_solve(p, iters, kernel="fused", storage=storage, return_q=True, gap_every=gap_every)
        b = gpu_solve(p, iters, kernel="fused2", storage=storage, return_q=True, gap_every=gap_every)
        assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and torch.equal(a.labels, b.labels)
        assert a.energy == b.energy and a.dual == b.dual
        assert a.iters_done == b.iters_done == iters


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_fused2_full_size_equals_fused(storage):
    """At the full 256^3 Potts workload in the benchmark's launch
    configuration: six iterations as three two-iteration passes equal six
    one-iteration passes bit for bit."""
    p = synth.potts3d_voronoi(n=256, iters=6)
    D, S = torch.from_numpy(p.D).cuda(), torch.from_numpy(p.S).cuda()
    kw = dict(c=p.c, tau=p.tau, iters=6, ndim=3, s_mode="shared_field", storage=storage,
              return_q=True, final_energy=True)
    a = pf.solve_potts(D, S, kernel="fused", **kw)
    b = pf.solve_potts(D, S, kernel="fused2", **kw)
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q)
    assert a.energy == b.energy and a.dual == b.dual


def _solve_direct(p, iters, **kw):
    """The C entry point of p's model, without the skip table of gpu_solve."""
    D, S = device_inputs(p)
    args = dict(c=p.c, tau=p.tau, iters=iters, ndim=p.ndim, s_mode=p.s_mode, **kw)
    if p.kind == "potts":
        return pf.solve_potts(D, S, **args)
    if p.kind == "ishikawa":
        return pf.solve_ishikawa(D, S, **args)
    if p.kind == "hmf":
        return pf.solve_hmf(D, S, p.graph, **args)
    return pf.solve_dagmf(D, S, p.graph, **args)


def test_unsupported_kernels_are_rejected():
    """Every documented PF_EUNSUPPORTED case returns that code through the
    C ABI (and leaves nothing half-done): two iterations per pass outside 3-D
    Potts up to 8 labels, the fused pass for the 2-D Ishikawa chain or beyond
    16 flows, the LDS-resident solve for 3-D problems or more than 8 labels."""
    deep = synth.random_problem(201, (3, 5, 6), 3, synth.random_dag(np.random.default_rng(7), 15, 16,
                                                                    max_parents=2))
    cases = ((synth.random_potts(1, (1, 9, 11), 2, 4), "fused2", "2-D"),
             (synth.random_potts(2, (3, 5, 7), 3, 12), "fused2", "12 labels"),
             (synth.hmf_ellipsoids(shape=(4, 6, 8), iters=2), "fused2", "label graph"),
             (synth.ishikawa_levels(shape=(1, 9, 10), iters=2), "fused", "Ishikawa chain"),
             (synth.ishikawa_levels(shape=(1, 9, 10), iters=2), "fused2", "Ishikawa chain"),
             (deep, "fused", "30 flows"),
             (synth.random_potts(3, (3, 5, 7), 3, 3), "lds", "3-D"),
             (synth.random_potts(5, (1, 30, 30), 2, 12), "lds", "12 labels"))
    for p, kernel, why in cases:
        assert kernel not in supported_kernels(p), why
        with pytest.raises(pf.PseudoflowError) as ei:
            _solve_direct(p, 2, kernel=kernel)
        assert ei.value.code == pf.PF_EUNSUPPORTED, why


def test_largest_admitted_grid_two_iterations():
    """The largest grid the library admits per problem, 1022 x 1024 x 1024
    voxels (the voxel byte offsets reach 4.29e9, just below 2^32), 3-D Potts
    with 2 labels and float32 state under AUTO (two iterations per pass):
    after two iterations from the initial state, u and q at sampled voxels
    (the last voxel and the corners included) match the float64 reference
    run on 9^3 patches of the same inputs (exact there: two iterations reach
    three voxels)."""
    Z, Y, X = 1022, 1024, 1024
    free, _ = torch.cuda.mem_get_info()
    if free < 150e9:
        pytest.skip(f"needs about 120 GB of device memory ({free / 1e9:.0f} GB free)")
    assert pf.auto_kernel((1, Z, Y, X), 2, 2, 3) == "fused2"
    g = torch.Generator(device="cuda").manual_seed(5)
    D = torch.rand((1, 2, Z, Y, X), generator=g, device="cuda", dtype=torch.float32)
    S = np.array([0.3, 0.25], np.float32)
    c, tau = 1.0, 0.125
    print(f"[max grid] {Z}x{Y}x{X}, 2 labels", flush=True)
    r = pf.solve_potts(D, S, c=c, tau=tau, iters=2, ndim=3, return_q=True, final_energy=False)
    rng = np.random.default_rng(97)
    pts = [(int(rng.integers(0, Z)), int(rng.integers(0, Y)), int(rng.integers(0, X))) for _ in range(12)]
    pts += [(0, 0, 0), (Z - 1, Y - 1, X - 1), (Z - 1, 0, X - 1), (0, Y - 1, 0), (Z // 2, Y - 1, X - 1)]
    worst_u = worst_q = 0.0
    for (z, y, x) in pts:
        (z0, z1), (y0, y1), (x0, x1) = (_patch_bounds(z, Z, 9), _patch_bounds(y, Y, 9),
                                        _patch_bounds(x, X, 9))
        Dp = D[:, :, z0:z1, y0:y1, x0:x1].double().cpu()
        ref = O.solve_potts(Dp, S.astype(np.float64), "node_scalar", c, tau, 2, 3, history=False)
        cz, cy, cx = z - z0, y - y0, x - x0
        u_gpu = r.u[0, :, z, y, x].double().cpu()
        q_gpu = r.q[0, :, :, z, y, x].double().cpu()
        worst_u = max(worst_u, float((ref["u"][0, :, cz, cy, cx] - u_gpu).abs().max()))
        worst_q = max(worst_q, float((ref["q"][0, :, :, cz, cy, cx] - q_gpu).abs().max()))
    print(f"[max grid] max|du| {worst_u:.2e}, max|dq| {worst_q:.2e}", flush=True)
    del D, r
    torch.cuda.empty_cache()
    assert worst_u <= 1e-5 and worst_q <= 1e-5


def _patch_bounds(x, n, w=5):
    lo = min(max(x - w // 2, 0), max(n - w, 0))
    return lo, min(lo + w, n)


@pytest.mark.parametrize("kernel", ["fused", "two_pass"])
def test_full_size_sampled_one_step(kernel):
    """At the full 256^3 Potts workload, in the launch configuration the
    benchmark times: the state after k iterations, advanced by one more
    iteration on the GPU, matches the float64 one-iteration map applied to 5^3
    patches around sampled voxels (exact there: a patch edge that is not the
    volume edge lies two voxels from the sample).  Also checks feasibility and
    weak duality of the full-size state."""
    p = synth.potts3d_voronoi(n=256, iters=20)
    D, S = torch.from_numpy(p.D).cuda(), torch.from_numpy(p.S).cuda()
    kw = dict(c=p.c, tau=p.tau, ndim=3, s_mode="shared_field", kernel=kernel, return_q=True)
    r0 = pf.solve_potts(D, S, iters=20, final_energy=True, **kw)
    assert r0.max_simplex_err < 1e-5 and r0.max_flow_excess <= 1e-6
    assert r0.gap >= -1e-7 * abs(r0.energy)
    u0, q0 = r0.u.clone(), r0.q.clone()
    r1 = pf.solve_potts(D, S, iters=1, warm_start=True, workspace=r0.workspace,
                        final_energy=False, **kw)
    n = 256
    rng = np.random.default_rng(99)
    pts = [tuple(rng.integers(0, n, size=3)) for _ in range(40)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 17), (n - 1, 5, 0), (128, 0, n - 1)]
    worst_u = worst_q = 0.0
    for (z, y, x) in pts:
        (z0, z1), (y0, y1), (x0, x1) = (_patch_bounds(z, n), _patch_bounds(y, n),
                                        _patch_bounds(x, n))
        sl = (slice(None), slice(None), slice(z0, z1), slice(y0, y1), slice(x0, x1))
        u = u0[sl].double().cpu()
        q = q0[:, :, :, z0:z1, y0:y1, x0:x1].double().cpu()
        Dp = torch.tensor(p.D[sl], dtype=torch.float64)
        Sp = torch.tensor(p.S[:, z0:z1, y0:y1, x0:x1], dtype=torch.float64).unsqueeze(1)
        ell = torch.log(u)
        ell1, q1, _ = O.potts_iteration(ell, q, Dp, Sp, p.c, p.tau, 3)
        cz, cy, cx = z - z0, y - y0, x - x0
        u_ref = torch.exp(ell1[0, :, cz, cy, cx])
        u_gpu = r1.u[0, :, z, y, x].double().cpu()
        q_ref = q1[0, :, :, cz, cy, cx]
        q_gpu = r1.q[0, :, :, z, y, x].double().cpu()
        worst_u = max(worst_u, float((u_ref - u_gpu).abs().max()))
        worst_q = max(worst_q, float((q_ref - q_gpu).abs().max()))
    print(f"[full-size one-step] {kernel}: max|du| {worst_u:.2e}, max|dq| {worst_q:.2e}", flush=True)
    assert worst_u <= 1e-5 and worst_q <= 1e-5


def test_full_size_dagmf_auto_equals_two_pass_bitwise():
    """The benchmark's workload and launch configuration (DAGMF 256x512x512,
    AUTO: the flow-then-label pass in its exact build) against the two-pass
    kernels (checked against the reference at this size by the sampled
    one-step test below), 5 iterations from the initial state, in fp32 and
    bf16 state: every output and the energies bit for bit."""
    p = synth.dagmf_blobs(iters=5)
    D = torch.from_numpy(p.D).cuda()
    for storage in ("fp32", "bf16"):
        assert pf.auto_kernel(p.shape, p.n_leaf, p.n_node, 3, storage, identity=False) == "fused"
        kw = dict(c=p.c, tau=p.tau, iters=p.iters, ndim=3, s_mode=p.s_mode, storage=storage,
                  return_q=True)
        print(f"[full-size auto] dagmf 256x512x512 {storage}", flush=True)
        a = pf.solve_dagmf(D, p.S, p.graph, kernel="two_pass", **kw)
        ua, qa, la, ea = a.u.clone(), a.q.clone(), a.labels.clone(), (a.energy, a.dual)
        del a
        torch.cuda.empty_cache()
        b = pf.solve_dagmf(D, p.S, p.graph, **kw)
        assert torch.equal(ua, b.u) and torch.equal(qa, b.q) and torch.equal(la, b.labels)
        assert ea == (b.energy, b.dual)
        del ua, qa, la, b
        torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["hmf", "dagmf"])
def test_full_size_graph_sampled_one_step(name, storage):
    """At the full HMF (128x256x256, 3 -> 8 tree) and DAGMF (256x512x512,
    4 parents x 12 leaves) workloads, in the launch configuration the
    benchmark times (AUTO kernel choice): the state after a few iterations,
    advanced by one more iteration on the GPU, matches the float64 iteration
    of Algorithm 2 applied to 5^3 patches around sampled voxels, from the
    same stored state.  float32: within 1e-5.  bf16 state: the GPU rounds
    its outputs to bf16 (log-labels: 2^-8 of the value), and its flow step
    reads the new labels after that rounding: |du_L| <= u_L |ln u_L| 2^-9,
    so |dU_A| <= (sum_L u_L |ln u_L|) 2^-9 <= ln(n_leaf) 2^-9 at a voxel and
    the 1-Lipschitz projection moves the flow by at most
    c tau 2 sqrt(3) ln(n_leaf) 2^-9, plus its own rounding 2^-8 |q|."""
    p = synth.hmf_ellipsoids(iters=4) if name == "hmf" else synth.dagmf_blobs(iters=3)
    solve = pf.solve_hmf if name == "hmf" else pf.solve_dagmf
    D = torch.from_numpy(p.D).cuda()
    kw = dict(c=p.c, tau=p.tau, ndim=3, s_mode=p.s_mode, storage=storage, return_q=True)
    r0 = solve(D, p.S, p.graph, iters=p.iters, final_energy=True, **kw)
    assert r0.max_simplex_err < (1e-5 if storage == "fp32" else 2e-2)
    assert r0.gap >= -1e-6 * abs(r0.energy)
    u0, q0 = r0.u, r0.q
    r1 = solve(D, p.S, p.graph, iters=1, warm_start=True, workspace=r0.workspace,
               final_energy=False, **kw)
    g = O.OracleGraph(p.graph.n_nodes, p.graph.parent, p.graph.child, p.graph.weight)
    _, Z, Y, X = p.shape
    Sx = O.expand_S(p.S, p.s_mode, 1, g.n_node, 1, 1, 1)
    rng = np.random.default_rng(98)
    pts = [(int(rng.integers(0, Z)), int(rng.integers(0, Y)), int(rng.integers(0, X))) for _ in range(24)]
    pts += [(0, 0, 0), (Z - 1, Y - 1, X - 1), (0, Y - 1, 17), (Z - 1, 5, 0)]
    bf = storage != "fp32"
    worst_l = worst_q = 0.0
    for (z, y, x) in pts:
        (z0, z1), (y0, y1), (x0, x1) = (_patch_bounds(z, Z), _patch_bounds(y, Y),
                                        _patch_bounds(x, X))
        sl = (slice(None), slice(None), slice(z0, z1), slice(y0, y1), slice(x0, x1))
        ell = torch.log(u0[sl].double().cpu())
        q = q0[:, :, :, z0:z1, y0:y1, x0:x1].double().cpu()
        Dp = torch.tensor(p.D[sl], dtype=torch.float64)
        ell1, q1, _ = O.dag_iteration(ell, q, Dp, Sx, g, p.c, p.tau, 3)
        cz, cy, cx = z - z0, y - y0, x - x0
        l_ref = ell1[0, :, cz, cy, cx]
        l_gpu = torch.log(r1.u[0, :, z, y, x].double().cpu())
        q_ref = q1[0, :, :, cz, cy, cx]
        q_gpu = r1.q[0, :, :, z, y, x].double().cpu()
        tol_l = (l_ref.abs() * 2.0 ** -8 if bf else 0.0) + 1e-5
        tol_q = ((q_ref.abs() * 2.0 ** -8 + p.c * p.tau * 2 * 3 ** 0.5 * np.log(p.n_leaf) * 2.0 ** -9)
                 if bf else 0.0) + 1e-5
        worst_l = max(worst_l, float(((l_ref - l_gpu).abs() / tol_l).max()))
        worst_q = max(worst_q, float(((q_ref - q_gpu).abs() / tol_q).max()))
    print(f"[full-size one-step] {name} {storage}: max err / tol: ell {worst_l:.3f}, "
          f"q {worst_q:.3f}", flush=True)
    assert worst_l <= 1.0 and worst_q <= 1.0
