"""The static-scratch DAGMF solve (solve_dagmf_static, for callers that cannot
allocate device memory) against solve_dagmf with a caller workspace: the same
kernels run on the same inputs, so the results agree bit for bit.  Two calls
in a row with the second smaller, warm starts from the static scratch, the
LDS-resident kernels on a batch of 2-D problems and in tiles on one, AUTO's
fall-back to the single-state kernels where two state copies do not fit, the
size limit and the argument checks, all through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1501_07844_amd as pf
from paper_1501_07844_amd import synth

from parity_util import device_inputs

pytestmark = pytest.mark.gpu


def _both(p, iters, **kw):
    D, S = device_inputs(p)
    args = dict(c=p.c, tau=p.tau, iters=iters, ndim=p.ndim, s_mode=p.s_mode, return_q=True)
    args.update(kw)
    a = pf.solve_dagmf(D, S, p.graph, **args)
    b = pf.solve_dagmf_static(D, S, p.graph, **args)
    return a, b


def _same(a, b):
    assert torch.equal(a.u, b.u) and torch.equal(a.q, b.q) and torch.equal(a.labels, b.labels)
    assert a.energy == b.energy and a.dual == b.dual and a.gap == b.gap
    assert a.gap_history == b.gap_history and a.iters_done == b.iters_done


def test_static_scratch_equals_workspace_solve_on_two_calls():
    # first call: the DAGMF workload's graph (4 parents x 12 leaves) on a
    # 20 x 48 x 70 grid, fp32 state (the flow-then-label pass), gap every 7
    p1 = synth.dagmf_blobs(shape=(20, 48, 70), iters=30)
    print(f"[static] call 1: {p1.shape} dagmf fp32", flush=True)
    a, b = _both(p1, 30, gap_every=7, gap_history_cap=8)
    _same(a, b)
    assert len(b.gap_history) == 4
    # second call, smaller: a tree on 2 x 6 x 17 x 23 voxels, per-node
    # capacity fields, bf16 state (the two-pass kernels)
    tree = synth.random_tree(np.random.default_rng(41), 2, 5)
    p2 = synth.random_problem(41, (6, 17, 23), 3, tree, batch=2, s_mode="node_field", kind="hmf")
    print(f"[static] call 2: {p2.shape} tree bf16", flush=True)
    a, b = _both(p2, 25, storage="bf16")
    _same(a, b)


def test_static_scratch_warm_start_and_lds_batch():
    # a warm start continues from the state the previous call on this GPU left
    p = synth.dagmf_blobs(shape=(8, 20, 30), iters=20)
    D, S = device_inputs(p)
    kw = dict(c=p.c, tau=p.tau, ndim=3, s_mode=p.s_mode, return_q=True)
    full = pf.solve_dagmf(D, S, p.graph, iters=20, **kw)
    pf.solve_dagmf_static(D, S, p.graph, iters=12, **kw)
    rest = pf.solve_dagmf_static(D, S, p.graph, iters=8, warm_start=True, **kw)
    assert torch.equal(full.u, rest.u) and torch.equal(full.q, rest.q)
    # a batch of 16 small 2-D problems: the LDS-resident solve under AUTO
    dag = synth.random_dag(np.random.default_rng(43), 3, 5)
    q = synth.random_problem(43, (1, 24, 31), 2, dag, batch=16, s_mode="shared_field")
    assert pf.auto_kernel(q.shape, q.n_leaf, q.n_node, 2, identity=False) == "lds"
    a, b = _both(q, 17, gap_every=5, gap_history_cap=4)
    _same(a, b)
    # one 2-D problem: LDS tiles with ghost zones (ping-pong state), 21
    # iterations at once against 13 then 8 more from the static scratch
    t = synth.random_problem(44, (1, 40, 52), 2, dag, s_mode="node_field")
    assert pf.auto_kernel(t.shape, t.n_leaf, t.n_node, 2, identity=False) == "lds"
    Dt, St = device_inputs(t)
    kt = dict(c=t.c, tau=t.tau, ndim=2, s_mode=t.s_mode, return_q=True)
    full = pf.solve_dagmf(Dt, St, t.graph, iters=21, **kt)
    pf.solve_dagmf_static(Dt, St, t.graph, iters=13, **kt)
    rest = pf.solve_dagmf_static(Dt, St, t.graph, iters=8, warm_start=True, **kt)
    assert torch.equal(full.u, rest.u) and torch.equal(full.q, rest.q)


def test_static_scratch_auto_takes_one_state_copy_where_two_do_not_fit():
    # 32 x 112 x 112 voxels of the DAGMF workload's graph in fp32: the
    # flow-then-label pass (two copies of the state) needs 184 MiB, the
    # two-pass kernels 92 MiB; AUTO on the static scratch runs the latter
    p = synth.dagmf_blobs(shape=(32, 112, 112), iters=10)
    lim = 128 << 20
    assert pf.workspace_bytes(p.shape, 12, 16, 3, kernel="two_pass") <= lim
    assert pf.workspace_bytes(p.shape, 12, 16, 3, kernel="fused") > lim
    D, S = device_inputs(p)
    kw = dict(c=p.c, tau=p.tau, iters=10, ndim=3, s_mode=p.s_mode, return_q=True)
    print(f"[static] {p.shape}: AUTO on the static scratch", flush=True)
    a = pf.solve_dagmf(D, S, p.graph, kernel="two_pass", **kw)
    b = pf.solve_dagmf_static(D, S, p.graph, **kw)
    _same(a, b)
    with pytest.raises(pf.PseudoflowError) as ei:
        pf.solve_dagmf_static(D, S, p.graph, kernel="fused", **kw)
    assert ei.value.code == pf.PF_ENOMEM


def _raw_params(**kw):
    p = pf._Params()
    p.iters, p.c, p.tau = 3, 2.0, 0.1
    p.final_energy = 1
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_static_scratch_limits_and_argument_checks():
    lib = pf.library()
    # a problem that needs more than the static scratch: PF_ENOMEM, no work
    big = synth.dagmf_blobs(shape=(64, 128, 128), iters=3)
    D, _ = device_inputs(big)
    keep = []
    g = pf._graph_struct(big.graph, keep)
    S = np.ascontiguousarray(np.asarray(big.S, np.float32))
    grid = pf._Grid(1, 3, 64, 128, 128)
    r = pf._Result()
    st = lib.solve_dagmf_static(C.byref(grid), C.byref(g), C.c_void_p(D.data_ptr()),
                                C.c_void_p(S.ctypes.data), 0, C.byref(_raw_params()), C.byref(r), None)
    msg = lib.pf_last_error().decode()
    print(f"[static] {big.shape}: status {st}, {msg}", flush=True)
    assert st == pf.PF_ENOMEM and "static scratch" in msg
    # a workspace, a tape or launch timing are refused before any work
    small = synth.dagmf_blobs(shape=(4, 8, 8), iters=3)
    D2, _ = device_inputs(small)
    grid2 = pf._Grid(1, 3, 4, 8, 8)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    for kw, code in ((dict(workspace=ws.data_ptr(), workspace_bytes=ws.numel()), pf.PF_EINVAL),
                     (dict(workspace_bytes=4096), pf.PF_EINVAL),
                     (dict(timing_stride=1), pf.PF_EUNSUPPORTED),
                     (dict(tape=ws.data_ptr(), tape_bytes=ws.numel(), ckpt_every=1), pf.PF_EUNSUPPORTED)):
        st = lib.solve_dagmf_static(C.byref(grid2), C.byref(g), C.c_void_p(D2.data_ptr()),
                                    C.c_void_p(S.ctypes.data), 0, C.byref(_raw_params(**kw)),
                                    C.byref(pf._Result()), None)
        assert st == code, (kw, st, lib.pf_last_error().decode())
    # the same small problem runs (the graph struct is reused: same graph)
    st = lib.solve_dagmf_static(C.byref(grid2), C.byref(g), C.c_void_p(D2.data_ptr()),
                                C.c_void_p(S.ctypes.data), 0, C.byref(_raw_params()),
                                C.byref(pf._Result()), None)
    assert st == pf.PF_OK, lib.pf_last_error().decode()
    torch.cuda.synchronize()
