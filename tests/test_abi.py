"""The C ABI library: it loads without a GPU, exports every symbol the header
declares, sizes workspaces, and rejects bad arguments with the documented
status before any device work (these calls never reach a launch)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1501_07844_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pseudoflow.h")


def _gpu_visible() -> bool:
    import torch
    return torch.cuda.device_count() > 0     # counts devices without initialising HIP


# These calls pass fake device addresses that the validation must reject
# before any launch; they run only where no GPU is visible, so a validation
# bug can never turn into a launch on a real device.
pytestmark = [
    pytest.mark.skipif(not os.path.exists(pf.lib_path()), reason="library not built"),
    pytest.mark.skipif(_gpu_visible(), reason="fake-pointer ABI checks run only without a GPU"),
]


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declarations_match_binding_list():
    assert _declared() == sorted(pf.EXPORTED)


def test_every_declared_symbol_is_exported():
    lib = pf.library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.pf_abi_version() == pf.ABI_VERSION == 3


def _grid(B=1, nd=3, Z=8, Y=9, X=10):
    return pf._Grid(B, nd, Z, Y, X)


def _params(**kw):
    p = pf._Params()
    p.iters, p.c, p.tau = 5, 1.0, 0.1
    p.workspace = 256 * 1024          # fake, aligned: never dereferenced by these calls
    p.workspace_bytes = 1 << 40
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_auto_kernel_choice():
    """The kernel AUTO resolves to: the LDS-resident solve for batches of 8
    or more 2-D problems of at most 4096 voxels, 8 leaves and 16 flows whose
    float32 state (n_leaf + 2 n_node floats per voxel) fits in 160 KB;
    two iterations per pass for 3-D Potts up to 8 labels in every storage
    type, the one-iteration fused pass beyond with float32 state, the
    two-pass kernels for 16-bit state beyond 8 labels and larger 2-D
    problems; the fused pass (flow step, then the next label step) for 3-D
    label graphs of 9 to 16 flows and at most 16 leaves with fp32 state."""
    k = pf.KERNEL
    assert pf.auto_kernel((1, 256, 256, 256), 8, 8, 3) == "fused2"
    assert pf.auto_kernel((2, 5, 7, 9), 3, 3, 3) == "fused2"
    assert pf.auto_kernel((1, 16, 16, 16), 12, 12, 3) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 8, 8, 3, "bf16") == "fused2"
    assert pf.auto_kernel((1, 16, 16, 16), 8, 8, 3, "fp16") == "fused2"
    assert pf.auto_kernel((1, 16, 16, 16), 12, 12, 3, "bf16") == "two_pass"
    # 2-D: whole problems in LDS for 8 or more that fit, tiles with ghost
    # zones up to 2^21 voxel-fields and 8 flows, two-pass beyond
    assert pf.auto_kernel((1, 1, 64, 64), 8, 8, 2) == "lds"                 # tiles
    assert pf.auto_kernel((8, 1, 64, 64), 3, 3, 2) == "lds"                 # 36864 of 40960 floats
    assert pf.auto_kernel((1, 1, 64, 64), 3, 3, 2) == "lds"                 # a single problem: tiles
    assert pf.auto_kernel((7, 1, 64, 64), 3, 3, 2) == "lds"
    assert pf.auto_kernel((16, 1, 40, 52), 5, 4, 2, identity=False) == "lds"
    assert pf.auto_kernel((8, 1, 64, 64), 4, 4, 2) == "lds"                 # 49152 floats: tiles
    assert pf.auto_kernel((8, 1, 52, 64), 4, 4, 2) == "lds"                 # 39936 floats
    assert pf.auto_kernel((8, 1, 64, 65), 3, 3, 2) == "lds"                 # 4160 voxels: tiles
    assert pf.auto_kernel((1, 1, 512, 682), 3, 3, 2) == "lds"               # just under 2^21 voxel-fields
    assert pf.auto_kernel((1, 1, 512, 683), 3, 3, 2) == "two_pass"          # just above
    assert pf.auto_kernel((64, 1, 64, 64), 5, 5, 2) == "two_pass"           # 2.6e6 voxel-fields
    assert pf.auto_kernel((8, 1, 40, 40), 9, 9, 2) == "two_pass"            # more than 8 labels
    assert pf.auto_kernel((1, 16, 16, 16), 8, 11, 3, identity=False) == "fused"
    assert pf.auto_kernel((1, 256, 512, 512), 12, 16, 3, identity=False) == "fused"
    # graphs that fill a build with identity slots (leaves last, 4 internal
    # nodes and 4-16 leaves, 8 and 8 or 12, 3 and 8): the pass in every storage type
    assert pf.auto_kernel((1, 256, 512, 512), 12, 16, 3, "bf16", identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 4, 8, 3, "fp16", identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 4, 8, 3, "fp32", identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 8, 16, 3, "bf16", identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 8, 11, 3, "bf16", identity=False) == "fused"      # HMF tree
    assert pf.auto_kernel((1, 16, 16, 16), 7, 10, 3, "bf16", identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 10, 14, 3, "bf16", identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 16, 16, 3, "fp16", identity=False) == "two_pass"
    # Ishikawa chains (n_node = n_leaf - 1): fp32 unless 3 padding labels in the build
    assert pf.auto_kernel((1, 16, 16, 16), 8, 7, 3, identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 10, 9, 3, identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 5, 4, 3, identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 13, 12, 3, identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 8, 7, 3, "bf16", identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 3, 2, 3, "fp16", identity=False) == "fused"
    assert pf.auto_kernel((1, 1, 64, 64), 8, 7, 2, identity=False) == "lds"
    assert pf.auto_kernel((1, 16, 16, 16), 4, 6, 3, identity=False) == "fused"      # fp32 DAG, 6 flows
    assert pf.auto_kernel((1, 16, 16, 16), 2, 3, 3, identity=False) == "fused"
    assert pf.auto_kernel((1, 16, 16, 16), 4, 6, 3, "bf16", identity=False) == "two_pass"
    assert pf.auto_kernel((1, 16, 16, 16), 16, 30, 3, identity=False) == "two_pass"  # 30 flows
    assert pf.auto_kernel((1, 1, 64, 64), 8, 11, 2, identity=False) == "two_pass"   # 2-D, 11 flows
    assert pf.auto_kernel((1, 1, 64, 64), 5, 8, 2, identity=False) == "lds"         # 2-D, 8 flows
    lib = pf.library()
    assert lib.pf_auto_kernel(C.byref(_grid()), 4, 5, 1, 0) == -1          # Potts needs n_node == n_leaf
    assert lib.pf_auto_kernel(C.byref(_grid()), 4, 4, 1, 9) == -1          # storage
    assert lib.pf_auto_kernel(None, 4, 4, 1, 0) == -1
    assert lib.pf_auto_kernel(C.byref(_grid()), 4, 4, 1, 0) == k["fused2"]
    with pytest.raises(ValueError):
        pf.auto_kernel((1, 4, 4, 4), 17, 17, 3)


def test_workspace_bytes_accounting():
    lib = pf.library()
    g = _grid(2, 3, 8, 9, 10)
    V = 8 * 9 * 10
    for storage, s in ((0, 4), (1, 2), (2, 2)):
        p = _params(storage=storage, kernel=pf.KERNEL["two_pass"])
        n = lib.pf_workspace_bytes(C.byref(g), 4, 6, C.byref(p))
        state = 2 * (4 + 6 * 3) * V * s
        assert state <= n <= state + 64 * 1024
    assert lib.pf_workspace_bytes(C.byref(_grid(nd=2, Z=3)), 3, 3, C.byref(_params())) == 0
    assert lib.pf_workspace_bytes(C.byref(g), 17, 17, C.byref(_params())) == 0


def test_state_memory_below_paper_buffer_count():
    """The DAGMF buffer count of the paper (five buffers per end-label, four
    per other non-source label, one accumulator; Algorithm 2 discussion) is an
    upper bound for the library's per-voxel state in 3-D."""
    lib = pf.library()
    golden = _golden_buffers()
    for nl, ni in ((8, 3), (12, 4), (3, 0)):
        g = _grid(1, 3, 16, 16, 16)
        p = _params(storage=0, kernel=pf.KERNEL["two_pass"])
        n = lib.pf_workspace_bytes(C.byref(g), nl, nl + ni, C.byref(p))
        fields = (n - 64 * 1024) / (16 ** 3 * 4)
        paper = golden["dagmf_per_end_label"] * nl + golden["dagmf_per_other_label"] * ni \
            + golden["dagmf_extra"]
        assert fields <= paper


def test_ishikawa_state_below_paper_buffer_count():
    """Ishikawa chain (Algorithm 3, discussion after it): 5N + 2 buffers for N
    levels (N + 1 labels, N flows).  The library keeps N + 1 log-labels and
    nd components per flow (d and U live in registers): 3N + 1 in 2-D, 4N + 1
    in 3-D.  With N = 1 the chain is the binary model, whose pseudo-flow form
    the paper counts as 4 buffers: 2 labels + one 2-D flow."""
    lib = pf.library()
    golden = _golden_buffers()
    for nd, (Z, Y, X) in ((2, (1, 256, 256)), (3, (64, 64, 64))):
        V = Z * Y * X                     # large enough that the < 64 KB of
        for N in (1, 2, 4, 8, 15):       # fixed workspace is under one field
            g = _grid(1, nd, Z, Y, X)
            p = _params(storage=0, kernel=pf.KERNEL["two_pass"])
            n = lib.pf_workspace_bytes(C.byref(g), N + 1, N, C.byref(p))
            fields = n // (V * 4)
            assert fields == (N + 1) + nd * N
            assert fields <= golden["ishikawa_per_level"] * N + golden["ishikawa_extra"]
            if N == 1 and nd == 2:
                assert fields == golden["binary_pseudoflow"]


def _golden_buffers():
    path = os.path.join(ROOT, "tests", "golden", "buffer_counts.txt")
    out = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            out[k.strip()] = int(v)
    return out


def _call_potts(g, n, D, S, mode, p, r=None):
    lib = pf.library()
    r = r or pf._Result()
    return lib.solve_potts(C.byref(g) if g is not None else None, n, C.c_void_p(D),
                           C.c_void_p(S), mode, C.byref(p) if p is not None else None,
                           C.byref(r), None)


S3 = (C.c_float * 3)(0.5, 0.5, 0.5)
SADDR = C.addressof(S3)
DEV = 1 << 20          # fake aligned pointers


@pytest.mark.parametrize("case,code", [
    ("null_grid", pf.PF_EINVAL), ("ndim4", pf.PF_EINVAL), ("nz_2d", pf.PF_EINVAL),
    ("zero_dim", pf.PF_EINVAL), ("neg_iters", pf.PF_EINVAL), ("c0", pf.PF_EINVAL),
    ("tau_neg", pf.PF_EINVAL), ("null_D", pf.PF_EINVAL), ("misaligned_D", pf.PF_EINVAL),
    ("null_ws", pf.PF_EINVAL), ("misaligned_ws", pf.PF_EINVAL), ("small_ws", pf.PF_ENOMEM),
    ("too_many_labels", pf.PF_EUNSUPPORTED), ("bad_storage", pf.PF_EINVAL),
    ("neg_S", pf.PF_EINVAL), ("nan_S", pf.PF_ENONFINITE), ("bad_smode", pf.PF_EINVAL),
    ("null_params", pf.PF_EINVAL), ("bad_kernel", pf.PF_EINVAL),
    ("fused2_2d", pf.PF_EUNSUPPORTED), ("fused2_9_labels", pf.PF_EUNSUPPORTED),
    ("fused2_recorded", pf.PF_EUNSUPPORTED), ("too_many_voxels", pf.PF_EUNSUPPORTED),
    ("lds_3d", pf.PF_EUNSUPPORTED), ("lds_9_labels", pf.PF_EUNSUPPORTED),
    ("lds_recorded", pf.PF_EUNSUPPORTED),
])
def test_potts_argument_errors(case, code):
    g, n, D, S, mode, p = _grid(), 3, DEV, SADDR, 0, _params()
    if case == "null_grid":
        g = None
    elif case == "ndim4":
        g.ndim = 4
    elif case == "nz_2d":
        g.ndim = 2
    elif case == "zero_dim":
        g.ny = 0
    elif case == "neg_iters":
        p.iters = -1
    elif case == "c0":
        p.c = 0.0
    elif case == "tau_neg":
        p.tau = -1.0
    elif case == "null_D":
        D = 0
    elif case == "misaligned_D":
        D = DEV + 2
    elif case == "null_ws":
        p.workspace = None
    elif case == "misaligned_ws":
        p.workspace = DEV + 64
    elif case == "small_ws":
        p.workspace_bytes = 1024
    elif case == "too_many_labels":
        n = 17
    elif case == "bad_storage":
        p.storage = 7
    elif case == "neg_S":
        keep = (C.c_float * 3)(0.5, -0.1, 0.5)
        S = C.addressof(keep)
    elif case == "nan_S":
        keep = (C.c_float * 3)(0.5, float("nan"), 0.5)
        S = C.addressof(keep)
    elif case == "bad_smode":
        mode = 9
    elif case == "null_params":
        p = None
    elif case == "bad_kernel":
        p.kernel = 5
    elif case == "lds_3d":
        p.kernel = pf.KERNEL["lds"]
    elif case == "lds_9_labels":
        g = _grid(1, 2, 1, 9, 10)
        n = 9
        keep = (C.c_float * 9)(*([0.5] * 9))
        S = C.addressof(keep)
        p.kernel = pf.KERNEL["lds"]
    elif case == "lds_recorded":
        g = _grid(1, 2, 1, 9, 10)
        p.kernel = pf.KERNEL["lds"]
        p.ckpt_every, p.tape, p.tape_bytes = 1, 512 * 1024, 1 << 30
    elif case == "fused2_2d":
        g = _grid(1, 2, 1, 9, 10)
        p.kernel = pf.KERNEL["fused2"]
    elif case == "fused2_9_labels":
        n = 9
        keep = (C.c_float * 9)(*([0.5] * 9))
        S = C.addressof(keep)
        p.kernel = pf.KERNEL["fused2"]
    elif case == "too_many_voxels":
        g = _grid(1, 3, 1023, 1024, 1024)      # 1022 planes of 1024^2 is the largest admitted
    elif case == "fused2_recorded":
        p.kernel = pf.KERNEL["fused2"]
        p.ckpt_every, p.tape, p.tape_bytes = 1, 512 * 1024, 1 << 30
    assert _call_potts(g, n, D, S, mode, p) == code
    assert pf.library().pf_last_error().decode() != ""


def _call_graph(fn, par, chi, w=None, n_nodes=None, S=None):
    lib = pf.library()
    par = np.asarray(par, np.int32)
    chi = np.asarray(chi, np.int32)
    n_nodes = n_nodes if n_nodes is not None else int(max(par.max(), chi.max())) + 1
    gs = pf._Graph(n_nodes, len(par), par.ctypes.data_as(C.POINTER(C.c_int32)),
                   chi.ctypes.data_as(C.POINTER(C.c_int32)), None)
    if w is not None:
        w = np.asarray(w, np.float64)
        gs.weight = w.ctypes.data_as(C.POINTER(C.c_double))
    Sv = (C.c_float * 32)(*([0.5] * 32))
    r = pf._Result()
    return getattr(lib, fn)(C.byref(_grid()), C.byref(gs), C.c_void_p(DEV), C.c_void_p(C.addressof(Sv)),
                            0, C.byref(_params()), C.byref(r), None)


@pytest.mark.parametrize("case", ["cycle", "orphan", "self", "dup", "weights", "into_source",
                                  "out_of_range", "zero_weight"])
def test_graph_errors(case):
    if case == "cycle":
        args = ([0, 1, 2, 3], [1, 2, 3, 1])
    elif case == "orphan":
        args = ([0, 0, 3], [1, 2, 4])
    elif case == "self":
        args = ([0, 1], [1, 1])
    elif case == "dup":
        args = ([0, 0, 0], [1, 2, 2])
    elif case == "weights":
        args = ([0, 0], [1, 2], [1.0, 0.5])
    elif case == "into_source":
        args = ([0, 1], [1, 0])
    elif case == "out_of_range":
        args = ([0, 0], [1, 5], None, 3)
    else:
        args = ([0, 0], [1, 2], [1.0, 0.0])
    assert _call_graph("solve_dagmf", *args) == pf.PF_EGRAPH


def test_hmf_rejects_a_dag():
    # node 3 has two parents
    assert _call_graph("solve_hmf", [0, 0, 1, 2], [1, 2, 3, 3]) == pf.PF_EGRAPH


def test_graph_limits():
    n = 40
    assert _call_graph("solve_dagmf", [0] * (n - 1), list(range(1, n))) == pf.PF_EUNSUPPORTED


def test_ishikawa_needs_two_labels():
    lib = pf.library()
    assert lib.solve_ishikawa(C.byref(_grid()), 1, C.c_void_p(DEV), C.c_void_p(SADDR), 0,
                              C.byref(_params()), C.byref(pf._Result()), None) == pf.PF_EINVAL


def test_binding_refuses_cpu_tensors():
    import torch
    D = torch.zeros(1, 3, 1, 4, 4)
    with pytest.raises(ValueError):
        pf.solve_potts(D, 0.5, c=1.0, tau=0.1, iters=1)


def test_tape_and_backward_workspace_accounting():
    """One float32 state (labels, then flows, each 256-byte aligned) per
    checkpoint, ceil(K / k) checkpoints; the backward workspace holds the k
    recomputed states of a segment, two adjoint flow and two adjoint label
    states (ping-pong) and the per-flow capacity gradients."""
    lib = pf.library()
    g = _grid(2, 3, 8, 9, 10)
    V = 8 * 9 * 10
    al = lambda n: (n + 255) // 256 * 256
    slot = al(2 * 4 * V * 4) + al(2 * 6 * 3 * V * 4)
    for K, k in ((10, 5), (11, 5), (1, 1), (7, 10), (0, 3)):
        assert lib.pf_tape_bytes(C.byref(g), 4, 6, K, k) == -(-K // k) * slot
    for k in (1, 4, 10):
        n = lib.pf_backward_workspace_bytes(C.byref(g), 4, 6, k)
        adj = 2 * al(2 * 6 * 3 * V * 4) + 2 * al(2 * 4 * V * 4) + al(2 * 6 * V * 4)
        assert k * slot + adj <= n <= k * slot + adj + 64 * 1024
    assert lib.pf_tape_bytes(C.byref(g), 4, 6, 10, 0) == 0
    assert lib.pf_tape_bytes(C.byref(g), 4, 6, -1, 2) == 0
    assert lib.pf_tape_bytes(C.byref(g), 17, 6, 10, 2) == 0
    assert lib.pf_backward_workspace_bytes(C.byref(g), 4, 6, 0) == 0


@pytest.mark.parametrize("case,code", [
    ("no_tape", pf.PF_EINVAL), ("bf16", pf.PF_EUNSUPPORTED), ("ckpt0", pf.PF_EINVAL),
    ("small_tape", pf.PF_ENOMEM), ("misaligned_tape", pf.PF_ENOMEM),
    ("small_ws", pf.PF_ENOMEM), ("null_grad", pf.PF_EINVAL), ("misaligned_grad", pf.PF_EINVAL),
    ("bad_params", pf.PF_EINVAL),
])
def test_backward_argument_errors(case, code):
    lib = pf.library()
    g = _grid()
    tb = lib.pf_tape_bytes(C.byref(g), 3, 3, 5, 2)
    p = _params(ckpt_every=2, tape=512 * 1024, tape_bytes=tb)
    p.workspace_bytes = lib.pf_backward_workspace_bytes(C.byref(g), 3, 3, 2)
    gl, gd, gs = DEV, DEV + 4096, DEV + 8192
    if case == "no_tape":
        p.tape = None
    elif case == "bf16":
        p.storage = 1
    elif case == "ckpt0":
        p.ckpt_every = 0
    elif case == "small_tape":
        p.tape_bytes = tb - 1
    elif case == "misaligned_tape":
        p.tape = 512 * 1024 + 4
    elif case == "small_ws":
        p.workspace_bytes -= 256
    elif case == "null_grad":
        gd = 0
    elif case == "misaligned_grad":
        gs += 2
    elif case == "bad_params":
        p.c = 0.0
    st = lib.pf_potts_backward(C.byref(g), 3, C.c_void_p(DEV), C.c_void_p(SADDR), 0,
                                  C.byref(p), C.c_void_p(gl), C.c_void_p(gd), C.c_void_p(gs), None)
    assert st == code, (case, lib.pf_last_error())


def test_dag_backward_rejects_bad_graph():
    lib = pf.library()
    g = _grid()
    par = (C.c_int32 * 2)(0, 1)
    chi = (C.c_int32 * 2)(1, 0)            # cycle
    gr = pf._Graph(2, 2, par, chi, None)
    p = _params(ckpt_every=1, tape=512 * 1024, tape_bytes=1 << 30)
    st = lib.pf_dagmf_backward(C.byref(g), C.byref(gr), C.c_void_p(DEV), C.c_void_p(SADDR), 0,
                                  C.byref(p), C.c_void_p(DEV), C.c_void_p(DEV), C.c_void_p(DEV), None)
    assert st == pf.PF_EGRAPH
