"""Checks run on the threaded CPU build of the library (see run.sh): the
library's own host code and kernel sources, compiled for the host under
AddressSanitizer and UBSan, driven through the C ABI with host buffers.

1. Forward: the fused and the two-pass iteration give the same state, energy
   and dual bit for bit (fp32, bf16, fp16; odd label and flow counts, ragged
   tiles, several z chunks), and so does the two-iterations-per-pass kernel
   (odd iteration counts and gap checks mixing in one-iteration passes).
2. The full-flow Potts solver against its float64 reference implementation,
   and solve_dagmf_static (the library's static scratch) against solve_dagmf
   with a workspace, bit for bit, on two calls in a row.
3. Reverse: recorded forward + backward against autograd through the float64
   reference implementation, and the fused reverse step bit for bit against
   the two-kernel one.

Usage: python check.py path/to/libcpu.so [forward] [fused2] [lds] [flowlabel] [fullflow] [static] [reverse]
"""
import ctypes as C
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import paper_1501_07844_amd as pf                      # noqa: E402  (structs only)
from paper_1501_07844_amd import synth                  # noqa: E402
from oracle import fullflow_oracle as FF                # noqa: E402
from oracle import pseudoflow_oracle as O               # noqa: E402

lib = C.CDLL(sys.argv[1])
for n in ("pf_tape_bytes", "pf_backward_workspace_bytes", "pf_workspace_bytes",
          "pf_fullflow_workspace_bytes"):
    getattr(lib, n).restype = C.c_size_t
lib.pf_last_error.restype = C.c_char_p


def aligned(nbytes):
    raw = np.zeros(nbytes + 512, np.uint8)
    return raw, raw.ctypes.data + (-raw.ctypes.data) % 256


def ptr(a):
    return C.c_void_p(a.ctypes.data)


def solve(p, iters, kernel, storage, tape=None, every=0, want_ell=False, gap_every=0, entry=None,
          c=None, tau=None):
    B, Z, Y, X = p.shape
    nl, nn = p.n_leaf, p.n_node
    D = np.ascontiguousarray(p.D, np.float32)
    S = np.ascontiguousarray(np.asarray(p.S, np.float32))
    grid = pf._Grid(B, p.ndim, Z, Y, X)
    keep = []
    prm = pf._Params()
    prm.iters, prm.c, prm.tau = iters, p.c if c is None else c, p.tau if tau is None else tau
    prm.storage, prm.kernel, prm.final_energy = pf.STORAGE[storage], pf.KERNEL[kernel], 1
    prm.gap_every = gap_every
    if entry == "fullflow":
        need = lib.pf_fullflow_workspace_bytes(C.byref(grid), nl)
    else:
        need = lib.pf_workspace_bytes(C.byref(grid), nl, nn, C.byref(prm))
    if entry != "static":
        wraw, wptr = aligned(need)
        keep.append(wraw)
        prm.workspace, prm.workspace_bytes = wptr, need
    if tape is not None:
        prm.ckpt_every, prm.tape, prm.tape_bytes = every, tape[1], tape[2]
    u = np.zeros((B, nl, Z, Y, X), np.float32)
    q = np.zeros((B, nn, p.ndim, Z, Y, X), np.float32)
    ell = np.zeros_like(u)
    r = pf._Result()
    r.u, r.q = u.ctypes.data, q.ctypes.data
    if want_ell:
        r.ell = ell.ctypes.data
    mode = pf.S_MODE[p.s_mode]
    if entry == "fullflow":
        st = lib.solve_potts_fullflow(C.byref(grid), nl, ptr(D), ptr(S), mode, C.byref(prm), C.byref(r), None)
    elif entry == "static":
        g = pf._graph_struct(p.graph, keep)
        st = lib.solve_dagmf_static(C.byref(grid), C.byref(g), ptr(D), ptr(S), mode, C.byref(prm), C.byref(r),
                                    None)
    elif p.kind == "potts":
        st = lib.solve_potts(C.byref(grid), nl, ptr(D), ptr(S), mode, C.byref(prm), C.byref(r), None)
    elif p.kind == "ishikawa":
        st = lib.solve_ishikawa(C.byref(grid), nl, ptr(D), ptr(S), mode, C.byref(prm), C.byref(r), None)
    else:
        g = pf._graph_struct(p.graph, keep)
        st = lib.solve_dagmf(C.byref(grid), C.byref(g), ptr(D), ptr(S), mode, C.byref(prm), C.byref(r), None)
    if st != 0:
        raise RuntimeError(lib.pf_last_error().decode())
    return u, q, ell, r.energy, r.dual


def forward_cases():
    rng = np.random.default_rng(3)
    dag = synth.random_dag(rng, 3, 5)
    return [
        ("potts3d nl3 B2 chunks", synth.random_potts(1, (40, 10, 140), 3, 3, batch=2, s_mode="node_field"), 5),
        ("potts2d nl5 shared", synth.random_potts(2, (1, 37, 129), 2, 5, s_mode="shared_field"), 6),
        ("potts3d nl8 scalar", synth.random_potts(3, (34, 9, 130), 3, 8, s_mode="node_scalar"), 4),
        ("dag3d nl5 nn8 B2", synth.random_problem(4, (33, 9, 66), 3, dag, batch=2, s_mode="node_field"), 4),
    ]


def check_forward():
    bad = 0
    for name, p, iters in forward_cases():
        for storage in ("fp32", "bf16", "fp16"):
            a = solve(p, iters, "two_pass", storage)
            b = solve(p, iters, "fused", storage)
            same = all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[3:] == b[3:]
            print(f"forward {name:24s} {storage}: fused == two-pass bitwise: {same}", flush=True)
            bad += not same
    return bad


def lds_cases():
    rng = np.random.default_rng(9)
    dag = synth.random_dag(rng, 3, 5)
    wide = synth.random_dag(rng, 5, 7)
    return [
        # tiles with ghost zones (fewer than 8 problems)
        ("potts2d nl3 64x64", synth.potts2d_rects(), 19, 0),
        ("potts2d nl5 B2 nodefield", synth.random_potts(7, (1, 37, 70), 2, 5, batch=2, s_mode="node_field"), 17, 3),
        ("dag2d nl5 nn8 shared", synth.random_problem(8, (1, 26, 37), 2, dag, s_mode="shared_field"), 11, 4),
        ("dag2d nl7 nn12 field", synth.random_problem(10, (1, 21, 30), 2, wide, s_mode="node_field"), 9, 0),
        ("potts2d nl2 B3 thin", synth.random_potts(12, (1, 3, 41), 2, 2, batch=3), 10, 0),
        # whole problems per block (8 or more)
        ("potts2d nl3 B8 whole", synth.random_potts(13, (1, 20, 30), 2, 3, batch=8), 5, 2),
    ]


def check_lds():
    """The LDS-resident 2-D solves (tiles with ghost zones, whole problems)
    against the two-pass kernels."""
    bad = 0
    for name, p, iters, gap_every in lds_cases():
        for storage in ("fp32", "bf16", "fp16"):
            a = solve(p, iters, "two_pass", storage, gap_every=gap_every)
            b = solve(p, iters, "lds", storage, gap_every=gap_every)
            same = all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[3:] == b[3:]
            print(f"forward {name:24s} {storage}: LDS-resident == two-pass bitwise: {same}", flush=True)
            bad += not same
    return bad


def fused2_cases():
    return [
        ("potts3d nl3 B2 chunks", synth.random_potts(1, (40, 10, 140), 3, 3, batch=2, s_mode="node_field"), 5, 0),
        ("potts3d nl8 scalar", synth.random_potts(3, (34, 9, 130), 3, 8, s_mode="node_scalar"), 4, 0),
        ("potts3d nl5 shared gap3", synth.random_potts(5, (35, 17, 66), 3, 5, s_mode="shared_field"), 7, 3),
        ("potts3d nl4 thin", synth.random_potts(6, (2, 3, 70), 3, 4, s_mode="node_scalar"), 4, 0),
    ]


def check_fused2():
    """Two iterations per pass against the one-iteration fused kernel."""
    bad = 0
    for name, p, iters, gap_every in fused2_cases():
        for storage in ("fp32", "bf16", "fp16"):
            a = solve(p, iters, "fused", storage, gap_every=gap_every)
            b = solve(p, iters, "fused2", storage, gap_every=gap_every)
            same = all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[3:] == b[3:]
            print(f"forward {name:24s} {storage}: two-iteration == fused bitwise: {same}", flush=True)
            bad += not same
    return bad


def flow_label_cases():
    rng = np.random.default_rng(11)
    dag = synth.random_dag(rng, 3, 5)
    tree = synth.hmf_tree()
    big = synth.random_dag(rng, 0, 16)
    tiny = synth.random_tree(rng, 1, 2)
    return [
        ("dag3d nl5 nn8 B2 field", synth.random_problem(4, (33, 9, 70), 3, dag, batch=2, s_mode="node_field"), 4, 0),
        ("hmf3d nl8 nn11 shared gap2", synth.random_problem(5, (20, 13, 35), 3, tree, s_mode="shared_field"), 5, 2),
        ("dagmf3d nl12 nn16", synth.dagmf_blobs(shape=(18, 14, 66)), 3, 0),
        ("ishikawa3d 8 levels", synth.ishikawa_levels(shape=(17, 7, 35), n_levels=7), 3, 0),
        # chains in builds with padding labels, and the largest chain build
        ("ishikawa3d 3 levels", synth.ishikawa_levels(shape=(18, 6, 67), n_levels=2), 3, 2),
        ("ishikawa3d 5 levels", synth.ishikawa_levels(shape=(9, 11, 30), n_levels=4), 3, 0),
        ("ishikawa3d 12 levels", synth.ishikawa_levels(shape=(5, 9, 20), n_levels=11), 2, 0),
        ("ishikawa3d 16 levels", synth.ishikawa_levels(shape=(4, 5, 66), n_levels=15), 2, 0),
        ("dag3d nl16 nn16", synth.random_problem(6, (9, 8, 34), 3, big, s_mode="node_scalar"), 2, 0),
        ("tree3d nl2 nn3 thin", synth.random_problem(7, (3, 2, 40), 3, tiny, s_mode="node_field"), 3, 0),
        # graphs filling every slot of a tail build (the EXACT forms)
        ("dag3d nl4 nn8 B2 exact", synth.random_problem(8, (21, 10, 70), 3, synth.random_dag(rng, 4, 4),
                                                        batch=2, s_mode="node_field"), 4, 3),
        ("dag3d nl8 nn12 exact", synth.random_problem(9, (12, 9, 66), 3, synth.random_dag(rng, 4, 8),
                                                      s_mode="shared_field"), 3, 0),
    ]


def check_flow_label():
    """The flow-then-label pass for 3-D label graphs against the two-pass
    kernels, bit for bit."""
    bad = 0
    for name, p, iters, gap_every in flow_label_cases():
        for storage in ("fp32", "bf16", "fp16"):
            a = solve(p, iters, "two_pass", storage, gap_every=gap_every)
            b = solve(p, iters, "fused", storage, gap_every=gap_every)
            same = all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[3:] == b[3:]
            print(f"forward {name:24s} {storage}: flow-label == two-pass bitwise: {same}", flush=True)
            bad += not same
    return bad


def check_fullflow():
    """The full-flow solver (float32) against its float64 reference: u and q
    within 1e-4, energy and dual within 1e-4 relative."""
    bad = 0
    cases = [
        ("potts2d nl3 rects", synth.potts2d_rects(), 0.3, 0.16, 30),
        ("potts3d nl5 B2 field", synth.random_potts(21, (6, 9, 70), 3, 5, batch=2, s_mode="node_field",
                                                    d_scale=3.0), 1.0, 0.1, 12),
        ("potts3d nl12 shared", synth.random_potts(22, (5, 7, 40), 3, 12, s_mode="shared_field",
                                                   d_scale=3.0), 1.0, 0.1, 8),
    ]
    for name, p, c, tau, iters in cases:
        u, q, _, E, P = solve(p, iters, "auto", "fp32", entry="fullflow", c=c, tau=tau)
        ref = FF.solve_potts_fullflow(p.D, p.S, p.s_mode, c, tau, iters, p.ndim)
        du = np.abs(u - ref["u"].numpy()).max()
        dq = np.abs(q - ref["q"].numpy()).max()
        ok = du <= 1e-4 and dq <= 1e-4 and abs(E - ref["E"][-1]) <= 1e-4 * abs(ref["E"][-1]) \
            and abs(P - ref["P"][-1]) <= 1e-4 * abs(ref["E"][-1])
        print(f"fullflow {name:24s} max|du| {du:.1e} max|dq| {dq:.1e}: {'ok' if ok else 'BAD'}", flush=True)
        bad += not ok
    return bad


def check_static():
    """solve_dagmf_static against solve_dagmf with a workspace, bit for bit,
    on two calls in a row (the second smaller)."""
    bad = 0
    rng = np.random.default_rng(23)
    dag = synth.random_dag(rng, 3, 5)
    for name, p in (("dag3d nl5 nn8 B2", synth.random_problem(24, (12, 9, 40), 3, dag, batch=2,
                                                             s_mode="node_field")),
                    ("dag2d nl5 nn8", synth.random_problem(25, (1, 11, 23), 2, dag, s_mode="shared_field"))):
        for storage in ("fp32", "bf16"):
            a = solve(p, 4, "auto", storage)
            b = solve(p, 4, "auto", storage, entry="static")
            same = all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[3:] == b[3:]
            print(f"static {name:24s} {storage}: static scratch == workspace bitwise: {same}", flush=True)
            bad += not same
    return bad


def grad(p, iters, every, bkernel, w):
    B, Z, Y, X = p.shape
    nl, nn = p.n_leaf, p.n_node
    grid = pf._Grid(B, p.ndim, Z, Y, X)
    tb = lib.pf_tape_bytes(C.byref(grid), nl, nn, iters, every)
    traw, tptr = aligned(tb)
    _, _, ell, _, _ = solve(p, iters, "two_pass", "fp32", tape=(traw, tptr, tb), every=every, want_ell=True)
    D = np.ascontiguousarray(p.D, np.float32)
    S = np.ascontiguousarray(np.asarray(p.S, np.float32))
    gD, gS = np.full_like(D, np.nan), np.full_like(S, np.nan)
    prm = pf._Params()
    prm.iters, prm.c, prm.tau, prm.kernel = iters, p.c, p.tau, pf.KERNEL[bkernel]
    bw = lib.pf_backward_workspace_bytes(C.byref(grid), nl, nn, every)
    braw, bptr = aligned(bw)
    prm.workspace, prm.workspace_bytes = bptr, bw
    prm.ckpt_every, prm.tape, prm.tape_bytes = every, tptr, tb
    gl = np.ascontiguousarray(w, np.float32)
    args = (ptr(D), ptr(S), pf.S_MODE[p.s_mode], C.byref(prm), ptr(gl), ptr(gD), ptr(gS), None)
    if p.kind == "potts":
        st = lib.pf_potts_backward(C.byref(grid), nl, *args)
    else:
        keep = []
        g = pf._graph_struct(p.graph, keep)
        st = lib.pf_dagmf_backward(C.byref(grid), C.byref(g), *args)
    if st != 0:
        raise RuntimeError(lib.pf_last_error().decode())
    return ell, gD, gS


def oracle_grad(p, iters, w):
    D = torch.tensor(p.D, dtype=torch.float64, requires_grad=True)
    S = torch.tensor(np.asarray(p.S), dtype=torch.float64, requires_grad=True)
    if p.kind == "potts":
        ell = O.solve_potts(D, S, p.s_mode, p.c, p.tau, iters, p.ndim, history=False)["ell"]
    else:
        g = O.OracleGraph(p.graph.n_nodes, p.graph.parent, p.graph.child, p.graph.weight)
        ell = O.solve_dagmf(D, S, p.s_mode, g, p.c, p.tau, iters, p.ndim, history=False)["ell"]
    (ell * torch.tensor(w, dtype=torch.float64)).sum().backward()
    return ell.detach().numpy(), D.grad.numpy(), S.grad.numpy()


def reverse_cases():
    rng = np.random.default_rng(7)
    dag = synth.random_dag(rng, 3, 5)
    tree = synth.random_tree(rng, 2, 4)
    small = synth.random_dag(rng, 3, 4)
    return [
        ("potts2d nl4 shared K13 k5", synth.random_potts(11, (1, 7, 11), 2, 4, batch=2, s_mode="shared_field", c=2.0, tau=0.125), 13, 5),
        ("potts3d nl3 scalar K9 k4", synth.random_potts(12, (4, 5, 6), 3, 3, s_mode="node_scalar", c=1.0, tau=0.125), 9, 4),
        ("potts2d nl5 nodefield K6 k1", synth.random_potts(13, (1, 6, 9), 2, 5, s_mode="node_field", c=2.0, tau=0.125), 6, 1),
        ("dag2d nodefield K8 k3", synth.random_problem(14, (1, 6, 7), 2, dag, batch=2, s_mode="node_field", c=4.0, tau=0.0625), 8, 3),
        ("tree3d scalar K7 k3", synth.random_problem(15, (3, 4, 5), 3, tree, s_mode="node_scalar", c=4.0, tau=0.0625, kind="hmf"), 7, 3),
        ("dag2d nl4 scalar K7 k3", synth.random_problem(17, (1, 19, 70), 2, small, s_mode="node_scalar", c=4.0, tau=0.0625), 7, 3),
        ("potts3d nl3 chunks K4 k2", synth.random_potts(18, (33, 10, 67), 3, 3, s_mode="node_field", c=1.0, tau=0.125), 4, 2),
        ("potts2d nl3 rows K5 k2", synth.random_potts(19, (1, 23, 130), 2, 3, s_mode="node_field", c=1.0, tau=0.125), 5, 2),
    ]


def fused_reverse_supported(p):
    """The buckets the fused reverse kernel is built for (pf_adjoint.hip)."""
    if p.ndim == 2:
        return p.n_leaf <= 8 if p.kind == "potts" else (p.n_leaf <= 4 and p.n_node <= 8)
    return p.kind == "potts" and p.n_leaf <= 4


def check_reverse():
    bad = 0
    for name, p, iters, every in reverse_cases():
        w = np.random.default_rng(0).standard_normal(p.D.shape).astype(np.float32)
        ell, gD, gS = grad(p, iters, every, "two_pass", w)
        rell, rD, rS = oracle_grad(p, iters, w)
        eD = np.abs(gD - rD).max() / np.abs(rD).max()
        eS = np.abs(gS - rS).max() / np.abs(rS).max()
        ok = np.abs(ell - rell).max() < 1e-5 and eD < 1e-4 and eS < 1e-4
        msg = f"reverse {name:28s} rel dD {eD:.1e} rel dS {eS:.1e}"
        if fused_reverse_supported(p):
            _, fD, fS = grad(p, iters, every, "fused", w)
            same = np.array_equal(fD, gD) and np.array_equal(fS, gS)
            msg += f"  fused == two-kernel bitwise: {same}"
            ok = ok and same
        print(msg + ("" if ok else "  BAD"), flush=True)
        bad += not ok
    return bad


if __name__ == "__main__":
    torch.set_num_threads(min(8, torch.get_num_threads()))
    only = sys.argv[2:]
    n_bad = 0
    if not only or "forward" in only:
        n_bad += check_forward()
    if not only or "fused2" in only:
        n_bad += check_fused2()
    if not only or "lds" in only:
        n_bad += check_lds()
    if not only or "flowlabel" in only:
        n_bad += check_flow_label()
    if not only or "fullflow" in only:
        n_bad += check_fullflow()
    if not only or "static" in only:
        n_bad += check_static()
    if not only or "reverse" in only:
        n_bad += check_reverse()
    print("ALL OK" if n_bad == 0 else f"{n_bad} FAILED")
    sys.exit(1 if n_bad else 0)
