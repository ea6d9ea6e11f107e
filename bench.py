"""Throughput of the pseudo-flow solvers on one MI355X.

Headline workload: DAGMF on a 3-D grid of 256 x 512 x 512 voxels, a label DAG
of 4 shared parents and 12 leaves (16 flows, two random parents per leaf),
bf16 flow and label storage with float32 arithmetic and float64 energy/gap
reductions, 300 iterations (seeded random-blob phantom: 64 balls of radius
U[16, 64] and class U{1..11} on background 0, noise 0.1, Gaussian-NLL data
terms, S_A ~ U[0.1, 1]).  One step is one complete solve: initialisation, 300
iterations, the float64 energy/dual/gap evaluation and the argmax export.
Inputs are resident in HBM before timing starts.

Prints one JSON line: voxel-label iterations per second (voxel-label = voxels
x non-source label nodes) of the headline solve; the roofline of its kernel,
timed with HIP events inside the timed region; whole solves of the 256^3
Potts workload (8 labels, float32, 500 iterations) with the roofline of its
two-iteration kernel; the per-iteration kernel rates of every workload
(Potts 3-D, HMF, DAGMF and an Ishikawa chain scaled to 128 x 256 x 256 with 8
ordered labels; float32, bf16 and fp16 state), whole-solve rates of the two
small 2-D cases (Potts and Ishikawa) and of a batch of 256 of the Potts case;
the primal-dual gap after every iteration of the Potts and DAGMF solves; the
full-flow counterpart against the pseudo-flow solver on the Potts workload
(state memory, time per iteration, gap reached); a plain device copy as the achievable bandwidth; the cost of the
differentiable solve; and the float64 reference implementation timed on a
bounded sample on the host.

``--counters`` runs only a short program for rocprofv3 counter passes: a
device copy of known size, then a few launches of the chosen workload's
kernel.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30          # the copy kernel moves 1 GiB in and 1 GiB out
HEADLINE_STORAGE = "bf16"
POTTS_ITERS = 500

# the sources each timed kernel is built from (its traffic record is valid
# only while they hash to the recorded value)
KERNEL_SOURCES = {
    "k_flow_label": ("pf_flowlabel.hip", "pf_device.h", "pf_internal.h"),
    "k_fused2": ("pf_fused.hip", "pf_device.h", "pf_internal.h"),
    "k_fused": ("pf_fused.hip", "pf_device.h", "pf_internal.h"),
    "k_label+k_flow": ("pf_kernels.hip", "pf_device.h", "pf_internal.h"),
}
TRAFFIC_FILES = {"dagmf": "traffic_dagmf_256x512x512_bf16.json",
                 "potts3d": "traffic_potts3d_256.json"}


def _kernel_source_hash(kernel: str) -> str:
    """Hash of the sources `kernel` is built from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1501_07844_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(which: str, kernel: str, source_hash: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of workload `which`, only while the kernel sources are the ones
    it was taken on."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[which])
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def bytes_alg(p, storage: str) -> int:
    """Algorithmic HBM bytes per voxel and iteration: every state field read
    and written once, the data terms and capacity fields read once."""
    s = 4 if storage == "fp32" else 2
    s_fields = {"node_scalar": 0, "shared_field": 1, "node_field": p.n_node}[p.s_mode]
    return 2 * s * (p.n_leaf + p.ndim * p.n_node) + 4 * p.n_leaf + 4 * s_fields


def _inputs(p, dev):
    import numpy as np
    import torch
    D = torch.from_numpy(p.D).to(dev)
    S = np.asarray(p.S) if p.s_mode == "node_scalar" else torch.from_numpy(p.S).to(dev)
    return D, S


def _solver(pf, p):
    if p.kind == "potts":
        return lambda D, S, **kw: pf.solve_potts(D, S, **kw)
    if p.kind == "hmf":
        return lambda D, S, **kw: pf.solve_hmf(D, S, p.graph, **kw)
    if p.kind == "ishikawa":
        return lambda D, S, **kw: pf.solve_ishikawa(D, S, **kw)
    return lambda D, S, **kw: pf.solve_dagmf(D, S, p.graph, **kw)


KERNEL_NAMES = {"fused2": "k_fused2", "fused": "k_fused", "two_pass": "k_label+k_flow",
                "lds": "k_lds2d"}


def _kernel_name(p, choice: str) -> str:
    """The kernel a choice launches per iteration: the fused kind on a 3-D
    label graph is the flow-then-label pass; the LDS kind holds whole
    problems for batches of 8 or more that fit (4096 voxels, 40960 floats),
    tiles with ghost zones otherwise."""
    if choice == "fused" and p.kind != "potts" and p.ndim == 3:
        return "k_flow_label"
    if choice == "lds":
        B, V = p.shape[0], p.shape[1] * p.shape[2] * p.shape[3]
        whole = B >= 8 and V <= 4096 and V * (p.n_leaf + 2 * p.n_node) <= 40960
        return "k_lds2d" if whole else "k_tile2d"
    return KERNEL_NAMES[choice]


def _kernel_choice(pf, p, storage: str, kernel: str) -> str:
    """The kernel the library runs (AUTO resolved by the library's own rule;
    the Ishikawa chain follows the label-graph rule)."""
    if kernel != "auto":
        return kernel
    return pf.auto_kernel(p.shape, p.n_leaf, p.n_node, p.ndim, storage,
                          identity=p.kind == "potts")


def kernel_leg(p, storage: str, iters: int, dev, kernel: str = "auto") -> dict:
    """Kernel time of one workload: one warm-up solve, then a solve with
    every launch bracketed by HIP events on the solver's stream; the mean
    per iteration (a k_fused2 launch covers two).  alg_GBs: algorithmic
    bytes of one iteration over the time per iteration; launch_alg_GBs: the
    bytes one launch must move over its duration (the roofline figure).
    energy_full / rel_gap_full: final energy and relative gap of the warm-up
    solve, run at the workload's own iteration budget (the figures the
    16-bit storage types are compared on)."""
    import paper_1501_07844_amd as pf
    D, S = _inputs(p, dev)
    solve = _solver(pf, p)
    kw = dict(c=p.c, tau=p.tau, ndim=p.ndim, s_mode=p.s_mode, storage=storage,
              kernel=kernel, final_energy=True, return_u=False, return_labels=False)
    full = solve(D, S, iters=p.iters, **kw)          # warm-up, and the energy at the full budget
    r = solve(D, S, iters=iters, workspace=full.workspace, timing_stride=1, **kw)
    ms = r.kernel_ms / max(r.kernel_timed, 1)
    choice = _kernel_choice(pf, p, storage, kernel)
    per_launch = 2 if choice == "fused2" else 1
    V = p.voxels
    ba = bytes_alg(p, storage)
    achieved = ba * V / (ms * 1e-3) / 1e9
    launch = ba * V / (per_launch * ms * 1e-3) / 1e9
    out = {"workload": f"{p.name} {'x'.join(map(str, p.shape[1:]))}"
                       + (f" x{p.shape[0]}" if p.shape[0] > 1 else ""),
           "storage": storage, "kernel": _kernel_name(p, choice),
           "ms_per_iter": round(ms, 4), "iterations_timed": r.kernel_timed,
           "iterations_per_launch": per_launch,
           "voxel_label_its_per_s": V * p.n_node / (ms * 1e-3),
           "alg_bytes_per_voxel": ba, "alg_GBs": round(achieved, 1),
           "launch_alg_GBs": round(launch, 1),
           "hbm_frac": round(launch / HBM_PEAK_GBS, 4), "energy": r.energy,
           "iterations_full": p.iters, "energy_full": full.energy,
           "rel_gap_full": full.gap / abs(full.energy)}
    del D, S, r, full
    return out


def copy_leg(dev) -> dict:
    """Achievable bandwidth: a plain device-to-device copy of 1 GiB (read +
    write bytes over the kernel time), median of 5 after a warm-up."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    ts = []
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        if i:
            ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    return {"bytes": 2 * COPY_BYTES, "ms": round(ms, 4),
            "GBs": round(2 * COPY_BYTES / (ms * 1e-3) / 1e9, 1)}


def adjoint_leg(dev, reps: int = 5) -> dict:
    """Cost of the differentiable solve on its own workload: 16 Potts problems
    of 256 x 256, 5 labels, 100 unrolled iterations, checkpoint every 10,
    cross-entropy loss against the ground-truth labels.  Times (HIP events on
    the stream the library launches on, median of `reps` after one warm-up):
    the plain forward solve, the recorded forward, and the backward."""
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth

    p = synth.diff_batch()
    D = torch.from_numpy(p.D).to(dev)
    S = torch.from_numpy(p.S).to(dev)
    gt = torch.from_numpy(p.gt.astype("int64")).to(dev).unsqueeze(1)
    k = p.extra["checkpoint_every"]

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1), r

    ws = [None]

    def plain():
        r = pf.solve_potts(D, S, c=p.c, tau=p.tau, iters=p.iters, s_mode="shared_field", ndim=2,
                           kernel="two_pass", final_energy=False, return_u=False,
                           return_labels=False, return_ell=True, workspace=ws[0])
        ws[0] = r.workspace
        return r

    f_ms, r_ms, b_ms = [], [], []
    for i in range(reps + 1):
        tf, _ = timed(plain)
        Dg = D.clone().requires_grad_(True)
        Sg = S.clone().requires_grad_(True)
        tr, ell = timed(lambda: pf.potts_layer(Dg, Sg, c=p.c, tau=p.tau, iters=p.iters,
                                               ckpt_every=k))
        loss = -torch.gather(ell, 1, gt).mean()
        tb, _ = timed(lambda: loss.backward())
        if i:
            f_ms.append(tf), r_ms.append(tr), b_ms.append(tb)
    med = lambda v: sorted(v)[len(v) // 2]
    f, r, b = med(f_ms), med(r_ms), med(b_ms)
    print(f"[bench] adjoint: forward {f:.2f} ms, recorded {r:.2f} ms, backward {b:.2f} ms",
          file=sys.stderr, flush=True)
    # algorithmic bytes per voxel and unrolled step of the backward: the
    # recomputed forward step (state read and written once, D and S read) and
    # the reverse step (forward state q_k, ell_{k+1}; adjoints lbar, pbar read
    # and written; dD and dS read and written; S read)
    nl, nn, nd = p.n_leaf, p.n_node, p.ndim
    s_f = 1 if p.s_mode == "shared_field" else (nn if p.s_mode == "node_field" else 0)
    fwd_b = 8 * (nl + nd * nn) + 4 * nl + 4 * s_f
    rev_b = 4 * ((nd * nn + nl) + 2 * (nl + nd * nn) + 2 * nl + 2 * s_f + s_f)
    V = p.voxels
    alg = (fwd_b + rev_b) * V * p.iters / (b * 1e-3) / 1e9
    return {"workload": f"diff_batch 16x256x256, 5 labels, {p.iters} iterations, checkpoint "
                        f"every {k}, fp32", "forward_ms": round(f, 3),
            "forward_recorded_ms": round(r, 3), "backward_ms": round(b, 3),
            "backward_over_forward": round(b / f, 3), "total_over_forward": round((r + b) / f, 3),
            "backward_alg_bytes_per_voxel_step": fwd_b + rev_b, "backward_alg_GBs": round(alg, 1),
            "backward_hbm_frac": round(alg / HBM_PEAK_GBS, 4)}


def potts2d_leg(dev, reps: int = 7) -> dict:
    """The small 2-D Potts case (64 x 64, 3 labels, 200 iterations, final
    energy included): whole solves per second, median of `reps`, with the
    kernel AUTO takes (LDS tiles with ghost zones, eight iterations per
    launch) against the forced two-pass kernels (two launches per
    iteration), and the two solutions compared bit for bit."""
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    p = synth.potts2d_rects()
    D, S = _inputs(p, dev)
    out = {"workload": "potts2d_rects 64x64, 3 labels, 200 iterations, fp32"}
    sols = {}
    for name, kernel in (("auto", "auto"), ("two_pass", "two_pass")):
        kw = dict(c=p.c, tau=p.tau, iters=p.iters, s_mode=p.s_mode, ndim=2, kernel=kernel,
                  final_energy=True, return_q=True)
        r = pf.solve_potts(D, S, **kw)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pf.solve_potts(D, S, workspace=r.workspace, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[len(ts) // 2]
        sols[name] = r
        out[name] = {"ms_per_solve": round(1e3 * t, 3), "iterations_per_s": round(p.iters / t, 1)}
    choice = _kernel_choice(pf, p, "fp32", "auto")
    out["auto"]["kernel"] = _kernel_name(p, choice)
    out["ms_per_solve"] = out["auto"]["ms_per_solve"]
    out["iterations_per_s"] = out["auto"]["iterations_per_s"]
    out["speedup_vs_two_pass"] = round(out["two_pass"]["ms_per_solve"] / out["auto"]["ms_per_solve"], 3)
    a, b = sols["auto"], sols["two_pass"]
    out["same_u_q_bitwise"] = bool(torch.equal(a.u, b.u) and torch.equal(a.q, b.q))
    out["energy"], out["gap"] = a.energy, a.gap
    return out


def potts2d_batch_leg(dev, batch: int = 256, reps: int = 5) -> dict:
    """A batch of `batch` copies of the 64 x 64 Potts case (3 labels, 200
    iterations): the kernel AUTO takes (the LDS-resident solve, one compute
    unit per problem) against the forced two-pass kernels, whole batch
    solves per second, median of `reps`, and the two solutions compared."""
    import numpy as np
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    p = synth.potts2d_rects()
    _, S = _inputs(p, dev)                       # node constants: the same for every copy
    D = torch.from_numpy(np.ascontiguousarray(np.repeat(p.D, batch, axis=0))).to(dev)
    out = {"workload": f"potts2d_rects 64x64 x{batch}, 3 labels, 200 iterations, fp32"}
    sols = {}
    for name, kernel in (("auto", "auto"), ("two_pass", "two_pass")):
        kw = dict(c=p.c, tau=p.tau, iters=p.iters, s_mode=p.s_mode, ndim=2, kernel=kernel,
                  final_energy=False, return_labels=False)
        r = pf.solve_potts(D, S, **kw)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pf.solve_potts(D, S, workspace=r.workspace, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[len(ts) // 2]
        sols[name] = r.u
        out[name] = {"ms_per_solve": round(1e3 * t, 3),
                     "voxel_label_its_per_s": batch * p.voxels * p.n_node * p.iters / t}
    out["auto"]["kernel"] = pf.auto_kernel((batch,) + tuple(p.shape[1:]), p.n_leaf, p.n_node, 2)
    out["speedup_vs_two_pass"] = round(out["two_pass"]["ms_per_solve"] / out["auto"]["ms_per_solve"], 3)
    out["same_u_bitwise"] = bool(torch.equal(sols["auto"], sols["two_pass"]))
    return out


def ishikawa2d_leg(dev, reps: int = 5) -> dict:
    """The ordered-label workload at its own size (96 x 128, 5 levels, 200
    iterations): whole solves per second, median of `reps`."""
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    p = synth.ishikawa_levels()
    D, S = _inputs(p, dev)
    kw = dict(c=p.c, tau=p.tau, iters=p.iters, s_mode=p.s_mode, ndim=2, final_energy=True)
    r = pf.solve_ishikawa(D, S, **kw)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pf.solve_ishikawa(D, S, workspace=r.workspace, **kw)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t = sorted(ts)[len(ts) // 2]
    return {"workload": "ishikawa_levels 96x128, 5 ordered labels, 200 iterations, fp32",
            "ms_per_solve": round(1e3 * t, 3), "iterations_per_s": round(p.iters / t, 1),
            "energy": r.energy, "gap": r.gap}


def counters_program(which: str = "dagmf", kernel: str = "auto",
                     storage: str = HEADLINE_STORAGE) -> int:
    """Short program for rocprofv3 counter passes.  "dagmf": one copy of
    COPY_BYTES (the calibration kernel), then 3 iterations of the headline
    solve (3 launches of its kernel).  "potts3d": the copy, then 6 iterations
    of the 256^3 Potts solve (3 launches of k_fused2 with the AUTO choice).
    "graphs": 3 two-pass iterations of DAGMF at 128x256x256 and of Potts-3D
    at 128^3 (fp32).  `kernel` overrides the AUTO choice, `storage` the
    headline's state type."""
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    dev = torch.device("cuda:0")
    if which == "graphs":
        p = synth.dagmf_blobs(shape=(128, 256, 256))
        D = torch.from_numpy(p.D).to(dev)
        pf.solve_dagmf(D, p.S, p.graph, c=p.c, tau=p.tau, iters=3, ndim=3, s_mode=p.s_mode,
                       kernel="two_pass", final_energy=False, return_u=False, return_labels=False)
        q = synth.potts3d_voronoi(n=128)
        D2, S2 = _inputs(q, dev)
        pf.solve_potts(D2, S2, c=q.c, tau=q.tau, iters=3, ndim=3, s_mode=q.s_mode,
                       kernel="two_pass", final_energy=False, return_u=False, return_labels=False)
        torch.cuda.synchronize()
        print(json.dumps({"counters_program": "graphs", "done": True}), flush=True)
        return 0
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    if which == "potts3d":
        p = synth.potts3d_voronoi(n=256, iters=6)
        D, S = _inputs(p, dev)
        r = pf.solve_potts(D, S, c=p.c, tau=p.tau, iters=6, ndim=3, s_mode=p.s_mode,
                           kernel=kernel, final_energy=False, return_u=False, return_labels=False)
        choice = _kernel_choice(pf, p, "fp32", kernel)
    else:
        p = synth.dagmf_blobs(iters=3)
        D = torch.from_numpy(p.D).to(dev)
        r = pf.solve_dagmf(D, p.S, p.graph, c=p.c, tau=p.tau, iters=3, ndim=3, s_mode=p.s_mode,
                           storage=storage, kernel=kernel, final_energy=False,
                           return_u=False, return_labels=False)
        choice = _kernel_choice(pf, p, storage, kernel)
    torch.cuda.synchronize()
    name = _kernel_name(p, choice)
    print(json.dumps({"counters_program": which, "iters": r.iters_done, "kernel": name,
                      "source_hash": _kernel_source_hash(name) if name in KERNEL_SOURCES else None}),
          flush=True)
    return 0


def timed_solves(pf, solve, D, S, kw, steps: int, warmup: int, stride: int):
    """`warmup` untimed solves, then `steps` solves timed as a whole
    (synchronised on both sides) with the launch starting every `stride`-th
    iteration also bracketed by HIP events on the library's stream."""
    import torch
    ws = res = None
    for _ in range(warmup):
        res = solve(D, S, workspace=ws, **kw)
        ws = res.workspace
    torch.cuda.synchronize()
    kms, kn = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        res = solve(D, S, workspace=ws, timing_stride=stride, **kw)
        ws = res.workspace
        kms += res.kernel_ms
        kn += res.kernel_timed
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kms, kn, res


def roofline_of(which: str, kernel_name: str, per_launch: int, bytes_per_launch: int,
                kms: float, kn: int) -> dict:
    """Roofline object of a timed kernel: algorithmic bytes per launch (the
    state read and written once, data terms and capacity fields read once)
    over the mean launch duration from HIP events, against 8 TB/s."""
    avg_ms = kms / max(kn, 1) * per_launch
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    src_hash = _kernel_source_hash(kernel_name) if kernel_name in KERNEL_SOURCES else None
    traffic = _traffic(which, kernel_name, src_hash) if src_hash else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel_name, "kernel_avg_ms": round(avg_ms, 4),
            "iterations_per_launch": per_launch, "kernel_launches_timed": kn // per_launch,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "iteration_equivalent_GBs": round(achieved * per_launch, 1),
            "iteration_equivalent_frac": round(achieved * per_launch / HBM_PEAK_GBS, 4),
            "source_hash": src_hash}


def potts3d_leg(dev, n: int, steps: int = 2) -> dict:
    """Whole solves of the 256^3 Potts workload (8 labels, float32 state, 500
    iterations; two iterations per launch under AUTO), one warm-up, and the
    roofline of its kernel from HIP events around every 25th iteration."""
    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    p = synth.potts3d_voronoi(n=n, iters=POTTS_ITERS)
    D, S = _inputs(p, dev)
    kw = dict(c=p.c, tau=p.tau, iters=POTTS_ITERS, ndim=3, s_mode=p.s_mode, kernel="auto",
              final_energy=True, return_u=False, return_labels=True)
    elapsed, kms, kn, res = timed_solves(pf, pf.solve_potts, D, S, kw, steps, 1, 25)
    choice = _kernel_choice(pf, p, "fp32", "auto")
    per_launch = 2 if choice == "fused2" else 1
    V = p.voxels
    out = {"workload": f"potts3d_voronoi {n}x{n}x{n}, 8 labels, {POTTS_ITERS} iterations, "
                       f"c={p.c}, tau={p.tau}, fp32 state",
           "ms_per_solve": round(1e3 * elapsed / steps, 2),
           "voxel_label_its_per_s": V * p.n_node * POTTS_ITERS * steps / elapsed,
           "energy": res.energy, "gap": res.gap,
           "roofline": roofline_of("potts3d", _kernel_name(p, choice), per_launch,
                                   bytes_alg(p, "fp32") * V, kms, kn)}
    print(f"[bench] potts3d: {out['ms_per_solve']} ms/solve", file=sys.stderr, flush=True)
    return out


FULLFLOW_C, FULLFLOW_TAU = 1.0, 0.11     # frozen on the reference at reduced size


def fullflow_leg(dev, n: int) -> dict:
    """The full-flow counterpart against the pseudo-flow solver on the 256^3
    Potts workload (8 labels, float32, 500 iterations): device state bytes
    (each solver's workspace; the pseudo-flow two-pass layout and the
    ping-ponged layout of its AUTO kernel), per-iteration kernel time (HIP
    events around every iteration of a 20-iteration solve after a warm-up),
    algorithmic bytes per iteration, and the energy and relative gap each
    reaches in 500 iterations."""
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth
    p = synth.potts3d_voronoi(n=n, iters=POTTS_ITERS)
    D, S = _inputs(p, dev)
    kw = dict(ndim=3, s_mode=p.s_mode, final_energy=True, return_u=False, return_labels=False)
    ff = pf.solve_potts_fullflow(D, S, c=FULLFLOW_C, tau=FULLFLOW_TAU, iters=POTTS_ITERS, **kw)
    r = pf.solve_potts_fullflow(D, S, c=FULLFLOW_C, tau=FULLFLOW_TAU, iters=20,
                                workspace=ff.workspace, timing_stride=1, **kw)
    ff_ms = r.kernel_ms / max(r.kernel_timed, 1)
    ps = pf.solve_potts(D, S, c=p.c, tau=p.tau, iters=POTTS_ITERS, kernel="auto", **kw)
    pr = pf.solve_potts(D, S, c=p.c, tau=p.tau, iters=20, kernel="auto", workspace=ps.workspace,
                        timing_stride=1, **kw)
    ps_ms = pr.kernel_ms / max(pr.kernel_timed, 1)
    nl, nd, V = p.n_leaf, 3, p.voxels
    ff_bytes = pf.fullflow_workspace_bytes(p.shape, nl, nd)
    ps_two = pf.workspace_bytes(p.shape, nl, nl, nd, kernel="two_pass")
    ps_auto = pf.workspace_bytes(p.shape, nl, nl, nd, kernel="auto")
    d_bytes = 4 * nl * V
    ff_alg = 4 * (nl * (3 * nd + 5) + 3)          # bytes per voxel and iteration (two passes)
    out = {"workload": f"potts3d_voronoi {n}x{n}x{n}, 8 labels, fp32, {POTTS_ITERS} iterations",
           "fullflow": {"c": FULLFLOW_C, "tau": FULLFLOW_TAU, "state_bytes": ff_bytes,
                        "state_fields_per_voxel": (nd + 2) * nl + 1,
                        "ms_per_iter": round(ff_ms, 4), "alg_bytes_per_voxel_iter": ff_alg,
                        "alg_GBs": round(ff_alg * V / (ff_ms * 1e-3) / 1e9, 1),
                        "energy": ff.energy, "rel_gap": ff.gap / abs(ff.energy)},
           "pseudoflow": {"c": p.c, "tau": p.tau, "state_bytes_two_pass": ps_two,
                          "state_bytes_auto": ps_auto, "state_fields_per_voxel": (nd + 1) * nl,
                          "ms_per_iter": round(ps_ms, 4), "kernel": "k_fused2 (two iterations per launch)",
                          "energy": ps.energy, "rel_gap": ps.gap / abs(ps.energy)},
           "data_term_bytes": d_bytes,
           "state_saving": round(1 - ps_two / ff_bytes, 4),
           "saving_with_data_terms": round(1 - (ps_two + d_bytes) / (ff_bytes + d_bytes), 4),
           "speedup_per_iteration": round(ff_ms / ps_ms, 3)}
    print(f"[bench] full flow {ff_ms:.3f} ms/iter ({ff_bytes / 1e9:.2f} GB state), pseudo-flow "
          f"{ps_ms:.3f} ms/iter ({ps_two / 1e9:.2f} GB)", file=sys.stderr, flush=True)
    del D, S, ff, r, ps, pr
    torch.cuda.empty_cache()
    return out


def gap_leg(dev, p, storage: str) -> dict:
    """The primal-dual gap after every iteration of a whole solve (not
    timed): how often it increases and by how much relative to the energy."""
    import torch

    import paper_1501_07844_amd as pf
    D, S = _inputs(p, dev)
    solve = _solver(pf, p)
    r = solve(D, S, c=p.c, tau=p.tau, iters=p.iters, ndim=p.ndim, s_mode=p.s_mode,
              storage=storage, gap_every=1, gap_history_cap=p.iters, final_energy=False,
              return_u=False, return_labels=False)
    g = r.gap_history
    energy = r.energy
    inc = [(k + 1, (b - a) / abs(energy)) for k, (a, b) in enumerate(zip(g, g[1:])) if b > a]
    del D, S, r
    torch.cuda.empty_cache()
    return {"workload": f"{p.name} {'x'.join(map(str, p.shape[1:]))}", "storage": storage,
            "iterations": len(g), "gap_first": g[0] if g else None, "gap_last": g[-1] if g else None,
            "increases": len(inc), "first_increase_after": inc[0][0] if inc else None,
            "max_increase_rel_energy": max((d for _, d in inc), default=0.0),
            "last_gap_rel_energy": g[-1] / abs(energy) if g else None}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="Potts grid edge (default 256)")
    ap.add_argument("--kernel", default="auto",
                    choices=["auto", "two_pass", "fused", "fused2", "lds"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--counters", nargs="?", const="dagmf", default=None,
                    choices=["dagmf", "potts3d", "graphs"])
    ap.add_argument("--storage", default=HEADLINE_STORAGE, choices=["fp32", "bf16", "fp16"],
                    help="state type of the --counters dagmf program")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "z-slab design is not built", file=sys.stderr)
        return 2
    if args.counters:
        return counters_program(args.counters, args.kernel, args.storage)

    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth

    t0 = time.time()
    p = synth.dagmf_blobs()
    print(f"[bench] inputs {p.shape} x {p.n_leaf} leaves / {p.n_node} flows generated in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    D, S = _inputs(p, dev)
    B, Z, Y, X = p.shape
    V = B * Z * Y * X
    iters = p.iters
    kw = dict(c=p.c, tau=p.tau, iters=iters, ndim=3, s_mode=p.s_mode, storage=HEADLINE_STORAGE,
              kernel=args.kernel, final_energy=True, return_u=False, return_labels=True)
    solve = _solver(pf, p)
    elapsed, kms, kn, res = timed_solves(pf, solve, D, S, kw, args.steps, args.warmup, 10)
    ms_per_step = 1e3 * elapsed / args.steps
    value = V * p.n_node * iters * args.steps / elapsed
    print(f"[bench] dagmf {HEADLINE_STORAGE}: {ms_per_step:.1f} ms/step, energy {res.energy:.6e}, "
          f"gap {res.gap:.3e}", file=sys.stderr, flush=True)
    choice = _kernel_choice(pf, p, HEADLINE_STORAGE, args.kernel)
    roofline = roofline_of("dagmf", _kernel_name(p, choice), 1, bytes_alg(p, HEADLINE_STORAGE) * V,
                           kms, kn)
    headline_energy, headline_gap = res.energy, res.gap
    del D, S, res
    torch.cuda.empty_cache()

    out = {
        "metric": "voxel-label iterations/s + % HBM peak; FP32 vs BF16-storage at \u22641e-3 rel energy",
        "value": value, "unit": "voxel-label-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded random-blob phantom)",
        "config": {"workload": f"dagmf_blobs {Z}x{Y}x{X}, 4 parents x 12 leaves (16 flows), "
                               f"{iters} iterations, c={p.c}, tau={p.tau:.6g}, "
                               f"{HEADLINE_STORAGE} state, fp32 arithmetic, fp64 gap",
                   "voxels": V, "leaves": p.n_leaf, "label_nodes": p.n_node,
                   "iterations": iters, "storage": HEADLINE_STORAGE, "kernel": args.kernel,
                   "energy": headline_energy, "rel_gap": headline_gap / abs(headline_energy)},
        "roofline": roofline,
    }
    out["copy_peak"] = copy_leg(dev)
    # the same rate against what a plain device copy reaches on this GPU
    roofline["frac_of_copy_peak"] = round(roofline["achieved"] / out["copy_peak"]["GBs"], 4)
    torch.cuda.empty_cache()

    if not args.no_workloads:
        out["potts3d"] = potts3d_leg(dev, args.n)
        out["potts3d"]["roofline"]["frac_of_copy_peak"] = round(
            out["potts3d"]["roofline"]["achieved"] / out["copy_peak"]["GBs"], 4)
        torch.cuda.empty_cache()
        legs = []
        for make, kiters in ((lambda: synth.potts3d_voronoi(n=args.n), 20),
                             (synth.hmf_ellipsoids, 20), (lambda: p, 10),
                             (lambda: synth.ishikawa_levels(shape=(128, 256, 256), n_levels=7), 20)):
            q = make()
            for storage in ("fp32", "bf16", "fp16"):
                leg = kernel_leg(q, storage, kiters, dev)
                print(f"[bench] {leg['workload']} {storage}: {leg['ms_per_iter']} ms/iter, "
                      f"{leg['alg_GBs']} GB/s alg", file=sys.stderr, flush=True)
                legs.append(leg)
                torch.cuda.empty_cache()
            del q
        for i in range(0, len(legs), 3):
            for j in (1, 2):
                legs[i + j]["speedup_vs_fp32"] = round(legs[i]["ms_per_iter"] / legs[i + j]["ms_per_iter"], 3)
                legs[i + j]["rel_energy_vs_fp32"] = (abs(legs[i + j]["energy"] - legs[i]["energy"])
                                                     / abs(legs[i]["energy"]))
                legs[i + j]["rel_energy_full_vs_fp32"] = (
                    abs(legs[i + j]["energy_full"] - legs[i]["energy_full"]) / abs(legs[i]["energy_full"]))
        for leg in legs:
            leg["launch_frac_of_copy_peak"] = round(leg["launch_alg_GBs"] / out["copy_peak"]["GBs"], 4)
        out["workloads"] = legs
        # the metric's storage clause: bf16 state against fp32 per workload
        out["bf16_vs_fp32"] = [{"workload": g["workload"], "kernel": g["kernel"],
                                "speedup": g["speedup_vs_fp32"],
                                "rel_energy_at_budget": g["rel_energy_full_vs_fp32"],
                                "iterations": g["iterations_full"]}
                               for g in legs if g["storage"] == "bf16"]
        out["fullflow_vs_pseudoflow"] = fullflow_leg(dev, args.n)
        out["gap_behaviour"] = [gap_leg(dev, synth.potts3d_voronoi(n=args.n, iters=POTTS_ITERS), "fp32"),
                                gap_leg(dev, p, HEADLINE_STORAGE)]
        out["potts2d"] = potts2d_leg(dev)
        out["potts2d_batch"] = potts2d_batch_leg(dev)
        torch.cuda.empty_cache()
        out["ishikawa2d"] = ishikawa2d_leg(dev)

    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(dev)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)

    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(p, nz: int = 64, iters: int = 2) -> dict:
    """The float64 reference implementation, as it stands, on a bounded
    sample of the headline workload: its first `nz` z-planes (all of y and
    x, the same graph, data terms and capacities), `iters` iterations (about
    15 s on 16 host threads)."""
    import torch
    from oracle import pseudoflow_oracle as O

    nz = min(nz, p.shape[1])
    D = p.D[:, :, :nz]
    g = O.OracleGraph(p.graph.n_nodes, p.graph.parent, p.graph.child, p.graph.weight)
    n_threads = max(1, min(16, os.cpu_count() or 1))
    torch.set_num_threads(n_threads)
    t0 = time.perf_counter()
    O.solve_dagmf(D, p.S, p.s_mode, g, p.c, p.tau, iters, 3, history=False)
    dt = time.perf_counter() - t0
    V = D.shape[0] * nz * D.shape[3] * D.shape[4]
    return {"value": V * p.n_node * iters / dt, "unit": "voxel-label-iterations/s",
            "cores": n_threads, "kind": "oracle",
            "sample": f"first {nz} z-planes of the headline volume ({nz}x{D.shape[3]}x{D.shape[4]}, "
                      f"{p.n_leaf} leaves / {p.n_node} flows), {iters} iterations, float64, "
                      f"{dt:.1f}s"}


if __name__ == "__main__":
    sys.exit(main())
