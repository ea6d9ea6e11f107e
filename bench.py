"""Throughput of the pseudo-flow Potts solve on one MI355X.

Workload: Potts 3-D, 256^3 voxels, 8 labels, float32 state and arithmetic,
500 iterations (seeded 64-site Voronoi phantom, noise 0.15, Gaussian-NLL data
terms, S(x) = 0.3 exp(-|grad I|^2 / 0.01)).  One step is one complete solve:
initialisation, 500 iterations, the float64 energy/dual/gap evaluation and the
argmax export.  Inputs are resident in HBM before timing starts.

Prints one JSON line: voxel-label iterations per second (voxel-label = voxels
x non-source label nodes), the roofline of the per-iteration kernel measured
with HIP events inside the timed region, the same solve with bf16 state
storage, and the float64 reference implementation timed on a bounded sample
on the host.
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
ITERS = 500


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pf_kernels.hip", "pf_fused.hip", "pf_device.h", "pf_api.cpp", "pf_internal.h"):
        with open(os.path.join(ROOT, "paper_1501_07844_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, source_hash: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, only while the kernel sources are the ones it was taken on."""
    path = os.path.join(ROOT, "profiles", "traffic_potts3d_256.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid edge (default 256)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "two_pass", "fused"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "z-slab design is not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1501_07844_amd as pf
    from paper_1501_07844_amd import synth

    t0 = time.time()
    p = synth.potts3d_voronoi(n=args.n, iters=ITERS)
    print(f"[bench] inputs {p.shape} x {p.n_leaf} labels generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    D = torch.from_numpy(p.D).to(dev)
    S = torch.from_numpy(p.S).to(dev)
    B, Z, Y, X = p.shape
    V = B * Z * Y * X
    n_node = p.n_node
    kw = dict(c=p.c, tau=p.tau, iters=ITERS, ndim=3, s_mode="shared_field",
              kernel=args.kernel, final_energy=True, return_u=False, return_labels=True)

    def run_steps(storage, steps, warmup, timing_stride):
        ws = None
        res = None
        for _ in range(warmup):
            res = pf.solve_potts(D, S, storage=storage, workspace=ws, **kw)
            ws = res.workspace
        torch.cuda.synchronize()
        kernel_ms, kernel_n = 0.0, 0
        t_start = time.perf_counter()
        for _ in range(steps):
            res = pf.solve_potts(D, S, storage=storage, workspace=ws,
                                 timing_stride=timing_stride, **kw)
            ws = res.workspace
            kernel_ms += res.kernel_ms
            kernel_n += res.kernel_timed
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        return res, elapsed, kernel_ms, kernel_n

    res, elapsed, kms, kn = run_steps("fp32", args.steps, args.warmup, timing_stride=25)
    ms_per_step = 1e3 * elapsed / args.steps
    value = V * n_node * ITERS * args.steps / elapsed
    print(f"[bench] fp32: {ms_per_step:.1f} ms/step, energy {res.energy:.6e}, gap {res.gap:.3e}",
          file=sys.stderr, flush=True)

    fused = args.kernel == "fused" or (args.kernel == "auto" and res.workspace.numel() >
                                       pf.workspace_bytes(p.shape, p.n_leaf, n_node, 3, "fp32",
                                                          "two_pass"))
    kernel_name = "k_fused" if fused else "k_label+k_flow"
    bytes_alg = (2 * 4 * (p.n_leaf + 3 * n_node) + 4 * p.n_leaf + 4) * V   # per iteration
    avg_ms = kms / max(kn, 1)
    achieved = bytes_alg / (avg_ms * 1e-3) / 1e9
    src_hash = _kernel_source_hash()
    traffic = _traffic(kernel_name, src_hash)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_name, "kernel_avg_ms": round(avg_ms, 4),
                "kernel_launches_timed": kn, "algorithmic_bytes_per_launch": bytes_alg}

    out = {
        "metric": "voxel-label iterations/s (Potts 3D 256^3, 8 labels, fp32)",
        "value": value, "unit": "voxel-label-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Voronoi phantom)",
        "config": {"workload": f"potts3d_voronoi {Z}x{Y}x{X}, 8 labels, {ITERS} iterations, "
                               f"c={p.c}, tau={p.tau}, fp32 state",
                   "voxels": V, "labels": p.n_leaf, "iterations": ITERS,
                   "kernel": args.kernel, "energy": res.energy, "gap": res.gap},
        "roofline": roofline,
    }

    if not args.no_bf16:
        rb, eb, kmsb, knb = run_steps("bf16", args.steps, args.warmup, timing_stride=25)
        vb = V * n_node * ITERS * args.steps / eb
        out["bf16_storage"] = {
            "value": vb, "ratio_vs_fp32": vb / value,
            "rel_energy_vs_fp32": abs(rb.energy - res.energy) / abs(res.energy),
            "kernel_avg_ms": round(kmsb / max(knb, 1), 4), "ms_per_step": 1e3 * eb / args.steps}
        print(f"[bench] bf16: {1e3 * eb / args.steps:.1f} ms/step", file=sys.stderr, flush=True)

    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)

    print(json.dumps(out), flush=True)
    return 0


def adjoint_leg(dev, reps: int = 3) -> dict:
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
    return {"workload": f"diff_batch 16x256x256, 5 labels, {p.iters} iterations, checkpoint "
                        f"every {k}, fp32", "forward_ms": round(f, 3),
            "forward_recorded_ms": round(r, 3), "backward_ms": round(b, 3),
            "backward_over_forward": round(b / f, 3), "total_over_forward": round((r + b) / f, 3)}


def cpu_baseline(p) -> dict:
    """The float64 reference implementation, as it stands, on a bounded
    sample: the first 64 z-planes of the same volume, 5 iterations."""
    import torch
    from oracle import pseudoflow_oracle as O

    nz = min(64, p.shape[1])
    D = p.D[:, :, :nz]
    S = p.S[:, :nz]
    iters = 5
    torch.set_num_threads(max(1, min(16, os.cpu_count() or 1)))
    t0 = time.perf_counter()
    O.solve_potts(D, S, p.s_mode, p.c, p.tau, iters, 3, history=False)
    dt = time.perf_counter() - t0
    V = D.shape[0] * nz * D.shape[3] * D.shape[4]
    return {"value": V * p.n_node * iters / dt, "unit": "voxel-label-iterations/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"first {nz} z-planes ({nz}x{D.shape[3]}x{D.shape[4]}), {iters} iterations, "
                      f"float64, {dt:.1f}s"}


if __name__ == "__main__":
    sys.exit(main())
