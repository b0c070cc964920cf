#!/usr/bin/env python3
"""Benchmark of the hot path: forward element integration of the p=4 workload
(64x64x16 perturbed prism mesh, 131072 elements, 75 shape functions,
125 collapsed-Gauss points) on one MI355X.

A step is one pass of the forward integration over the whole batch (geometry
in FP64, fused coefficient blocks, the B^T W B contraction, load vector,
stores), inputs resident in HBM.  The headline form is the split-bf16 MFMA
form (bf16x3); the plain FP64, FP32 and fp16x3 forms are timed beside it, and
every form's relative error against the FP64 oracle on a sample of elements is
stated in the same line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-cal]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

from paper_1310_1194_amd import costmodel, meshgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}
FORMS = ["bf16x3", "fp16x3", "fp32", "fp64"]
HEADLINE = "bf16x3"
KERNEL_SOURCES = ["paper_1310_1194_amd/csrc/fwd_kernels.h", "paper_1310_1194_amd/csrc/device_common.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


def traffic_record(key: str):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/traffic.json),
    or None when absent or taken on other kernel sources."""
    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    rec = json.loads(path.read_text()).get(key)
    if not rec or rec.get("source_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(batch, p, budget_s: float, chunk: int = 4096):
    """The oracle on the host's cores over the first elements of the workload,
    chunk by chunk until about `budget_s` seconds have been spent."""
    import oracle
    done, spent, first = 0, 0.0, None
    while done < batch.ne and (spent < budget_s or done == 0):
        sub = batch.subset(np.arange(done, min(batch.ne, done + chunk)))
        t0 = time.perf_counter()
        A, b, _ = oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
        spent += time.perf_counter() - t0
        if first is None:
            first = (A, b)
        done += sub.ne
    return done / spent, done, spent, oracle.max_threads(), first


def rel_err(got, ref):
    got = np.asarray(got, np.float64).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    per = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), float(per.max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="p4_131072")
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (CPU baseline and errors)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-cal", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the element batch "
                                   "is independent per element and is not sharded here",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1310_1194_amd as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = meshgen.WORKLOADS[args.workload]
    p = w["p"]
    n, q = costmodel.nshp(p), costmodel.nq(p)
    batch = meshgen.workload(args.workload)
    ne = batch.ne
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))
    forms = [f for f in args.forms.split(",") if f]
    assert HEADLINE in forms

    if args.copy_cal:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    results = {}
    A = b = None
    for form in forms:
        dt = torch.float64 if form == "fp64" else torch.float32
        del A, b
        torch.cuda.empty_cache()
        A = torch.empty((ne, n, n), dtype=dt, device=dev)
        b = torch.empty((ne, n), dtype=dt, device=dev)
        tile_ms = None
        if not args.no_tune:
            tile_ms = F.autotune(*X, p, form, A, b, reps=2)
        tile = F.tile_describe(p, form, F.tile_get(p, form))
        for _ in range(args.warmup):
            F.integrate_raw(*X, p, form, A=A, b=b)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(args.steps):
            F.integrate_raw(*X, p, form, A=A, b=b)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
        ms = float(np.mean(per))
        sample_idx = torch.arange(min(ne, 4096), device=dev)
        results[form] = dict(ms_per_step=wall * 1e3 / args.steps, kernel_ms_mean=ms,
                             kernel_ms_min=float(np.min(per)), tile=tile, tune_ms=tile_ms,
                             elements_per_s=ne * args.steps / wall,
                             A_sample=A[sample_idx].cpu().numpy(), b_sample=b[sample_idx].cpu().numpy())
        print(f"[bench] {form}: {ms:.3f} ms/launch (min {np.min(per):.3f}), tile {tile}", file=sys.stderr, flush=True)

    fdom = costmodel.f_dom(p)
    for form, r in results.items():
        es = costmodel.out_bytes(p, 8 if form == "fp64" else 4)
        alg_bytes = ne * (costmodel.INPUT_BYTES + es)
        r["gflops"] = fdom * ne / (r["kernel_ms_mean"] * 1e-3) / 1e9
        r["tflops_frac_of_peak"] = r["gflops"] / 1e3 / PEAK_TFLOPS[form]
        r["hbm_gbs_algorithmic"] = alg_bytes / (r["kernel_ms_mean"] * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu:
        rate, done, spent, cores, (Ar, br) = cpu_baseline(batch, p, args.cpu_budget)
        cpu = {"value": rate, "unit": "elements/s", "cores": cores, "kind": "oracle",
               "sample": f"first {done} of the {ne} elements of {args.workload} "
                         f"({spent:.1f} s, FP64, OpenMP over elements)",
               "cpu": platform.processor() or platform.machine()}
        m = Ar.shape[0]
        for form, r in results.items():
            gA, mA = rel_err(r["A_sample"][:m], Ar)
            gb, mb = rel_err(r["b_sample"][:m], br)
            r["rel_err_A"] = gA
            r["rel_err_A_max_elem"] = mA
            r["rel_err_b"] = gb
            r["err_sample"] = m

    h = results[HEADLINE]
    traffic = traffic_record(f"fwd:{HEADLINE}:{args.workload}")
    roofline = {"bound": "mfma", "achieved": h["gflops"] / 1e3, "peak": PEAK_TFLOPS[HEADLINE],
                "unit": "TFLOP/s", "frac": h["gflops"] / 1e3 / PEAK_TFLOPS[HEADLINE],
                "traffic": traffic,
                "kernel_ms": h["kernel_ms_mean"], "flops_per_launch": fdom * ne,
                "note": "algorithmic flops 8 n^2 nq per element (one product per entry; "
                        "the split form issues three bf16 products)"}
    forms_out = {}
    for form, r in results.items():
        forms_out[form] = {k: (float(f"{v:.5g}") if isinstance(v, float) else v) for k, v in r.items()
                           if not k.endswith("_sample")}
    line = {
        "metric": "elements/s + GFLOP/s (roofline %) at p=4, plain FP64 vs MFMA form at stated error",
        "value": h["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3 (split bf16 MFMA, fp32 accumulate, fp64 geometry)",
        "data": "synthetic (seeded perturbed prism mesh and coefficients)",
        "config": {"workload": args.workload, "p": p, "ne": ne, "nshp": n, "nq": q,
                   "mesh": f"{w['nx']}x{w['ny']}x{w['nz']}", "perturbation": w["amp"], "seed": w["seed"],
                   "form": HEADLINE, "parallelism": "single GPU"},
        "gflops": h["gflops"],
        "speedup_vs_fp64_gpu": results["fp64"]["kernel_ms_mean"] / h["kernel_ms_mean"] if "fp64" in results else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms_out,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
