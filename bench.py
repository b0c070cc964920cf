#!/usr/bin/env python3
"""Benchmark of the hot path: forward element integration of the p=4 workload
(64x64x16 perturbed prism mesh, 131072 elements, 75 shape functions,
125 collapsed-Gauss points) on one MI355X.

A step is one pass of the forward integration over the whole batch (geometry
in FP64, fused coefficient blocks, the B^T W B contraction, load vector,
stores), inputs resident in HBM.  The headline form is the split-bf16 MFMA
form (bf16x3); the plain FP64, FP32 and fp16x3 forms are timed beside it, and
every form's relative error against the FP64 oracle on a sample of elements is
stated in the same line.  The default run (mode "suite") adds, as keys of
`configs` in the same line, every other configured workload in its own launch
configuration: p = 1 at 4096 and 524288 elements, the mixed-degree batch
replayed from a HIP graph, the p = 3 adjoint, the p = 7 forward and
adjoint, hexahedra at p = 4..7 (sum factorisation in three directions beside
the contraction along xi3 only), tetrahedra at p = 4 (FP64 and FP32 from
reference matrices; FP32 heads the tetrahedral lines, where the split forms
integrate point by point and are slower), and the paper's own term (Laplace) on its
quadrature at its batch sizes for p = 1..7, each with its roofline, its error
against the oracle and its CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-cal]
                    [--mode suite|forward|fields|hex|tet|adjoint|mixed|assemble|laplace]
                    [--workload NAME] [--forms LIST] [--hex-ps LIST]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
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
DTYPE_DESC = {"bf16x3": "bf16x3 (split bf16 MFMA, fp32 accumulate, fp64 geometry)",
              "fp16x3": "fp16x3 (split fp16 MFMA, fp32 accumulate, fp64 geometry)",
              "fp32": "fp32 (fp32 MFMA, fp64 geometry)", "fp64": "fp64"}
KERNEL_SOURCES = ["paper_1310_1194_amd/csrc/fwd_kernels.h", "paper_1310_1194_amd/csrc/fwd_staged.h",
                  "paper_1310_1194_amd/csrc/fwd_pipe.h", "paper_1310_1194_amd/csrc/fwd_valu.h",
                  "paper_1310_1194_amd/csrc/fwd_fact.h", "paper_1310_1194_amd/csrc/fwd_ymfma.h",
                  "paper_1310_1194_amd/csrc/fwd_registry.h", "paper_1310_1194_amd/csrc/fwd_bf16.hip",
                  "paper_1310_1194_amd/csrc/fwd_f16.hip", "paper_1310_1194_amd/csrc/fwd_f32.hip",
                  "paper_1310_1194_amd/csrc/fwd_f64.hip",
                  "paper_1310_1194_amd/csrc/device_common.h", "paper_1310_1194_amd/csrc/tables.cpp",
                  "paper_1310_1194_amd/csrc/fwd_hsf.h", "paper_1310_1194_amd/csrc/hex_factors.h",
                  "paper_1310_1194_amd/csrc/fwd_hex.hip", "paper_1310_1194_amd/csrc/fwd_tref.h",
                  "paper_1310_1194_amd/csrc/fwd_tet.hip"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


def traffic_record(key: str, tile: str):
    """HBM bytes per launch of the compiled variant `tile` measured by rocprofv3
    counters (profiles/traffic.json), or None when absent or taken on other
    kernel sources."""
    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    rec = json.loads(path.read_text()).get(key)
    if not rec or rec.get("source_sha") != kernel_source_sha():
        return None
    return rec.get("tiles", {}).get(tile)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def single_thread_rate(fn, m: int):
    """Elements/s of fn(m) with the oracle on one thread (its OpenMP pool
    restored afterwards)."""
    import oracle
    nt = oracle.max_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        fn(m)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(nt)
    return {"value": m / dt, "unit": "elements/s", "cores": 1, "sample": f"first {m} elements ({dt:.2f} s)"}


def cpu_baseline(batch, p, budget_s: float, chunk: int = 4096, fields=None, rule=None, kind=None):
    """The oracle on the host's cores over the first elements of the workload,
    chunk by chunk until about `budget_s` seconds have been spent (with vertex
    coefficient fields when `fields` = (Dv, betav, cv, fv) is given)."""
    import oracle
    done, spent, first = 0, 0.0, None
    while done < batch.ne and (spent < budget_s or done == 0):
        sl = np.arange(done, min(batch.ne, done + chunk))
        sub = batch.subset(sl)
        t0 = time.perf_counter()
        if kind:
            fn = oracle.integrate_hex if kind == "hex" else oracle.integrate_tet
            A, b, _ = fn(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
        elif fields is None:
            A, b, _ = oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, rule=rule)
        else:
            A, b, _ = oracle.integrate_fields(p, sub.coords, *[np.ascontiguousarray(a[sl]) for a in fields],
                                              rule=rule)
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


def graph_replay_ms(fn, n):
    """Mean time per launch of n launches of fn captured in one HIP graph
    (torch.cuda.CUDAGraph) and replayed, events around each replay."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(n):
            fn()
    g.replay()
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * n)


def timed(fn, steps, warmup, stream=None):
    """Warm up, then time `steps` calls with HIP events on the launch stream
    (bracketed by device synchronisation); returns (mean, min) ms per call and
    the wall-clock ms per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = stream or torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return float(np.mean(per)), float(np.min(per)), wall


def fmt(d):
    return {k: (float(f"{v:.5g}") if isinstance(v, float) else (fmt(v) if isinstance(v, dict) else v))
            for k, v in d.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="suite",
                    choices=["suite", "forward", "fields", "hex", "tet", "adjoint", "mixed", "assemble", "laplace"])
    ap.add_argument("--workload", default=None)
    ap.add_argument("--hex-ps", default=None, help="--mode hex: degrees (default 4,5,6,7)")
    ap.add_argument("--rule", default="collapsed", choices=["collapsed", "symmetric"],
                    help="quadrature rule of the forward, fields and adjoint modes")
    ap.add_argument("--sc", action="store_true",
                    help="forward/fields: time the variant that computes shape functions at each point "
                         "(the paper's SC strategy) instead of autotuning over the table-reading ones; "
                         "FP64 and FP32 forms")
    ap.add_argument("--forms", default=None)
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
    if args.mode == "suite":
        line = bench_suite(args)
    elif args.mode == "adjoint":
        line = bench_adjoint(args)
    elif args.mode == "mixed":
        line = bench_mixed(args)
    elif args.mode == "assemble":
        line = bench_assemble(args)
    elif args.mode == "laplace":
        line = bench_laplace(args)
    elif args.mode == "hex":
        line = bench_hex(args)
    else:
        line = bench_forward(args, fields=args.mode == "fields",
                             kind=args.mode if args.mode in ("hex", "tet") else None)
    print(json.dumps(line))


def bench_forward(args, fields=False, kind=None, err_idx=None, cpu_budget=None):
    """Forward integration; with `fields` the coefficients are vertex fields
    evaluated at every point (feint_integrate_fields); with `kind` "hex" or
    "tet" the elements are hexahedra or tetrahedra (feint_integrate_hex/_tet)."""
    other_elem = kind is not None
    args.workload = args.workload or {"hex": "hex_p4_65536", "tet": "tet_p4_393216"}.get(kind, "p4_131072")
    args.forms = args.forms or ("fp64,fp32" if args.sc else ",".join(FORMS))
    import torch
    import paper_1310_1194_amd as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = meshgen.WORKLOADS[args.workload]
    p = w["p"]
    rule = args.rule
    n, q = costmodel.nshp(p), costmodel.nq(p, rule)
    if other_elem:
        if rule != "collapsed" or args.sc or fields:
            raise SystemExit(f"{kind}: its own Gauss rule, table-reading kernels, element constants")
        n, q = F.ELEMENTS[kind][1](p), F.ELEMENTS[kind][2](p)
    batch = meshgen.workload(args.workload)
    ne = batch.ne
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    vf = meshgen.vertex_fields(ne, 1000 + w["seed"]) if fields else None
    if other_elem:
        X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))

        def integrate(*a, A=None, b=None, rule=None):
            return F.integrate_elem_raw(kind, *a, A=A, b=b)
    elif fields:
        X = (t(batch.coords),) + tuple(t(a) for a in vf)
        integrate = F.integrate_fields_raw
    else:
        X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))
        integrate = F.integrate_raw
    forms = [f for f in args.forms.split(",") if f]
    # tetrahedra: the FP32 reference-matrix GEMM is faster than the split forms
    # (which integrate point by point) at a smaller error, so it heads their line
    hform = "fp32" if kind == "tet" else HEADLINE
    headline = hform if hform in forms else forms[0]
    if args.sc and not set(forms) <= {"fp64", "fp32"}:
        raise SystemExit("--sc: the SC variants are compiled for the fp64 and fp32 forms")

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
        if args.sc:
            sc = [t for t in range(F.tile_count(p, form, rule=rule))
                  if re.fullmatch(r"\d+x\d+c(o2)?", F.tile_describe(p, form, t, rule=rule))]
            if not sc:
                raise SystemExit(f"no SC variant compiled for p={p} form={form}")
            F.tile_set(p, form, sc[0], rule=rule)
        elif not args.no_tune:
            if other_elem:
                tile_ms = F.elem_autotune(kind, *X, p, form, A, b, reps=2)
            elif fields:
                tile_ms = F.autotune_fields(*X, p, form, A, b, reps=2, rule=rule)
            else:
                tile_ms = F.autotune(*X, p, form, A, b, reps=2, rule=rule)
        if other_elem:
            tile = F.elem_tile_describe(kind, p, form, F.elem_tile_get(kind, p, form))
        else:
            tile = F.tile_describe(p, form, F.tile_get(p, form, rule=rule), rule=rule)
        for _ in range(args.warmup):
            integrate(*X, p, form, A=A, b=b, rule=rule)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(args.steps):
            integrate(*X, p, form, A=A, b=b, rule=rule)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
        ms = float(np.mean(per))
        sample_idx = torch.from_numpy(err_idx).to(dev) if err_idx is not None else torch.arange(min(ne, 4096), device=dev)
        results[form] = dict(ms_per_step=wall * 1e3 / args.steps, kernel_ms_mean=ms,
                             kernel_ms_min=float(np.min(per)), tile=tile, tune_ms=tile_ms,
                             elements_per_s=ne * args.steps / wall,
                             A_sample=A[sample_idx].cpu().numpy(), b_sample=b[sample_idx].cpu().numpy())
        if ne <= 8192 and not other_elem and not fields:
            # a launch this small is bound by its submission: the same launches
            # replayed from a HIP graph show what the kernel itself takes
            results[form]["graph_replay_ms_per_launch"] = graph_replay_ms(
                lambda: integrate(*X, p, form, A=A, b=b, rule=rule), 32)
        print(f"[bench] {form}: {ms:.3f} ms/launch (min {np.min(per):.3f}), tile {tile}", file=sys.stderr, flush=True)

    fdom = 8 * n * n * q if other_elem else costmodel.f_dom(p, rule)
    in_bytes = (8 * (3 * F.ELEMENTS[kind][0] + 9 + 3 + 1 + 1) if other_elem else
                costmodel.FIELD_INPUT_BYTES if fields else costmodel.INPUT_BYTES)
    for form, r in results.items():
        es = (n * n + n) * (8 if form == "fp64" else 4)
        alg_bytes = ne * (in_bytes + es)
        # gflops: the B^T W B formulation's work (F_dom) per second, comparable across
        # kernels and with the paper; gflops_alg: the work of the algorithm the chosen
        # tile runs (fewer flops for the triangle-point contraction), the roofline numerator
        if costmodel.is_kf_tile(r["tile"]):       # prisms and hexahedra: factorised along the third coordinate
            r["alg_flops_per_element"] = (costmodel.f_factored_zfirst(n, p + 1, q) if costmodel.is_zfirst_tile(r["tile"])
                                          else costmodel.f_factored(n, p + 1, q))
        elif kind == "tet" and costmodel.is_tet_ref_tile(r["tile"]):   # the reference-matrix GEMM
            r["alg_flops_per_element"] = costmodel.f_tet_reference(n)
        else:
            r["alg_flops_per_element"] = fdom
        r["fdom_equiv_gflops"] = fdom * ne / (r["kernel_ms_mean"] * 1e-3) / 1e9
        r["gflops_alg"] = r["alg_flops_per_element"] * ne / (r["kernel_ms_mean"] * 1e-3) / 1e9
        r["tflops_frac_of_peak"] = r["gflops_alg"] / 1e3 / PEAK_TFLOPS[form]
        r["hbm_gbs_algorithmic"] = alg_bytes / (r["kernel_ms_mean"] * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu:
        import oracle
        orule = None if rule == "collapsed" else rule
        budget = args.cpu_budget if cpu_budget is None else cpu_budget
        chunk = 4096 if p < 6 else 256
        rate, done, spent, cores, (Ar, br) = cpu_baseline(batch, p, budget, chunk=chunk, fields=vf, rule=orule,
                                                          kind=kind)

        def one(m):
            sub = batch.subset(np.arange(min(m, ne)))
            if kind:
                fn = oracle.integrate_hex if kind == "hex" else oracle.integrate_tet
                fn(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
            elif vf is not None:
                oracle.integrate_fields(p, sub.coords, *[np.ascontiguousarray(a[:sub.ne]) for a in vf], rule=orule)
            else:
                oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, rule=orule)
        cpu = {"value": rate, "unit": "elements/s", "cores": cores, "kind": "oracle",
               "sample": f"first {done} of the {ne} elements of {args.workload} "
                         f"({spent:.1f} s, FP64, OpenMP over elements)",
               "cpu": cpu_model(),
               "single_thread": single_thread_rate(one, min(ne, 1024 if p <= 4 else 64 >> max(0, p - 5)))}
        if err_idx is not None:       # the sampled elements, one by one
            sub = batch.subset(err_idx)
            if kind:
                fn = oracle.integrate_hex if kind == "hex" else oracle.integrate_tet
                Ar, br, _ = fn(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
            else:
                Ar, br, _ = oracle.integrate(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, rule=orule)
        m = Ar.shape[0]
        for form, r in results.items():
            gA, mA = rel_err(r["A_sample"][:m], Ar)
            gb, mb = rel_err(r["b_sample"][:m], br)
            r["rel_err_A"] = gA
            r["rel_err_A_max_elem"] = mA
            r["rel_err_b"] = gb
            r["rel_err_b_max_elem"] = mb
            r["err_sample"] = m if err_idx is None else f"{m} elements (every {ne // m}th)"

    h = results[headline]
    rkey = "" if rule == "collapsed" else ":" + rule
    traffic = traffic_record(f"{kind or ('fields' if fields else 'fwd')}:{headline}:{args.workload}{rkey}",
                             results[headline]["tile"])
    es = 8 if headline == "fp64" else 4
    alg_bytes = ne * (in_bytes + (n * n + n) * es)
    # bound = the larger ideal time: MFMA work (three products for a split
    # form) at the dtype's dense peak, or the algorithmic bytes at HBM peak
    products = 3 if headline in ("bf16x3", "fp16x3") else 1
    falg = h["alg_flops_per_element"]
    t_mfma = products * falg * ne / (PEAK_TFLOPS[headline] * 1e12)
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    if t_hbm > t_mfma:
        roofline = {"bound": "hbm", "achieved": h["hbm_gbs_algorithmic"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": h["hbm_gbs_algorithmic"] / HBM_PEAK_GBS}
    else:
        roofline = {"bound": "mfma", "achieved": h["gflops_alg"] / 1e3, "peak": PEAK_TFLOPS[headline],
                    "unit": "TFLOP/s", "frac": h["gflops_alg"] / 1e3 / PEAK_TFLOPS[headline]}
    npad, nqp = (n + 15) // 16 * 16, (q + 7) // 8 * 8
    kf = costmodel.is_kf_tile(h["tile"])
    tref = kind == "tet" and costmodel.is_tet_ref_tile(h["tile"])
    hw_flops = (products * costmodel.kf_mfma_flops(p, rule, n, q) * ne if kf else
                costmodel.tet_reference_mfma_flops(n) * ne if tref else
                products * 8.0 * npad * npad * (nqp if products == 3 else q) * ne)
    roofline.update({"traffic": traffic, "kernel_ms": h["kernel_ms_mean"], "flops_per_launch": falg * ne,
                     "fdom_per_launch": fdom * ne,
                     "hw_mfma_frac": hw_flops / (h["kernel_ms_mean"] * 1e-3) / (PEAK_TFLOPS[headline] * 1e12),
                     "alg_bytes_per_launch": alg_bytes,
                     "note": ("algorithmic flops of the triangle-point contraction with the line-point sums "
                              "first per element (8 n^2 nij + 26 (p+1)^3 nij + 32 (p+1) n nij)"
                              if kf and costmodel.is_zfirst_tile(h["tile"]) else
                              "algorithmic flops of the triangle-point contraction per element "
                              "(8 n^2 nij + 8 (p+1)^2 nij n + 24 nq ntri + 12 nq n)" if kf else
                              "algorithmic flops of the reference-matrix GEMM per element (26 n^2 + n)" if tref else
                              "algorithmic flops 8 n^2 nq per element (one product per entry; "
                              "a split form issues three products)") + "; bytes %d in + (n^2+n) outputs" % in_bytes})
    forms_out = {}
    for form, r in results.items():
        forms_out[form] = {k: (float(f"{v:.5g}") if isinstance(v, float) else v) for k, v in r.items()
                           if k not in ("A_sample", "b_sample")}
    line = {
        "metric": "elements/s + GFLOP/s (roofline %) at p=4, plain FP64 vs MFMA form at stated error"
                  + (" (coefficients varying in space, given at the vertices)" if fields else "")
                  + ({"hex": " (hexahedral elements)", "tet": " (tetrahedral elements)"}.get(kind, "")),
        "value": h["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_DESC[headline],
        "data": "synthetic (seeded perturbed prism mesh and coefficients)",
        "config": {"workload": args.workload + ("+vertex_fields" if fields else "")
                   + ("+symmetric_rule" if rule != "collapsed" else "") + ("+sc" if args.sc else ""),
                   "p": p, "ne": ne, "rule": rule, "shape_functions": "computed per point" if args.sc else "tables",
                   "element": {"hex": "hexahedron", "tet": "tetrahedron"}.get(kind, "prism"),
                   "nshp": n, "nq": q, "coefficients": "vertex fields" if fields else "element constants",
                   "mesh": f"{w['nx']}x{w['ny']}x{w['nz']}", "perturbation": w["amp"], "seed": w["seed"],
                   "form": headline, "parallelism": "single GPU"},
        "fdom_equiv_gflops": h["fdom_equiv_gflops"],
        "speedup_vs_fp64_gpu": results["fp64"]["kernel_ms_mean"] / h["kernel_ms_mean"] if "fp64" in results else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms_out,
        "device": torch.cuda.get_device_name(0),
    }
    return line


SUMMARY_DROP = ("n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "data", "metric")


def summarise(line):
    """A workload's line without the keys the enclosing line already states."""
    return {k: v for k, v in line.items() if k not in SUMMARY_DROP}


def bench_suite(args):
    """The default run: the p = 4 headline (all four forms) and, as keys of the
    same line, every other configured workload in its own launch
    configuration: p = 1 at 4096 elements (latency-bound) and at 524288 (HBM),
    the mixed-degree batch replayed from a HIP graph, the p = 3 adjoint,
    the p = 7 forward (split forms beside FP32 and FP64) and adjoint,
    hexahedra at p = 4..7, tetrahedra at p = 4 and the paper's Laplace sweep."""
    import copy
    import torch

    def sub(**kw):
        a = copy.copy(args)
        for k, v in kw.items():
            setattr(a, k, v)
        return a
    steps, warm = min(args.steps, 10), min(args.warmup, 3)
    budget = min(args.cpu_budget, 4.0)
    line = bench_forward(sub(workload="p4_131072", forms=None))
    cfg = {}
    stage = lambda name: print(f"[bench] suite: {name}", file=sys.stderr, flush=True)
    stage("p1_4096")
    cfg["p1_4096"] = summarise(bench_forward(sub(workload="p1_4096", forms="fp64,fp32"),
                                             err_idx=np.arange(4096), cpu_budget=budget))
    torch.cuda.empty_cache()
    stage("p1_524288")
    cfg["p1_524288"] = summarise(bench_forward(sub(workload="p1_524288", forms="fp64,fp32"), cpu_budget=budget))
    torch.cuda.empty_cache()
    stage("mixed_262144")
    cfg["mixed_262144"] = summarise(bench_mixed(sub(workload="mixed_262144", forms="fp32", steps=steps,
                                                    warmup=warm)))
    torch.cuda.empty_cache()
    stage("adj_p3_131072")
    cfg["adj_p3_131072"] = summarise(bench_adjoint(sub(workload="adj_p3_131072", forms="fp32,fp64", steps=steps,
                                                       warmup=warm, cpu_budget=budget)))
    torch.cuda.empty_cache()
    stage("p7_16384")
    cfg["p7_16384"] = summarise(bench_forward(sub(workload="p7_16384", forms="bf16x3,fp16x3,fp32,fp64",
                                                  steps=steps, warmup=warm),
                                              err_idx=np.arange(0, 16384, 16), cpu_budget=budget))
    torch.cuda.empty_cache()
    stage("adj_p7_16384")
    cfg["adj_p7_16384"] = summarise(bench_adjoint(sub(workload="p7_16384", forms="fp32,fp64", steps=steps,
                                                      warmup=warm, cpu_budget=budget)))
    torch.cuda.empty_cache()
    stage("hex_p4_p7")
    cfg["hex_p4_p7"] = summarise(bench_hex(sub(workload=None, forms="fp64,fp32", steps=steps, warmup=warm)))
    torch.cuda.empty_cache()
    stage("tet_p4_393216")
    cfg["tet_p4_393216"] = summarise(bench_forward(sub(workload="tet_p4_393216", forms="fp64,fp32", steps=steps,
                                                       warmup=warm, rule="collapsed", sc=False),
                                                   kind="tet", err_idx=np.arange(0, 393216, 96),
                                                   cpu_budget=min(budget, 2.0)))
    torch.cuda.empty_cache()
    stage("laplace_paper_sweep")
    cfg["laplace_paper_sweep"] = summarise(bench_laplace(sub(workload=None, forms="fp32", steps=steps,
                                                             warmup=warm)))
    line["configs"] = cfg
    return line


HEX_WORKLOADS = {4: "hex_p4_65536", 5: "hex_p5_16384", 6: "hex_p6_8192", 7: "hex_p7_2048"}
VEC_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def bench_hex(args):
    """Hexahedra at p = 4..7 (hex_p4_65536, hex_p5_16384, hex_p6_8192,
    hex_p7_2048; element matrices of 4.3 to 8.2 GB in FP64), FP64 and FP32: the
    sum factorisation in all three directions next to the contraction
    factorised along xi3 only, each in its fastest compiled variant, and a
    device fill of the same output buffer (the practical write ceiling).  Per
    kernel: mean launch time (HIP events on the launch stream), elements/s, the
    flops of its own algorithm per second, and its roofline -- the larger of
    (own flops at the peak of the unit it runs on: FP64/FP32 vector for the sum
    factorisation, the matrix cores for the xi3 contraction) and (input bytes +
    element matrix and load vector written, at the HBM peak), as a fraction of
    the measured time; errors against the oracle on a spread sample."""
    import torch
    import paper_1310_1194_amd as F
    from paper_1310_1194_amd import costmodel
    dev = torch.device("cuda:0")
    ps = [int(x) for x in (args.hex_ps or "4,5,6,7").split(",")]
    forms = [f for f in (args.forms or "fp64,fp32").split(",") if f]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    in_bytes = 8 * (24 + 9 + 3 + 1 + 1)
    out, head = {}, None
    if args.copy_cal:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for p in ps:
        name = HEX_WORKLOADS[p]
        batch = meshgen.workload(name)
        ne, n = batch.ne, (p + 1) ** 3
        X = tuple(t(a) for a in (batch.coords, batch.D, batch.beta, batch.c, batch.f))
        nsamp = {4: 256, 5: 128, 6: 64, 7: 64}[p]
        idx = np.unique(np.linspace(0, ne - 1, nsamp).astype(np.int64))
        ref = None
        if not args.no_cpu:
            import oracle
            sub = batch.subset(idx)
            Ar, br, _ = oracle.integrate_hex(p, sub.coords, sub.D, sub.beta, sub.c, sub.f)
            ref = (Ar, br)
        per_p = {"workload": name, "ne": ne, "nshp": n, "nq": n}
        for form in forms:
            dt = torch.float64 if form == "fp64" else torch.float32
            A = torch.empty((ne, n, n), dtype=dt, device=dev)
            b = torch.empty((ne, n), dtype=dt, device=dev)
            cnt = F.elem_tile_count("hex", p, form)
            descs = [F.elem_tile_describe("hex", p, form, k) for k in range(cnt)]
            kinds = {"sumfact": [k for k in range(cnt) if costmodel.is_sf_tile(descs[k])],
                     "xi3": [k for k in range(cnt) if costmodel.is_kf_tile(descs[k])]}

            def timed(tile, steps, warm):
                F.elem_tile_set("hex", p, form, tile)
                for _ in range(warm):
                    F.integrate_elem_raw("hex", *X, p, form, A=A, b=b)
                torch.cuda.synchronize()
                stream = torch.cuda.current_stream()
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
                ev[0].record(stream)
                for k in range(steps):
                    F.integrate_elem_raw("hex", *X, p, form, A=A, b=b)
                    ev[k + 1].record(stream)
                torch.cuda.synchronize()
                return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]

            # the practical write ceiling: a device fill of the same output buffer
            A.zero_()
            torch.cuda.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record()
            for _ in range(3):
                A.zero_()
            f1.record()
            torch.cuda.synchronize()
            fill_gbs = A.numel() * A.element_size() / (f0.elapsed_time(f1) / 3 * 1e-3) / 1e9
            res = {"fill_gbs": round(fill_gbs, 1)}
            for kname, tiles in kinds.items():
                if not tiles:
                    continue
                best = min(tiles, key=lambda k: float(np.min(timed(k, 4, 1))))
                per = timed(best, args.steps, args.warmup)
                ms = float(np.mean(per))
                es = 8 if form == "fp64" else 4
                nbytes = ne * (in_bytes + (n * n + n) * es)
                if kname == "sumfact":
                    flops, peak, unit = costmodel.f_hex_sumfact(p) * ne, VEC_PEAK_TFLOPS[form], "alu"
                else:
                    flops, peak, unit = costmodel.f_factored(n, p + 1, n) * ne, PEAK_TFLOPS[form], "mfma"
                t_alu, t_hbm = flops / (peak * 1e12), nbytes / (HBM_PEAK_GBS * 1e9)
                bound = "hbm" if t_hbm >= t_alu else unit
                r = {"tile": descs[best], "kernel_ms_mean": ms, "kernel_ms_min": float(np.min(per)),
                     "elements_per_s": ne / (ms * 1e-3), "alg_flops_per_element": flops / ne,
                     "gflops_alg": flops / (ms * 1e-3) / 1e9,
                     "fdom_equiv_gflops": 8.0 * n * n * n * ne / (ms * 1e-3) / 1e9,
                     "hbm_gbs_algorithmic": nbytes / (ms * 1e-3) / 1e9,
                     "roofline": {"bound": bound, "peak": HBM_PEAK_GBS if bound == "hbm" else peak,
                                  "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                                  "achieved": (nbytes / (ms * 1e-3) / 1e9 if bound == "hbm"
                                               else flops / (ms * 1e-3) / 1e12),
                                  "frac": max(t_alu, t_hbm) / (ms * 1e-3),
                                  "alu_frac": t_alu / (ms * 1e-3), "hbm_frac": t_hbm / (ms * 1e-3),
                                  "write_frac_of_fill": n * n * es * ne / (ms * 1e-3) / 1e9 / fill_gbs}}
                if kname == "sumfact":
                    r["roofline"]["traffic"] = traffic_record(f"hexsf:{form}:{name}", descs[best])
                if ref is not None:
                    ti = torch.from_numpy(idx).to(dev)
                    gA, mA = rel_err(A[ti].cpu().numpy(), ref[0])
                    gb, _ = rel_err(b[ti].cpu().numpy(), ref[1])
                    r.update(rel_err_A=gA, rel_err_A_max_elem=mA, rel_err_b=gb, err_sample=len(idx))
                res[kname] = {k: (float(f"{v:.5g}") if isinstance(v, float) else v) for k, v in r.items()}
                print(f"[bench] hex p={p} {form} {kname} {descs[best]}: {ms:.3f} ms", file=sys.stderr, flush=True)
            F.elem_tile_set("hex", p, form, 0)
            if "sumfact" in res and "xi3" in res:
                res["speedup_vs_xi3"] = round(res["xi3"]["kernel_ms_mean"] / res["sumfact"]["kernel_ms_mean"], 3)
            per_p[form] = res
            del A, b
            torch.cuda.empty_cache()
        out[f"p{p}"] = per_p
        if head is None and forms[0] in per_p and "sumfact" in per_p[forms[0]]:
            head = (p, forms[0], per_p[forms[0]]["sumfact"], name)
    hp, hform, h, hname = head
    return {
        "metric": "elements/s, hexahedra p = 4..7: sum factorisation in three directions vs along xi3 only",
        "value": h["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["kernel_ms_mean"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE_DESC[hform],
        "data": "synthetic (seeded perturbed hexahedral meshes and coefficients)",
        "config": {"workload": hname, "p": hp, "form": hform, "element": "hexahedron",
                   "parallelism": "single GPU"},
        "roofline": h["roofline"], "degrees": out, "device": torch.cuda.get_device_name(0)}


def bench_laplace(args):
    """The paper's own term (Laplace, eq. (1)) on its quadrature (the symmetric
    rule, N_I points), FP32 (its precision), at the paper's batch sizes: element
    matrices of about 500 MB, N_e = 500e6 / (4 n^2), for p = 1..7, on the
    perturbed prism mesh (first N_e elements).  GFLOP/s in the paper's
    convention = Table 2's operation count per element (shape functions,
    Jacobian, 7 per matrix entry, all per point) times N_e / kernel time."""
    import torch
    import paper_1310_1194_amd as F
    dev = torch.device("cuda:0")
    form = (args.forms or "fp32").split(",")[0]
    degrees = [int(x) for x in (args.workload or "1,2,3,4,5,6,7").split(",")] if args.workload and \
        args.workload[0].isdigit() else list(range(1, 8))
    steps, warm = max(3, min(args.steps, 10)), max(1, min(args.warmup, 3))
    rows = {}
    cpu = None
    for p in degrees:
        n = costmodel.nshp(p)
        ne = 500_000_000 // (4 * n * n)
        cells = -(-ne // 2)
        nx = ny = min(128, max(4, int(round(cells ** (1 / 3)))))
        nz = -(-cells // (nx * ny))
        batch = meshgen.make_batch(nx, ny, nz, amp=0.2, seed=10 + p).subset(np.arange(ne))
        X = torch.from_numpy(np.ascontiguousarray(batch.coords)).to(dev)
        dt = torch.float64 if form == "fp64" else torch.float32
        A = torch.empty((ne, n, n), dtype=dt, device=dev)
        tune = None if args.no_tune else F.laplace_autotune(X, p, form, A, reps=2)
        tile = F.laplace_tile_describe(p, form, F.laplace_tile_get(p, form))
        ms, mn, wall = timed(lambda: F.integrate_laplace_raw(X, p, form, A=A), steps, warm)
        points = F.nq(p, "symmetric")
        paper_ops = costmodel.laplace_paper_ops(p, points)
        own = ((costmodel.f_factored_zfirst(costmodel.nshp(p), p + 1, costmodel.nq(p, "symmetric"))
                if costmodel.is_zfirst_tile(tile) else costmodel.f_kf(p, "symmetric"))
               if costmodel.is_kf_tile(tile) else costmodel.f_dom(p, "symmetric"))
        peak = PEAK_TFLOPS[form]
        r = dict(ne=ne, mesh=f"{nx}x{ny}x{nz}", points=points, tile=tile, tune_ms=tune, kernel_ms_mean=ms,
                 kernel_ms_min=mn, us_per_element=ms * 1e3 / ne, elements_per_s=ne / (ms * 1e-3),
                 paper_convention_gflops=paper_ops * ne / (ms * 1e-3) / 1e9,
                 own_count_tflops=own * ne / (ms * 1e-3) / 1e12, own_count_frac_of_peak=own * ne / (ms * 1e-3) / 1e12 / peak,
                 hbm_gbs_algorithmic=ne * (8 * 18 + n * n * (8 if form == "fp64" else 4)) / (ms * 1e-3) / 1e9)
        if not args.no_cpu:
            import oracle
            idx = np.unique(np.linspace(0, ne - 1, min(ne, 64)).astype(np.int64))
            Ar, _ = oracle.integrate_laplace(p, batch.coords[idx])
            r["rel_err_A"], r["rel_err_A_max_elem"] = rel_err(A[torch.from_numpy(idx).to(dev)].cpu().numpy(), Ar)
            r["err_sample"] = len(idx)
            if p == 4:
                m = min(ne, 4096)
                t0 = time.perf_counter()
                oracle.integrate_laplace(p, batch.coords[:m])
                spent = time.perf_counter() - t0
                cpu = {"value": m / spent, "unit": "elements/s", "cores": oracle.max_threads(), "kind": "oracle",
                       "sample": f"p = 4: the first {m} of the {ne} elements ({spent:.2f} s, FP64)", "cpu": cpu_model(),
                       "single_thread": single_thread_rate(lambda k: oracle.integrate_laplace(p, batch.coords[:k]),
                                                           min(ne, 1024))}
        rows[f"p{p}"] = r
        print(f"[bench] laplace p={p} ne={ne}: {ms:.3f} ms, {r['paper_convention_gflops']:.0f} GFLOP/s (paper "
              f"convention), tile {tile}", file=sys.stderr, flush=True)
        del A, X
        torch.cuda.empty_cache()
    h = rows.get("p4") or next(iter(rows.values()))
    line = {"metric": "Laplace-term integration (the paper's eq. (1) on its N_I points) at its 500 MB batch sizes: "
                      "elements/s and GFLOP/s in the paper's convention",
            "value": h["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": steps, "warmup": warm,
            "ms_per_step": h["kernel_ms_mean"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": form, "data": "synthetic (seeded perturbed prism meshes)",
            "config": {"workload": "laplace_paper_sweep", "rule": "symmetric", "degrees": degrees,
                       "batch": "N_e = 500e6 / (4 n^2) per degree (element matrices of about 500 MB)"},
            "roofline": {"bound": "mfma", "achieved": h["own_count_tflops"], "peak": PEAK_TFLOPS[form],
                         "unit": "TFLOP/s", "frac": h["own_count_frac_of_peak"], "traffic": None,
                         "note": "p = 4 row; flops of the algorithm the variant runs (the factorised count for "
                                 "KxTNf shapes, 8 n^2 N_I point by point)"},
            "cpu_baseline": cpu, "degrees": fmt(rows)}
    return line


def bench_adjoint(args):
    """Adjoint of the p=3 workload (or another): gradients of
    sum_e <G_e,A_e> + <g_e,b_e>, FP64 and FP32 forms."""
    import torch
    import paper_1310_1194_amd as F
    args.workload = args.workload or "adj_p3_131072"
    forms = (args.forms or "fp64,fp32").split(",")
    w = meshgen.WORKLOADS[args.workload]
    p = w["p"]
    rule = args.rule
    orule = None if rule == "collapsed" else rule
    batch = meshgen.workload(args.workload)
    dev = torch.device("cuda:0")
    if costmodel.nshp(p) ** 2 * batch.ne > 2 ** 28:       # large G: drawn on the device
        Gdev, gdev, sample = meshgen.adjoint_seeds_device(batch, p, seed=w["seed"])
        G = g = None
    else:
        G, g, sample = meshgen.adjoint_seeds(batch, p)
        Gdev = gdev = None
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))
    ne = batch.ne
    res = {}
    for form in forms:
        dt = torch.float64 if form == "fp64" else torch.float32
        Gd, gd = (t(G).to(dt), t(g).to(dt)) if G is not None else (Gdev.to(dt), gdev.to(dt))
        out = None
        tune_ms = None
        if args.no_tune:
            pass
        elif rule == "collapsed":
            tune_ms = F.adjoint_autotune(*X, Gd, gd, p, form, reps=2)
        else:                       # time every block shape on this rule's kernels
            best = None
            for tt in range(F.adjoint_tile_count(p, form)):
                F.adjoint_tile_set(p, form, tt)
                ms_t, _, _ = timed(lambda: F.adjoint_raw(*X, Gd, gd, p, form, rule=rule), 2, 1)
                best = min(best, (ms_t, tt)) if best else (ms_t, tt)
            F.adjoint_tile_set(p, form, best[1])
            tune_ms = best[0]
        block = F.adjoint_tile_describe(p, form, F.adjoint_tile_get(p, form))

        def step():
            nonlocal out
            out = F.adjoint_raw(*X, Gd, gd, p, form, rule=rule)
        ms, mn, wall = timed(step, args.steps, args.warmup)
        es = 8 if form == "fp64" else 4
        res[form] = dict(kernel_ms_mean=ms, kernel_ms_min=mn, ms_per_step=wall, elements_per_s=ne / (wall * 1e-3),
                         block=block, tune_ms=tune_ms,
                         fdom_equiv_gflops=costmodel.f_dom(p, rule) * ne / (ms * 1e-3) / 1e9,
                         gflops_alg=(costmodel.f_adjoint_factored(p, rule) if costmodel.is_kf_tile(block)
                                     else costmodel.f_dom(p, rule)) * ne / (ms * 1e-3) / 1e9,
                         hbm_gbs_algorithmic=ne * costmodel.adjoint_bytes_per_element(p, es) / (ms * 1e-3) / 1e9,
                         grads=[o[torch.from_numpy(sample).to(dev)].cpu().numpy() for o in out])
        del Gd, gd
        print(f"[bench] adjoint {form}: {ms:.3f} ms, block {block}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        import oracle
        sub = batch.subset(sample)
        si = torch.from_numpy(sample).to(dev)
        Gs = G[sample] if G is not None else Gdev[si].cpu().numpy()
        gs = g[sample] if g is not None else gdev[si].cpu().numpy()
        ref = oracle.adjoint(p, sub.coords, sub.D, sub.beta, sub.c, sub.f, Gs, gs, rule=orule)
        names = ("dcoords", "dD", "dbeta", "dc", "df")
        for form, r in res.items():
            r["rel_err"] = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(r["grads"], ref[:5]))
            r["rel_err_per_array"] = {nm: dict(zip(("global", "max_elem"), rel_err(a, b)))
                                      for nm, a, b in zip(names, r["grads"], ref[:5])}
            r["err_sample"] = len(sample)
        chunk = min(ne, max(16, 2048 >> (2 * max(0, p - 3))))
        m, spent = 0, 0.0
        while spent < args.cpu_budget and m < ne:     # whole chunks until the time budget is spent
            lo, hi = m, min(ne, m + chunk)
            part = batch.subset(np.arange(lo, hi))
            Gm = G[lo:hi] if G is not None else Gdev[lo:hi].cpu().numpy()
            gm = g[lo:hi] if g is not None else gdev[lo:hi].cpu().numpy()
            t0 = time.perf_counter()
            oracle.adjoint(p, part.coords, part.D, part.beta, part.c, part.f, Gm, gm, rule=orule)
            spent += time.perf_counter() - t0
            m = hi
        m1 = min(ne, 256 if p <= 3 else 4)

        def one(k):
            part = batch.subset(np.arange(k))
            Gk = G[:k] if G is not None else Gdev[:k].cpu().numpy()
            gk = g[:k] if g is not None else gdev[:k].cpu().numpy()
            oracle.adjoint(p, part.coords, part.D, part.beta, part.c, part.f, Gk, gk, rule=orule)
        cpu = {"value": m / spent, "unit": "elements/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"first {m} of {ne} elements ({spent:.1f} s, FP64 reverse mode)", "cpu": cpu_model(),
               "single_thread": single_thread_rate(one, m1)}
    for r in res.values():
        r.pop("grads", None)
    h = res[forms[0]]
    peak = PEAK_TFLOPS["fp64" if forms[0] == "fp64" else "fp32"]
    line = {"metric": "adjoint elements/s (gradients w.r.t. D, beta, c, f, coordinates)", "value": h["elements_per_s"],
            "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": h["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": forms[0], "data": "synthetic (seeded mesh, coefficients, G, g ~ N(0,1))",
            "config": {"workload": args.workload + ("+symmetric_rule" if orule else ""), "p": p, "ne": ne,
                       "form": forms[0], "rule": rule},
            "roofline": {"bound": "mfma", "achieved": h["gflops_alg"] / 1e3, "peak": peak, "unit": "TFLOP/s",
                         "frac": h["gflops_alg"] / 1e3 / peak, "traffic": None,
                         "note": "flops of the algorithm the chosen block shape runs: 8 n^2 nq per element "
                                 "point by point; the factorised kernel's count for TKxTBf shapes "
                                 "(8 n^2 nij + 8 (p+1)^2 nij n + 36 nq n)"},
            "cpu_baseline": cpu, "forms": fmt(res)}
    return line


def bench_mixed(args):
    """Mixed-degree batch (p ~ U{1..6}, shuffled): bucketing + persistent
    launch, eager and as a replayed HIP graph."""
    import torch
    import paper_1310_1194_amd as F
    args.workload = args.workload or "mixed_262144"
    form = (args.forms or "fp32").split(",")[0]
    batch = meshgen.workload(args.workload)
    ne = batch.ne
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))
    pd = t(batch.p)
    plan = F.MixedPlan(ne, form)
    offA, offb = plan.bucket(pd)
    A, b = plan.alloc_outputs(offA, offb)
    tune_ms = None if args.no_tune else plan.autotune(*X, A, b, offA, offb, reps=2)
    chosen = plan.tile
    sets_ms = {}
    for ts in range(plan.tile_count):       # every compiled tile set, for the record
        plan.tile = ts
        sets_ms[plan.tile_describe(ts)] = timed(lambda: plan.integrate(*X, A, b, offA, offb), 3, 1)[0]
        print(f"[bench] mixed tile set {plan.tile_describe(ts)}: {sets_ms[plan.tile_describe(ts)]:.3f} ms",
              file=sys.stderr, flush=True)
    plan.tile = chosen
    ms_b, _, _ = timed(lambda: plan.bucket(pd), args.steps, args.warmup)
    ms_p, mn_p, _ = timed(lambda: plan.integrate(*X, A, b, offA, offb), args.steps, args.warmup)
    gA, gb = torch.empty_like(A), torch.empty_like(b)
    goA, gob = torch.empty_like(offA), torch.empty_like(offb)
    plan.capture(*X, pd, gA, gb, goA, gob)
    ms_g, mn_g, wall_g = timed(plan.replay, args.steps, args.warmup)
    errs = None
    if not args.no_cpu:
        # the first 1024 elements of each degree, from the graph replay's outputs, against the oracle
        import oracle
        torch.cuda.synchronize()
        oA, ob = goA.cpu().numpy(), gob.cpu().numpy()
        errs = {}
        for d in range(1, 7):
            idx = np.nonzero(batch.p == d)[0][:1024]
            n = costmodel.nshp(d)
            ia = torch.from_numpy(np.concatenate([np.arange(oA[e], oA[e] + n * n) for e in idx])).to(dev)
            ib = torch.from_numpy(np.concatenate([np.arange(ob[e], ob[e] + n) for e in idx])).to(dev)
            sub = batch.subset(idx)
            Ar, br, _ = oracle.integrate(d, sub.coords, sub.D, sub.beta, sub.c, sub.f)
            gA_, mA_ = rel_err(gA[ia].cpu().numpy().reshape(len(idx), n, n), Ar)
            gb_, _ = rel_err(gb[ib].cpu().numpy().reshape(len(idx), n), br)
            errs[f"p{d}"] = {"rel_err_A": gA_, "rel_err_A_max_elem": mA_, "rel_err_b": gb_, "elements": len(idx)}
    counts = np.bincount(batch.p, minlength=7)
    fdom = sum(int(counts[d]) * costmodel.f_dom(d) for d in range(1, 7))
    shapes = plan.tile_describe(plan.tile).split(",")     # one entry per degree 1..6
    flops = sum(int(counts[d]) * costmodel.f_kernel(d, "collapsed", shapes[d - 1]) for d in range(1, 7))
    es = 8 if form == "fp64" else 4
    bytes_ = sum(int(counts[d]) * costmodel.bytes_per_element(d, es) for d in range(1, 7))
    peak = PEAK_TFLOPS[form]
    cpu = None
    if not args.no_cpu:
        import oracle
        rates = {}
        for d in range(1, 7):
            idx = np.nonzero(batch.p == d)[0][: max(16, 4096 >> (2 * (d - 1)))]
            sub = batch.subset(idx)
            t0 = time.perf_counter()
            oracle.integrate(d, sub.coords, sub.D, sub.beta, sub.c, sub.f)
            rates[d] = len(idx) / (time.perf_counter() - t0)
        frac = counts[1:] / ne
        rate = 1.0 / sum(frac[d - 1] / rates[d] for d in range(1, 7))
        cpu = {"value": rate, "unit": "elements/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": "per degree the first elements of that degree (4096 >> 2(p-1), at least 16); "
                         "rate combined with the batch's degree mix", "cpu": cpu_model()}
    line = {"metric": "mixed-degree elements/s (one persistent degree-bucketed launch, HIP graph)",
            "value": ne / (ms_g * 1e-3), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall_g, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": form, "data": "synthetic (seeded mesh, p ~ U{1..6}, shuffled)",
            "config": {"workload": args.workload, "ne": ne, "form": form, "degree_counts": counts[1:].tolist(),
                       "tile_set": plan.tile, "tile_set_shapes": plan.tile_describe(plan.tile)},
            "tile_sets_ms": sets_ms,
            "bucket_ms": ms_b, "persistent_ms": ms_p, "persistent_ms_min": mn_p, "graph_ms": ms_g,
            "graph_ms_min": mn_g, "tune_ms": tune_ms, "fdom_equiv_gflops": fdom / (ms_p * 1e-3) / 1e9,
            "roofline": {"bound": "mfma", "achieved": flops / (ms_p * 1e-3) / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / (ms_p * 1e-3) / 1e12 / peak, "traffic": None,
                         "flops_per_launch": flops, "fdom_per_launch": fdom, "alg_bytes_per_launch": bytes_,
                         "note": "flops of the algorithm each degree's kernel runs: 8 n^2 nq per element "
                                 "point by point, the triangle-point contraction's count for KxTNf shapes"},
            "cpu_baseline": cpu, "errors_vs_oracle": errs}
    plan.close()
    return fmt(line)


def bench_assemble(args):
    """Global assembly of the p=4 element matrices (CSR, colour by colour):
    set-up on the host once, then the timed device assembly per form."""
    import torch
    import paper_1310_1194_amd as F
    args.workload = args.workload or "p4_131072"
    forms = (args.forms or "fp32,fp64").split(",")
    w = meshgen.WORKLOADS[args.workload]
    p = w["p"]
    batch = meshgen.workload(args.workload)
    ne, n = batch.ne, costmodel.nshp(p)
    dofs, ndof = meshgen.dof_map(w["nx"], w["ny"], w["nz"], p)
    t0 = time.perf_counter()
    plan = F.AsmPlan(dofs, ndof)
    setup_s = time.perf_counter() - t0
    print(f"[bench] assembly set-up {setup_s:.1f} s: ndof {ndof}, nnz {plan.nnz}, {plan.ncolors} colours",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    X = (t(batch.coords), t(batch.D), t(batch.beta), t(batch.c), t(batch.f))
    res = {}
    for form in forms:
        A, b = F.integrate_raw(*X, p, form)
        es = 8 if form == "fp64" else 4
        vals = torch.empty(plan.nnz, dtype=A.dtype, device=dev)
        rhs = torch.empty(ndof, dtype=A.dtype, device=dev)
        ms, mn, wall = timed(lambda: plan.assemble(A, b, form, values=vals, rhs=rhs), args.steps, args.warmup)
        # algorithmic bytes: element matrices, vectors and position map read once, the
        # global values and rhs cleared and written once, dof map and row starts read
        alg = ne * n * n * (es + 2) + ne * n * (es + 4) + 2 * (plan.nnz + ndof) * es + (ndof + 1) * 8
        res[form] = dict(kernel_ms_mean=ms, kernel_ms_min=mn, ms_per_step=wall, elements_per_s=ne / (ms * 1e-3),
                         alg_bytes=alg, gbs=alg / (ms * 1e-3) / 1e9)
        print(f"[bench] assembly {form}: {ms:.3f} ms, {alg / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic",
              file=sys.stderr, flush=True)
        del A, b, vals, rhs
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        import oracle
        m = 256                      # the oracle's assembly of the first m elements (their own system)
        part = batch.subset(np.arange(m))
        Ar, br, _ = oracle.integrate(p, part.coords, part.D, part.beta, part.c, part.f)
        t0 = time.perf_counter()
        oracle.assemble(dofs[:m], ndof, Ar, br)
        spent = time.perf_counter() - t0
        cpu = {"value": m / spent, "unit": "elements/s", "cores": 1, "kind": "oracle",
               "sample": f"assembly of the first {m} elements' matrices ({spent:.1f} s, FP64, one core)"}
    h = res[forms[0]]
    line = {"metric": "global assembly elements/s (CSR, colour by colour)", "value": h["elements_per_s"],
            "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": h["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": forms[0], "data": "synthetic (seeded mesh; element matrices from the forward pass)",
            "config": {"workload": args.workload, "p": p, "ne": ne, "ndof": ndof, "nnz": plan.nnz,
                       "colours": plan.ncolors, "setup_s": setup_s},
            "roofline": {"bound": "hbm", "achieved": h["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": h["gbs"] / HBM_PEAK_GBS, "traffic": None},
            "cpu_baseline": cpu, "forms": fmt(res)}
    plan.close()
    return fmt(line)


if __name__ == "__main__":
    main()
