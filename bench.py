#!/usr/bin/env python
"""Throughput of the pilot-wave exact sampler on one MI355X.

Default workload (the largest single-GPU configuration): ideal QAOA p=2
MaxCut on the 4 x 119 ladder (476 qubits, 16384 chains) together with 32
ladders 4 x W, W ~ U{25..100}, p ~ U{1,2} (100 to 400 qubits, 1536 chains
each): 65536 chains in one captured graph (pws_sample_batch, a branch per
instance), BF16x3 contraction (the dense-run sweep form on the matrix cores,
bf16 hi/lo split products accumulated in FP32), FP64 draws.  A "step" is one
full sampling pass of every instance (every non-monomial gate: the batched
prefix contraction and the transition draw), inputs resident on the device.

Prints one JSON line: samples/s; the contraction rate of the step kernels
against the roofline (HIP events over the timed replays); the same batch in
the other precisions (FP32 op by op on the vector ALUs, FP32 dense runs on
the matrix cores, FP64), each with its error against the FP64 engine on the
476-qubit instance (candidate amplitudes that sampling passes draw from,
chains at equal states, per chain ||a - r|| / ||r||) and its bar; and the CPU
oracle (path-sum amplitudes, Algorithm 1) timed on a bounded sample.
Other workloads: --workload grid6x8 | noisy3reg | grid6x8_noisy | ising_p1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3    # MI355X FP32 vector / matrix, published
BF16_MFMA_PEAK_TFLOPS = 2500.0     # MI355X dense bf16 matrix, published
BF16X3_PEAK_TFLOPS = BF16_MFMA_PEAK_TFLOPS / 3   # three bf16 products per FP32-equivalent product
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
METRIC = "exact samples/sec + contraction TFLOP/s (FP32 vs BF16x3) at fixed error vs FP64"
BARS = {"fp64": None, "fp32": 1e-5, "fp32_mfma": 1e-5, "bf16x3": 1e-3}
VARIANTS = {   # name -> (plan precision, dense runs)
    "fp32": ("fp32", False),          # op by op on the vector ALUs, per chain
    "fp32_mfma": ("fp32", True),      # dense runs, FP32 matrix-core products
    "bf16x3": ("bf16x3", True),       # dense runs, bf16 hi/lo split products
    "fp64": ("fp64", False),
}

SOURCES = ["paper_2510_24218_amd/csrc/kernels.hip", "paper_2510_24218_amd/csrc/network.cpp",
           "paper_2510_24218_amd/csrc/api.cpp", "paper_2510_24218_amd/csrc/program.hpp",
           "paper_2510_24218_amd/csrc/dense.cpp"]


def _source_sha():
    import hashlib
    h = hashlib.sha256()
    for s in SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()[:16]


def _plans(circs, variant, threads=16):
    """Plans of every circuit in one precision (host planning in threads: the
    C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2510_24218_amd as E
    prec, dense = VARIANTS[variant]
    with ThreadPoolExecutor(min(threads, len(circs))) as ex:
        return list(ex.map(lambda c: E.Plan(c, precision=prec, dense=dense), circs))


def _time_batch(plans, ks, seed0, reps, outs):
    """Wall time per replay of the batch and HIP-event kernel time of the
    replays (pws_last_timing of the first plan covers every branch)."""
    import torch
    import paper_2510_24218_amd as E
    kernel_ms, launches = 0.0, 0
    if reps <= 0:
        return 0.0, 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        seeds = [seed0 + 1000 * i + j for j in range(len(plans))]
        if len(plans) == 1:
            plans[0].sample(ks[0], seeds[0], out=outs[0])
        else:
            E.sample_batch(plans, ks, seeds, outs)
        ms, nl = plans[0].last_timing()
        kernel_ms += ms
        launches += nl
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps, kernel_ms / reps, launches / reps


def _probe_err(c, pa, p64, K, seed, steps):
    """Candidate amplitudes that sampling passes of `pa` and of the FP64 plan
    draw from at the given steps, compared on the chains whose states agree
    before the step: per chain ||a - r||_2 / ||r||_2 (the quantity the draw
    uses); max, p99.9 and the share of chains compared."""
    import numpy as np
    errs, n_cmp, n_all = [], 0, 0
    for k in steps:
        op, gate, m = pa.step_info(k)
        qs = list(c.gates[gate].qubits)
        sa, ma, ea = pa.sample_probe(K, seed, k)
        s6, m6, e6 = p64.sample_probe(K, seed, k)
        mask = np.zeros(pa.words, dtype=np.uint64)
        for q in qs:
            mask[q // 64] |= np.uint64(1) << np.uint64(q % 64)
        same = np.all((sa & ~mask) == (s6 & ~mask), axis=1)
        nr = np.linalg.norm(m6, axis=1)
        ok = same & (nr > 0)
        d = (ea.astype(np.int64) - e6.astype(np.int64)).astype(np.float64)
        a = ma * np.exp2(d)[:, None]
        errs.extend((np.linalg.norm(a[ok] - m6[ok], axis=1) / nr[ok]).tolist())
        n_cmp += int(ok.sum())
        n_all += K
    errs = np.array(errs)
    return {"max": float(errs.max()), "p99.9": float(np.quantile(errs, 0.999)),
            "chains_compared": n_cmp / n_all, "steps": [int(s) for s in steps]}


def _cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        pass
    return model, threads


def _cpu_baseline(c, n_probe_steps, budget_s=20.0):
    """The oracle (Algorithm 1 with path-sum amplitudes of every step's
    candidates) timed on one chain at n_probe_steps steps spread evenly over
    the pass, extrapolated to the whole pass (a bounded sample: the full pass
    of one chain takes minutes)."""
    import numpy as np
    from oracle import pathsum as PS
    steps = [g for g, gg in enumerate(c.gates) if gg.kind in ("H", "RX")]
    pick = sorted(set(int(x) for x in np.linspace(0, len(steps) - 1, n_probe_steps)))
    rng = np.random.default_rng(7)
    s = rng.integers(0, 2, c.n_qubits)
    t0 = time.perf_counter()
    done = 0
    for i in pick:
        gi = steps[i]
        PS.amplitude(c, gi + 1, s, open_qubits=(c.gates[gi].qubits[0],))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    per_pass = dt / done * len(steps)
    model, threads = _cpu_info()
    return {"value": 1.0 / per_pass, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": f"one chain of the {c.n_qubits}-qubit instance: path-sum candidate amplitudes at "
                      f"{done} of its {len(steps)} steps spread evenly over the pass ({dt:.1f} s, numpy with "
                      f"{threads} BLAS threads), extrapolated to all steps: {per_pass:.0f} s per sample"}


def _traffic(name):
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if os.path.exists(path):
        rec = json.load(open(path))
        if rec.get("source_sha") == _source_sha():
            return rec.get("bytes_per_pass")
    return None


def _pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, trace_dir, out_path, copy_bytes, kernel_key,
                 passes):
    """HBM traffic and time of one sampling pass (one graph replay: the step
    kernels of every instance), from rocprofv3 runs of one command that ran
    `passes` replays: two --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch, summed over the dispatches whose kernel name contains
    kernel_key, divided by `passes`), each scaled by what the counter reads
    for a plain device copy of copy_bytes; and a --kernel-trace run, whose
    engine dispatches split in order into `passes` equal replays give the
    pass's span (first start to last end) and summed kernel durations."""
    import csv

    def table(d, suffix):
        f = [x for x in os.listdir(d) if x.endswith(suffix)][0]
        return list(csv.DictReader(open(os.path.join(d, f))))

    def total(d):
        rows = [r for r in table(d, "counter_collection.csv") if kernel_key in r["Kernel_Name"]]
        return sum(float(r["Counter_Value"]) for r in rows) * 1024.0 / passes, len(rows) / passes

    def copy_kib(d):
        return max(float(r["Counter_Value"]) for r in table(d, "counter_collection.csv")) * 1024.0

    f_fac = copy_bytes / copy_kib(copy_fetch_dir)
    w_fac = copy_bytes / copy_kib(copy_write_dir)
    fetch, n = total(fetch_dir)
    write, _ = total(write_dir)
    tr = sorted((r for r in table(trace_dir, "kernel_trace.csv") if "pws::" in r["Kernel_Name"]),
                key=lambda r: int(r["Start_Timestamp"]))
    per = len(tr) // passes
    spans, busy = [], []
    for i in range(passes):
        g = tr[i * per:(i + 1) * per]
        spans.append((max(int(r["End_Timestamp"]) for r in g) - min(int(r["Start_Timestamp"]) for r in g)) / 1e6)
        busy.append(sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in g
                        if kernel_key in r["Kernel_Name"]) / 1e6)
    rec = {"bytes_per_pass": fetch * f_fac + write * w_fac, "fetch_bytes_per_pass": fetch * f_fac,
           "write_bytes_per_pass": write * w_fac, "fetch_factor": f_fac, "write_factor": w_fac,
           "step_kernels_per_pass": n, "engine_dispatches_per_pass": per, "passes": passes,
           "pass_span_ms": spans, "step_kernel_busy_ms": busy, "kernel_key": kernel_key,
           "source_sha": _source_sha(), "sources": SOURCES}
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec))


def _line(args, value, ms_per_step, dtype, config, roofline, **extra):
    d = {"metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
         "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline}
    d.update(extra)
    return d


def _run_variants(args, circs, ks, seed, main_variant, err_circ, err_K, err_steps, name):
    """Every precision on the same batch: samples/s, algorithmic TFLOP/s,
    error against FP64 on err_circ (the first instance) with its bar.
    Returns (main plans, main timings, variant table)."""
    import torch
    out = {}
    main = None
    first = {}     # each variant's plan of the first instance (error probes)
    order = [main_variant] + [v for v in VARIANTS if v != main_variant]
    for v in order:
        if args.variants == "main" and v != main_variant:
            continue
        plans = _plans([c for c in circs], v)
        outs = [torch.zeros((k, p.words), dtype=torch.int64, device="cuda") for p, k in zip(plans, ks)]
        batch_shapes = None
        if v == main_variant and args.autotune and len(plans) > 1:
            # a batch: its branches compete for the device, so the shapes each
            # plan's tuning picks alone need not be the batch's best; the batch
            # is timed with the default shapes and with the per-plan tuned
            # ones, and keeps the faster (both give the same samples)
            _time_batch(plans, ks, seed, 1, outs)
            ms_def = _time_batch(plans, ks, seed + 33, 3, outs)[0]
            tplans = _plans([c for c in circs], v)
            tuned = [p.autotune(k, seed + 5) for p, k in zip(tplans, ks)]
            _time_batch(tplans, ks, seed, 1, outs)
            ms_tun = _time_batch(tplans, ks, seed + 33, 3, outs)[0]
            if ms_tun < ms_def:
                plans, tplans = tplans, plans
            del tplans
            torch.cuda.empty_cache()
            batch_shapes = {"chosen": "tuned per plan" if ms_tun < ms_def else "default shapes",
                            "ms_default_shapes": ms_def, "ms_tuned_per_plan": ms_tun}
        elif v == main_variant and args.autotune:
            # the plan's sweep launch shapes, timed alone (pws_autotune)
            tuned = [p.autotune(k, seed + 5) for p, k in zip(plans, ks)]
        reps = args.steps if v == main_variant else max(2, min(args.steps, 3))
        warm = args.warmup if v == main_variant else 1
        _time_batch(plans, ks, seed, warm, outs)
        ms, kms, nl = _time_batch(plans, ks, seed + 77, reps, outs)
        flops = sum(p.stats()["flops_per_sample"] * k for p, k in zip(plans, ks))
        K = sum(ks)
        rec = {"samples_per_s": K / (ms / 1e3), "ms_per_step": ms, "kernel_ms_per_step": kms,
               "launches_per_step": nl, "tflops_algorithmic": flops / (kms / 1e3) / 1e12}
        first[v] = plans[0]
        out[v] = rec
        if v == main_variant and args.autotune:
            rec["tuned_shape_first_instance"] = tuned[0]
        if batch_shapes:
            rec["batch_shapes"] = batch_shapes
        if v == main_variant:
            main = (plans, ms, kms, nl, flops, outs)
        else:
            del plans, outs
            torch.cuda.empty_cache()
    # errors against the FP64 engine on the first instance
    if args.no_errors:
        return main, out
    if "fp64" not in first:
        first["fp64"] = _plans([err_circ], "fp64")[0]
    for v in out:
        if v == "fp64":
            out[v]["error_vs_fp64"] = None
            continue
        e = _probe_err(err_circ, first[v], first["fp64"], err_K, seed, err_steps)
        e["bar"] = BARS[v]
        e["meets_bar"] = e["max"] <= BARS[v]
        out[v]["error_vs_fp64"] = e
    return main, out


def _bench_batch(args, circs, ks, seed, name, config, err_steps, traffic_name, cpu_circ):
    main_variant = args.precision
    main, variants = _run_variants(args, circs, ks, seed, main_variant, circs[0], ks[0], err_steps, name)
    plans, ms, kms, nl, flops, outs = main
    K = sum(ks)
    tflops = flops / (kms / 1e3) / 1e12
    if main_variant == "bf16x3":
        peak, bound = BF16X3_PEAK_TFLOPS, "mfma"
        peak_note = "bf16 dense matrix peak / 3 (three bf16 products per FP32-equivalent product)"
    elif main_variant == "fp32_mfma":
        peak, bound, peak_note = FP32_VECTOR_PEAK_TFLOPS, "mfma", "FP32 matrix peak"
    elif main_variant == "fp64":
        peak, bound, peak_note = FP64_PEAK_TFLOPS, "alu", "FP64 vector peak"
    else:
        peak, bound, peak_note = FP32_VECTOR_PEAK_TFLOPS, "alu", "FP32 vector peak (packed)"
    roof = {"bound": bound, "achieved": tflops, "peak": peak, "unit": "TFLOP/s", "frac": tflops / peak,
            "traffic": _traffic(traffic_name),
            "kernel": "the step kernels of one sampling pass of every instance (one captured graph per pass, "
                      "launched once; dense runs on the matrix cores where the variant has them)",
            "launch": "one graph launch = one pass", "flops_per_launch": flops, "launch_ms": kms,
            "step_kernel_launches_per_pass": nl,
            "achieved_basis": "algorithmic flops of a pass (8 per complex multiply-add of every sweep op it runs) / "
                              "the pass's time between HIP events on the stream the graph is launched on",
            "traffic_basis": "HBM bytes of a pass (rocprofv3 FETCH_SIZE x fetch factor + WRITE_SIZE x write "
                             "factor over its step kernels, factors from a plain device copy)",
            "peak_basis": peak_note}
    cfg = dict(config)
    cfg["precision"] = main_variant
    line = _line(args, K / (ms / 1e3), ms, {"fp32": "f32", "fp32_mfma": "f32", "bf16x3": "bf16x3",
                                             "fp64": "f64"}[main_variant], cfg, roof,
                 kernel_ms_per_step=kms, launches_per_step=nl, flops_per_sample=flops / K,
                 contraction_tflops_fp32=variants.get("fp32", {}).get("tflops_algorithmic"),
                 contraction_tflops_fp32_mfma=variants.get("fp32_mfma", {}).get("tflops_algorithmic"),
                 contraction_tflops_bf16x3=variants.get("bf16x3", {}).get("tflops_algorithmic"),
                 variants=variants,
                 variant_forms={
                     "fp32": "plain FP32 per chain: every sweep op applied by each chain on the vector ALUs",
                     "fp32_mfma": "FP32 batched: each run of ops on four positions contracted once per plan "
                                  "(chain-independent, per chain-bit variant, in FP64 on the host) and shared by "
                                  "all chains, applied per chain on the FP32 matrix cores",
                     "bf16x3": "BF16x3 batched: the same shared run matrices as bf16 hi/lo pairs, three bf16 "
                               "matrix-core products per tile accumulated in FP32",
                     "fp64": "FP64 per chain (reference for the errors)"})
    if not args.no_cpu:
        line["cpu_baseline"] = _cpu_baseline(cpu_circ, args.cpu_steps)
    print(json.dumps(line))


def _ising_instances(args, n, K, config):
    """Instances 0 .. --instances - 1 of an Ising family at one size, each
    sampled alone (its own plan and captured pass, shapes autotuned): the
    line's value is the median samples/s over the instances, each one's
    figure beside it; the other precisions and the errors against FP64 on
    instance 0."""
    import statistics
    import torch
    import instances as I
    circs = [I.workload_ising_p1(args.topology, n, i) for i in range(args.instances)]
    plans = _plans([c for c, _, _ in circs], args.precision)
    print(f"[ising_p1 {args.topology} n={n}] {len(plans)} plans built", file=sys.stderr, flush=True)
    per = []
    for (c, _, seed), p in zip(circs, plans):
        out = torch.zeros((K, p.words), dtype=torch.int64, device="cuda")
        if args.autotune:
            p.autotune(K, seed + 5)
        _time_batch([p], [K], seed, args.warmup, [out])
        ms, kms, nl = _time_batch([p], [K], seed + 77, args.steps, [out])
        per.append({"instance": c.name, "samples_per_s": K / (ms / 1e3), "ms_per_step": ms})
        print(f"[ising_p1 {args.topology} n={n}] {c.name}: {per[-1]['samples_per_s']:.0f} samples/s",
              file=sys.stderr, flush=True)
        del out
    del plans
    torch.cuda.empty_cache()
    c0, _, seed0 = circs[0]
    ns = 2 * c0.n_qubits
    steps = [ns - 1 - 3 * i for i in range(4)][::-1]
    _, variants = _run_variants(args, [c0], [K], seed0, args.precision, c0, K, steps, "ising")
    vals = [r["samples_per_s"] for r in per]
    cfg = dict(config)
    cfg["workload"] = f"ising_p1_{args.topology}_n{c0.n_qubits}_x{args.instances}"
    cfg["instances"] = args.instances
    cfg["precision"] = args.precision
    med = statistics.median(vals)
    line = _line(args, med, K / med * 1e3, {"fp32": "f32", "fp32_mfma": "f32", "bf16x3": "bf16x3",
                                           "fp64": "f64"}[args.precision], cfg, None,
                 per_instance=per, samples_per_s_min=min(vals), samples_per_s_max=max(vals),
                 variants_instance0=variants)
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=list(VARIANTS),
                    help="the variant the line's value is measured in (default: bf16x3)")
    ap.add_argument("--variants", default="all", choices=["all", "main"],
                    help="time the other precisions beside the main one (default) or not")
    ap.add_argument("--chains", type=int, default=0, help="override the chain count of single-instance workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=24, help="steps of the CPU oracle sample")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default sweep launch shapes (no pws_autotune before timing)")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error probes against FP64 (profiling runs: only the timed replays)")
    ap.add_argument("--pmc-summary", nargs=5, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "TRACE_DIR"),
                    help="write profiles/traffic_<workload>.json from rocprofv3 output directories and exit")
    ap.add_argument("--kernel-key", default="step_kernel_sweep<float",
                    help="--pmc-summary: substring naming the step kernels of the timed variant")
    ap.add_argument("--copy-bytes", type=float, default=float(2 ** 30))
    ap.add_argument("--pmc-passes", type=int, default=3,
                    help="--pmc-summary: replays the profiled command ran (warmup + steps)")
    ap.add_argument("--workload", default="ladders_mixed",
                    choices=["ladders_mixed", "grid6x8", "noisy3reg", "grid6x8_noisy", "ising_p1"],
                    help="ladders_mixed: the 476-qubit ladder (16384 chains) and 32 ladders of 100-400 qubits "
                         "(1536 chains each) in one captured graph (default); grid6x8: the 48-qubit grid, 4096 "
                         "chains; noisy3reg: noisy QAOA p=2 on a random 3-regular graph of --qubits nodes, 8192 "
                         "chains; grid6x8_noisy: the grid with the same noise; ising_p1: Gaussian-weighted "
                         "Ising QAOA p=1 on --topology with --qubits nodes")
    ap.add_argument("--qubits", type=int, default=0, help="noisy3reg / ising_p1: graph size")
    ap.add_argument("--instances", type=int, default=1,
                    help="ising_p1: time instances 0 .. N-1 of the family one by one (median in the line)")
    ap.add_argument("--topology", default="grid",
                    choices=["grid", "heavy_hex", "kings", "chimera", "3reg"], help="ising_p1: graph family")
    args = ap.parse_args()
    if args.pmc_summary:
        _pmc_summary(*args.pmc_summary, os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json"),
                     args.copy_bytes, args.kernel_key, args.pmc_passes)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (chains shard "
              "trivially across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import instances as I

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "ladders_mixed":
        cl, Kl, seed = I.workload_ladder4x119()
        mixed = I.workload_mixed_ladders(32)
        circs = [cl] + [c for c, _ in mixed]
        ks = [Kl] + [k for _, k in mixed]
        config = {"workload": "qaoa_maxcut_ladder4x119_p2_plus_32_mixed_ladders", "instances": len(circs),
                  "n_qubits": [c.n_qubits for c in circs], "chains": ks, "total_chains": sum(ks),
                  "draw": "fp64", "execution": "one captured graph, a branch per instance"}
        _bench_batch(args, circs, ks, seed, "ladders_mixed", config, [700, 1000, 1300, 1427],
                     "ladders_mixed", cl)
        return
    if args.workload == "grid6x8":
        c, K, seed = I.workload_grid6x8()
        K = args.chains or K
        config = {"workload": "qaoa_maxcut_grid6x8_p2", "n_qubits": c.n_qubits, "edges": len(c.edges),
                  "p": 2, "chains": K, "draw": "fp64"}
        _bench_batch(args, [c], [K], seed, "grid6x8", config, [60, 90, 120, 143], "grid6x8", c)
        return
    if args.workload == "ising_p1":
        n = args.qubits or 100
        c, K, seed = I.workload_ising_p1(args.topology, n)
        K = args.chains or K
        config = {"workload": f"ising_p1_{args.topology}_n{c.n_qubits}", "n_qubits": c.n_qubits,
                  "edges": len(c.edges), "p": 1, "chains": K, "weights": "gaussian couplings and fields",
                  "draw": "fp64"}
        ns = 2 * c.n_qubits
        steps = [ns - 1 - 3 * i for i in range(4)][::-1]
        if args.instances > 1:
            _ising_instances(args, n, K, config)
            return
        _bench_batch(args, [c], [K], seed, f"ising_p1_{args.topology}", config, steps,
                     f"ising_p1_{args.topology}", c)
        return
    # noisy workloads: one precision (the noise records keep the vector form)
    if args.workload == "grid6x8_noisy":
        c, K, seed = I.workload_grid6x8()
        c = I.add_qaoa_noise(c, depol2=1e-3, ampdamp=5e-4)
        name = "qaoa_maxcut_grid6x8_p2_noisy"
    else:
        c, K, seed = I.workload_noisy3reg100(args.qubits or 40)
        name = f"qaoa_maxcut_3reg_n{c.n_qubits}_p2_noisy"
    K = args.chains or K
    import paper_2510_24218_amd as E
    p = E.Plan(c, precision="fp32")
    outs = [torch.zeros((K, p.words), dtype=torch.int64, device="cuda")]
    _time_batch([p], [K], seed, args.warmup, outs)
    ms, kms, nl = _time_batch([p], [K], seed + 77, args.steps, outs)
    st = p.stats()
    tflops = st["flops_per_sample"] * K / (kms / 1e3) / 1e12
    config = {"workload": name, "n_qubits": c.n_qubits, "edges": len(c.edges), "p": 2, "chains": K,
              "noise_sites": len(c.noise), "precision": "fp32", "draw": "fp64"}
    roof = {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
            "kernel": "step kernels of a pass (sweep form, and node form for steps wider than LDS)"}
    print(json.dumps(_line(args, K / (ms / 1e3), ms, "f32", config, roof, kernel_ms_per_step=kms,
                           launches_per_step=nl, flops_per_sample=st["flops_per_sample"])))


if __name__ == "__main__":
    main()
