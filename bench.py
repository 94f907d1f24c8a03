#!/usr/bin/env python
"""Throughput of the pilot-wave exact sampler on one MI355X.

Workload: ideal QAOA p=2 MaxCut on the 6x8 grid (48 qubits, 82 edges, seeded
angles), 4096 independent chains per step; a "step" here is one full sampling
pass: all 144 non-monomial gates, each a batched prefix contraction plus the
FP64 transition draw, over the 4096 chains (inputs resident on the device).

Prints one JSON line: samples/s (FP32 contraction), the contraction rate of
the step kernel against its roofline (HIP-event time of the step launches on
the plan's stream; every step runs in the on-chip sweep form, so the bound is
the vector ALU, with the on-chip tensor traffic beside it), the FP32 error
against the FP64 engine (per-chain normwise relative error of the candidate
amplitudes), and the CPU oracle (Algorithm 1 with path-sum amplitudes) timed
on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X: 256 CUs x 2.4 GHz, FP32 vector (published)
HBM_PEAK_GBS = 8000.0              # MI355X HBM3E (published)
LDS_PEAK_GBS = 256 * 128 * 2.4     # 256 CUs x 128 bytes/clock x 2.4 GHz


def _fp32_error_vs_fp64(c, p32, p64, rng, n_steps_probe=8, n_states=64):
    import numpy as np
    import instances as I
    errs, errs_inv = [], []
    ns = p32.n_steps()
    steps = sorted(set(int(x) for x in np.linspace(0, ns - 1, n_steps_probe)))
    n = c.n_qubits
    for k in steps:
        op, gate, m = p32.step_info(k)
        touched = {q for g in c.gates[:gate + 1] for q in g.qubits}
        s = rng.integers(0, 2, (n_states, n))
        for q in range(n):
            if q not in touched:
                s[:, q] = 0
        b = I.pack_bits(s)
        a32, e32 = p32.step_amplitudes(k, b)
        a64, e64 = p64.step_amplitudes(k, b)
        v32 = a32 * np.exp2(e32.astype(float))[:, None]
        v64 = a64 * np.exp2(e64.astype(float))[:, None]
        errs.extend(list(np.linalg.norm(v32 - v64, axis=1) / np.linalg.norm(v64, axis=1)))
        # the draw normalises the candidates: a complex factor common to all of
        # them cancels, so the error is also taken after the best such factor
        for x, y in zip(v32, v64):
            alpha = np.vdot(x, y) / np.vdot(x, x)
            errs_inv.append(np.linalg.norm(alpha * x - y) / np.linalg.norm(y))
    errs = np.array(errs)
    errs_inv = np.array(errs_inv)
    return {"max": float(errs.max()), "p99.9": float(np.quantile(errs, 0.999)), "bar": 1e-5,
            "up_to_common_factor": {"max": float(errs_inv.max()), "p99.9": float(np.quantile(errs_inv, 0.999))}}


def _cpu_baseline(c, seed, n_chains):
    from oracle import sampler as S
    t0 = time.perf_counter()
    S.sample_ideal_pathsum(c, n_chains, seed)
    dt = time.perf_counter() - t0
    return {"value": n_chains / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_chains} chains x all {sum(1 for g in c.gates if g.kind in ('H', 'RX'))} "
                      f"steps of the same workload, Algorithm 1 with path-sum amplitudes "
                      f"(numpy, one thread), {dt:.1f} s"}


SOURCES = ["paper_2510_24218_amd/csrc/kernels.hip", "paper_2510_24218_amd/csrc/network.cpp",
           "paper_2510_24218_amd/csrc/api.cpp", "paper_2510_24218_amd/csrc/program.hpp"]


def _source_sha():
    import hashlib
    h = hashlib.sha256()
    for s in SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()[:16]


def _pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, trace_dir, out_path, copy_bytes):
    """HBM traffic per step-kernel launch of a timed FP32 sampling pass, from
    two rocprofv3 --pmc runs of this script (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch), each scaled by what the counter reads for a plain device copy
    of copy_bytes; launch durations of the same pass from a --kernel-trace run."""
    import csv

    def table(d, suffix):
        f = [x for x in os.listdir(d) if x.endswith(suffix)][0]
        return list(csv.DictReader(open(os.path.join(d, f))))

    def fp32_passes(rows, key):
        rows = sorted(rows, key=lambda r: int(r[key]))
        out, cur = [], None
        for r in rows:
            n = r["Kernel_Name"]
            if "init_state_kernel" in n:
                cur = []
                out.append(cur)
            elif cur is not None and "step_kernel" in n and "<float" in n:
                cur.append(r)
        longest = max(len(x) for x in out)
        return [x for x in out if len(x) == longest]

    def counter_pass(d):
        ps = fp32_passes(table(d, "counter_collection.csv"), "Dispatch_Id")
        p = ps[1] if len(ps) > 1 else ps[0]   # the first timed pass (after the warm-up)
        return sum(float(r["Counter_Value"]) for r in p) * 1024.0, len(p)

    def copy_kib(d):
        return max(float(r["Counter_Value"]) for r in table(d, "counter_collection.csv")) * 1024.0

    f_fac = copy_bytes / copy_kib(copy_fetch_dir)
    w_fac = copy_bytes / copy_kib(copy_write_dir)
    fetch, n = counter_pass(fetch_dir)
    write, _ = counter_pass(write_dir)
    tr = fp32_passes(table(trace_dir, "kernel_trace.csv"), "Start_Timestamp")
    tp = tr[1] if len(tr) > 1 else tr[0]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in tp]
    rec = {"bytes_per_launch": (fetch * f_fac + write * w_fac) / n, "fetch_bytes_per_launch": fetch * f_fac / n,
           "write_bytes_per_launch": write * w_fac / n, "fetch_factor": f_fac, "write_factor": w_fac,
           "launches_per_pass": n, "avg_launch_ms": sum(durs) / len(durs), "pass_ms": sum(durs),
           "source_sha": _source_sha(), "sources": SOURCES}
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec))


def _bench_ladders_mixed(args):
    """Uneven instances in one replay: the 476-qubit ladder and 32 mixed
    ladders, each plan a branch of one captured graph (pws_sample_batch)."""
    import numpy as np
    import torch
    import instances as I
    import paper_2510_24218_amd as E

    cl, Kl, seed = I.workload_ladder4x119()
    circs = [(cl, Kl)] + I.workload_mixed_ladders(32)
    plans = [E.Plan(c, precision="fp32") for c, _ in circs]
    ks = [k for _, k in circs]
    K = sum(ks)
    outs = [torch.zeros((k, p.words), dtype=torch.int64, device="cuda") for p, k in zip(plans, ks)]
    seeds = lambda i: [seed + 100 * i + j for j in range(len(plans))]
    for i in range(args.warmup):
        E.sample_batch(plans, ks, seeds(i), outs)
    torch.cuda.synchronize()
    kernel_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        E.sample_batch(plans, ks, seeds(1000 + i), outs)
        ms, nl = plans[0].last_timing()
        kernel_ms += ms
        launches += nl
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same plans one after another (each its own captured pass)
    seq_ms = 0.0
    for p, k, o in zip(plans, ks, outs):
        p.sample(k, seed, out=o)
        seq_ms += p.last_timing()[0]
    flops = sum(p.stats()["flops_per_sample"] * k for p, k in zip(plans, ks))
    tflops = flops * args.steps / (kernel_ms / 1e3) / 1e12
    p64 = E.Plan(cl, precision="fp64")
    fp32_err = _fp32_error_vs_fp64(cl, plans[0], p64, np.random.default_rng(5))
    line = {
        "metric": "exact samples/sec + contraction TFLOP/s (FP32 vs BF16x3) at fixed error vs FP64",
        "value": K / (ms_per_step / 1e3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qaoa_maxcut_ladder4x119_p2_plus_32_mixed_ladders", "instances": len(plans),
                   "n_qubits": [c.n_qubits for c, _ in circs], "chains": ks, "total_chains": K,
                   "precision": "fp32", "draw": "fp64", "execution": "one captured graph, a branch per instance"},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "step kernels (sweep form) of every instance, one graph replay"},
        "kernel_ms_per_step": kernel_ms / args.steps,
        "launches_per_step": launches / args.steps,
        "sequential_ms_per_step": seq_ms,
        "fp32_error_vs_fp64_476q": fp32_err,
    }
    print(json.dumps(line))


def _bench_noisy(args):
    """Noisy QAOA p=2 (depolarising 1e-3 after each RZZ, amplitude damping
    5e-4 after each RX, Kraus branches drawn per chain): on a seeded random
    3-regular graph of --qubits nodes, 8192 chains (the noisy workload at a
    size one GPU can contract; steps wider than the LDS run as trees of nodes
    through device memory), or on the 6x8 grid, 4096 chains."""
    import numpy as np
    import torch
    import instances as I
    import paper_2510_24218_amd as E

    if args.workload == "grid6x8_noisy":
        c, K, seed = I.workload_grid6x8()
        c = I.add_qaoa_noise(c, depol2=1e-3, ampdamp=5e-4)
        name = "qaoa_maxcut_grid6x8_p2_noisy"
    else:
        c, K, seed = I.workload_noisy3reg100(args.qubits)
        name = f"qaoa_maxcut_3reg_n{c.n_qubits}_p2_noisy"
    if args.chains:
        K = args.chains
    p = E.Plan(c, precision="fp32")
    st = p.stats()
    sw = p.sweep_stats()
    out = torch.zeros((K, p.words), dtype=torch.int64, device="cuda")
    for i in range(args.warmup):
        p.sample(K, seed + i, out=out)
    torch.cuda.synchronize()
    kernel_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        p.sample(K, seed + 1000 + i, out=out)
        ms, nl = p.last_timing()
        kernel_ms += ms
        launches += nl
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    tflops = st["flops_per_sample"] * K * args.steps / (kernel_ms / 1e3) / 1e12
    # amplitudes of the noiseless circuit (noisy amplitudes are chain-dependent)
    ideal = c.without_noise()
    fp32_err = _fp32_error_vs_fp64(ideal, E.Plan(ideal, precision="fp32"), E.Plan(ideal, precision="fp64"),
                                   np.random.default_rng(5))
    line = {
        "metric": "exact samples/sec + contraction TFLOP/s (FP32 vs BF16x3) at fixed error vs FP64",
        "value": K / (ms_per_step / 1e3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "n_qubits": c.n_qubits,
                   "edges": len(c.edges), "p": 2, "chains": K, "noise_sites": len(c.noise),
                   "contraction_steps": p.n_steps(), "sweep_steps": sw["n_sweep_steps"],
                   "precision": "fp32", "draw": "fp64", "log2_width": st["log2_width"]},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "step kernels of a pass (sweep form, and node form for steps wider than LDS)"},
        "flops_per_sample": st["flops_per_sample"],
        "sweep_flops_per_sample": sw["flops_per_sample"],
        "kernel_ms_per_step": kernel_ms / args.steps,
        "launches_per_step": launches / args.steps,
        "fp32_error_vs_fp64_noiseless": fp32_err,
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chains", type=int, default=0, help="override the chain count (default 4096)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-chains", type=int, default=5)
    ap.add_argument("--no-tune", action="store_true", help="skip the execution-form autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (reuse a decision)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_step_kernel_grid6x8.json"))
    ap.add_argument("--pmc-summary", nargs=5, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "TRACE_DIR"),
                    help="write the traffic file (--traffic) from rocprofv3 output directories and exit")
    ap.add_argument("--copy-bytes", type=float, default=float(2 ** 30))
    ap.add_argument("--workload", default="grid6x8",
                    choices=["grid6x8", "ladders_mixed", "noisy3reg", "grid6x8_noisy"],
                    help="grid6x8: the 48-qubit grid, 4096 chains (default); ladders_mixed: the 476-qubit "
                         "ladder (16384 chains) and 32 ladders of 100-400 qubits (1536 chains each), "
                         "sampled together in one captured graph; noisy3reg: noisy QAOA p=2 on a random "
                         "3-regular graph of --qubits nodes, 8192 chains; grid6x8_noisy: the grid with "
                         "the same noise, 4096 chains")
    ap.add_argument("--qubits", type=int, default=40, help="noisy3reg: graph size")
    args = ap.parse_args()
    if args.pmc_summary:
        _pmc_summary(*args.pmc_summary, args.traffic, args.copy_bytes)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (chains shard "
              "trivially across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import instances as I
    import paper_2510_24218_amd as E

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "ladders_mixed":
        _bench_ladders_mixed(args)
        return
    if args.workload in ("noisy3reg", "grid6x8_noisy"):
        _bench_noisy(args)
        return
    c, K, seed = I.workload_grid6x8()
    if args.chains:
        K = args.chains
    p32 = E.Plan(c, precision="fp32")
    st = p32.stats()
    tuned = p32.autotune(K, seed + 5000, args.tune_cache) if not args.no_tune else "default"
    out = torch.zeros((K, p32.words), dtype=torch.int64, device="cuda")
    for i in range(args.warmup):
        p32.sample(K, seed + i, out=out)
    torch.cuda.synchronize()
    kernel_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        p32.sample(K, seed + 1000 + i, out=out)
        ms, nl = p32.last_timing()
        kernel_ms += ms
        launches += nl
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = K / (ms_per_step / 1e3)
    flops_total = st["flops_per_sample"] * K * args.steps
    tflops = flops_total / (kernel_ms / 1e3) / 1e12
    sw = p32.sweep_stats()
    lds_gbs = sw["tensor_bytes_per_sample"] * K * args.steps / (kernel_ms / 1e3) / 1e9
    # node-form steps (if any) move their tensors through device memory
    bytes_total = st["bytes_per_sample"] * K * args.steps
    hbm_alg_gbs = bytes_total / (kernel_ms / 1e3) / 1e9

    # FP64 engine: reference for the FP32 error and its own throughput
    p64 = E.Plan(c, precision="fp64")
    p64.sample(K, seed, out=out)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    p64.sample(K, seed + 7, out=out)
    torch.cuda.synchronize()
    fp64_sps = K / (time.perf_counter() - t2)
    fp32_err = _fp32_error_vs_fp64(c, p32, p64, np.random.default_rng(5))

    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a
    # plain-copy calibration), valid only while the kernel sources are unchanged
    traffic = None
    if os.path.exists(args.traffic):
        rec = json.load(open(args.traffic))
        if rec.get("source_sha") == _source_sha():
            traffic = rec.get("bytes_per_launch")

    line = {
        "metric": "exact samples/sec + contraction TFLOP/s (FP32 vs BF16x3) at fixed error vs FP64",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qaoa_maxcut_grid6x8_p2", "n_qubits": c.n_qubits, "edges": len(c.edges),
                   "p": 2, "chains": K, "contraction_steps": p32.n_steps(), "precision": "fp32",
                   "draw": "fp64", "planner": "best of greedy/sweep", "log2_width": st["log2_width"],
                   "execution": tuned.split(" |")[0]},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "step kernel (sweep form), all contraction launches of a pass",
                     "flops_per_launch": st["flops_per_sample"] * K / max(launches / args.steps, 1),
                     "lds": {"achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                             "frac": lds_gbs / LDS_PEAK_GBS,
                             "bytes_per_launch": sw["tensor_bytes_per_sample"] * K / max(launches / args.steps, 1)}},
        "sweep_steps": sw["n_sweep_steps"],
        "hbm_algorithmic_gbs_node_form_steps": hbm_alg_gbs,
        "contraction_tflops_fp32": tflops,
        "contraction_frac_of_fp32_vector_peak": tflops / FP32_VECTOR_PEAK_TFLOPS,
        "contraction_tflops_bf16x3": None,
        "flops_per_sample": st["flops_per_sample"],
        "kernel_ms_per_step": kernel_ms / args.steps,
        "launches_per_step": launches / args.steps,
        "fp32_error_vs_fp64": fp32_err,
        "fp64_samples_per_s": fp64_sps,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = _cpu_baseline(c, seed, args.cpu_chains)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
