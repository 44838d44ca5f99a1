#!/usr/bin/env python3
"""Benchmark of the field + stochastic Heun hot path on one MI355X.

Workload (default): bcc lattice as two sublattices, 128^3 cells (4,194,304
spins), periodic, exchange shells 1-5 (J = 1.33, 0.75, -0.05, -0.10, 0.07 meV),
K = 0.005 meV along z, ferromagnet + seeded tilt, stochastic LLG Heun at
T = 300 K, alpha = 0.05, dt = 0.1 fs, Philox noise, FP32 field / FP64 state.
A bench "step" is one full Heun step (predictor + corrector, both field
evaluations, noise, renormalisation) of the whole lattice; the throughput is
spin-steps per second with the state already resident in HBM.

Prints one JSON line with the roofline fraction of the dominant kernel (the
Heun corrector) measured live with HIP events on its launch stream, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "spin updates/s (field+Heun), % HBM peak; GNEB iters learned vs plain init"
# Algorithmic HBM bytes per spin for each kernel of one Heun step (FP64 SoA
# state, 24 B per spin state): the predictor reads S and writes S~ (48 B), the
# corrector reads S and S~ and writes S' (72 B); neighbour reuse is on chip.
BYTES_PER_SPIN = {"heun_predict": 48, "heun_correct": 72}
KERNEL_SOURCES = ["paper_2605_26016_amd/csrc/spx_kernels.hip", "paper_2605_26016_amd/csrc/spx_device.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(w, seconds: float):
    """The FP64 oracle (as it stands) on the full lattice, whole Heun steps,
    repeated until about `seconds` of CPU work."""
    import oracle
    from tests.helpers import oracle_model
    m = oracle_model(w)
    S = w.initial_state()
    steps = 0
    t0 = time.perf_counter()
    while True:
        S = oracle.heun(m, S, alpha=w.alpha, dt_fs=w.dt_fs, T_K=w.T_K, seed=w.philox_seed, step0=steps,
                        n_steps=1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or (steps >= 2 and el * (steps + 1) / steps > 2.5 * seconds):
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.N * steps / el, "unit": "spin-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full Heun step(s) of the {w.N}-spin lattice, FP64 oracle, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bcc128_5shell_stochastic_mixed")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_26016_amd import spx
    from workloads import WORKLOADS

    w = WORKLOADS[args.workload]()
    log(f"[bench] workload {w.name}: {w.N} spins, {args.warmup} warmup + {args.steps} timed Heun steps")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = spx.setup_hamiltonian(w.L, cell=w.cell, sub_frac=w.frac, mu=w.mu, periodic=w.periodic,
                              J_shell=w.J_shell, D_shell=w.D_shell, K=(w.K if w.K else None),
                              K_axis=w.K_axis, B=w.B, dipolar=w.dipolar, field_prec=w.field_prec)
    S = torch.from_numpy(w.initial_state()).cuda()
    params = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed)
    spx.llg_heun_step(h, S, step0=0, n_steps=args.warmup, **params)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    spx.set_kernel_timing(h, True)
    for k in ("heun_predict", "heun_correct"):
        spx.get_kernel_times(h, k)  # reset
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    spx.llg_heun_step(h, S, step0=args.warmup, n_steps=args.steps, **params)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    spx.set_kernel_timing(h, False)
    kt = {k: spx.get_kernel_times(h, k) for k in ("heun_predict", "heun_correct")}
    log(f"[bench] timed region: {gpu_ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall)")
    t = max(gpu_ms / 1e3, 1e-12)
    value = w.N * args.steps / t
    # sanity: the state stays on the unit sphere
    nrm = torch.sqrt((S * S).sum(0))
    assert float((nrm - 1).abs().max()) < 1e-12, "state left the unit sphere"

    kernels = {}
    for k, (cnt, tot) in kt.items():
        avg = tot / max(cnt, 1) / 1e3
        kernels[k] = {"launches": cnt, "avg_us": avg * 1e6,
                      "GBps_algorithmic": BYTES_PER_SPIN[k] * w.N / avg / 1e9}
    dom = "heun_correct"
    achieved = kernels[dom]["GBps_algorithmic"]
    traffic = measured_traffic(dom)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_heun_correct",
            "bytes_per_launch_algorithmic": BYTES_PER_SPIN[dom] * w.N}
    step_bytes = sum(BYTES_PER_SPIN.values())
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"[bench] cpu oracle: {cpu['value']:.3e} spin-steps/s on {cpu['cores']} threads")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 field + f64 state" if w.field_prec == "fp32" else "f64",
        "data": "synthetic (seeded FM + tilt start, Philox noise)",
        "config": {"workload": w.name, "lattice": "bcc (2 sublattices)" if w.n_sub == 2 else "sc",
                   "cells": list(w.L), "spins": w.N, "shells": w.n_shells, "T_K": w.T_K,
                   "alpha": w.alpha, "dt_fs": w.dt_fs, "field_prec": w.field_prec,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "step_effective_GBps": step_bytes * w.N * args.steps / t / 1e9,
        "hbm_frac_step": step_bytes * w.N * args.steps / t / 1e9 / HBM_PEAK_GBS,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
