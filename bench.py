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
TWO_SWEEP_BYTES = 120
# the temporally fused step reads S and writes S' once (predicted state on chip)
BYTES_FUSED = 48
# field only: FP64 spin in, FP32 field out
FIELD_BYTES = 36
# MI355X vector FP32 peak (packed FP32 instructions: two FMAs per lane; the
# library is built without them, which halves the rate it can reach)
FP32_VECTOR_PEAK_TFLOPS = 157.3
# dense 7^3 window of 3x3 blocks: 342 offsets x 9 multiply-adds x 2 flop
DENSE_FLOP_PER_SITE = 6156
MFMA_BF16_PEAK_TFLOPS = 2500.0
KERNEL_SOURCES = ["paper_2605_26016_amd/csrc/spx_kernels.hip", "paper_2605_26016_amd/csrc/spx_device.hpp",
                  "paper_2605_26016_amd/csrc/spx_stencil.hip", "paper_2605_26016_amd/csrc/spx_stencil.hpp",
                  "paper_2605_26016_amd/csrc/spx_internal.hpp", "paper_2605_26016_amd/csrc/spx_fused.hip",
                  "paper_2605_26016_amd/csrc/spx_math.hpp"]
# corrector kernel name per stencil engine (1 gather, 2 z-march)
CORRECT_KERNEL = {1: "k_heun_correct", 2: "k_zmarch (corrector instantiation)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(paths=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, heun_mode, zchunk, tile_rows=0):
    """HBM bytes per launch (per iteration for the GNEB entry) from the
    committed rocprofv3 --pmc summary, if it was taken on the current source
    of the files it lists, on this workload and in this launch configuration
    (else None).  An entry holds one record per launch configuration it was
    measured in ("configs": z chunk, Heun mode, fused rows, bytes)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(e.get("sources", KERNEL_SOURCES)):
        return None
    if e.get("workload") != workload:
        return None
    for c in e.get("configs", [e]):
        if (c.get("heun_mode"), c.get("zchunk"), c.get("tile_rows", 0)) == (heun_mode, zchunk, tile_rows or 0):
            return c.get("bytes_per_launch")
    return None


def cpu_baseline(w, seconds: float):
    """The FP64 oracle (as it stands) on the full lattice, whole Heun steps,
    repeated until about `seconds` of CPU work."""
    import oracle
    from tests.helpers import oracle_model
    what = f"the {w.N}-spin lattice"
    if w.N > 50_000_000:
        # the full lattice does not fit the host's memory three times over:
        # the same physics on 256^3 cells, per spin-step
        w = w.scaled((256, 256, 256))
        what = f"a {w.N}-spin (256^3) lattice of the same model"
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
            "sample": f"{steps} full Heun step(s) of {what}, FP64 oracle, {el:.1f} s"}


# GNEB per spin-image-iteration, the lower bound the roofline is scored
# against: a first pass reads S_n, S_n+1 and writes F (72 B), a second pass
# reads S_n, S_n+-1, F, v and writes S, v (168 B)
GNEB_BYTES = 240
# what the library's two z-march passes move (no stored force): the first
# reads S_n, S_n-1, S_n+1 and v (96 B), the second reads S_n, S_n-1, S_n+1, v
# and writes v, S' (120 B)
GNEB_PASS_BYTES = 216
# string method per spin-image: the projection pass without velocities
# (read S_n, S_n-1, S_n+1: 72 B), the update pass without velocities (read
# S_n, S_n-1, S_n+1, write S': 96 B), the reparameterisation's distance pass
# (2 images per pair: 48 B) and interpolation (2 images read, 1 written: 72 B)
STRING_BYTES = 72 + 96 + 48 + 72


def gneb_workload(args):
    """Batched ragged GNEB throughput on 48^3, 64^3, 96^3 x 32 images (one
    persistent launch set per pass), and the learned-versus-geodesic initial
    path comparison on hopfion annihilation paths."""
    import numpy as np
    import torch

    from paper_2605_26016_amd import pathinit, spx
    from workloads import hopfion_texture, sc_frustrated_gneb, uniform_state

    out = {"metric": "GNEB iterations to convergence, learned vs geodesic initial path; batched GNEB "
                     "spin-image-iterations/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (network f32)", "data": "synthetic (seeded hopfion textures)"}
    # -- throughput: the config as given (3-shell model), seeded texture -> FM, 32 images each
    sizes = (48, 64, 96)
    hams, imgs = [], []
    for L in sizes:
        w = sc_frustrated_gneb((L, L, L), shells="config3")
        h = spx.setup_hamiltonian(w.L, periodic=w.periodic, J_shell=w.J_shell, field_prec="fp64")
        Y = torch.zeros((32, 3, w.N), dtype=torch.float64, device="cuda")
        Y[0] = torch.from_numpy(hopfion_texture(w.L)).cuda()
        Y[-1] = torch.from_numpy(uniform_state(w.N)).cuda()
        hams.append(h)
        imgs.append(Y)
    g = spx.gneb_create(hams, imgs, ci_mode=1, ci_on_below=1e-2, tol_force=0.0)
    spx.gneb_init_path(g)
    spx.gneb_step(g, 5)
    torch.cuda.synchronize()
    n_it = args.steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    spx.gneb_step(g, n_it)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    spin_images = sum(32 * L ** 3 for L in sizes)
    rate = spin_images * n_it / (ms / 1e3)
    out.update({"value": rate, "unit": "spin-image-iterations/s", "steps": n_it, "warmup": 5,
                "ms_per_step": ms / n_it,
                "roofline": {"bound": "hbm", "achieved": rate * GNEB_BYTES / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": rate * GNEB_BYTES / 1e9 / HBM_PEAK_GBS,
                             "traffic": measured_traffic("gneb_iteration", "sc_frustrated_gneb", None, 16),
                             "kernel": "GNEB iteration (two z-march passes + reductions)",
                             "bytes_per_spin_image_iteration": GNEB_BYTES,
                             "bytes_per_spin_image_iteration_of_the_passes": GNEB_PASS_BYTES,
                             "GBps_of_the_passes": rate * GNEB_PASS_BYTES / 1e9}})
    log(f"[bench] batched GNEB: {rate:.3e} spin-image-iterations/s ({ms / n_it:.3f} ms per iteration)")
    # -- the same three instances as three separate GNEB objects, one after
    # another on the same stream (the unbatched path)
    singles = [spx.gneb_create([h], [Y], ci_mode=1, ci_on_below=1e-2, tol_force=0.0) for h, Y in zip(hams, imgs)]
    for gs in singles:
        spx.gneb_step(gs, 5)
    torch.cuda.synchronize()
    e0.record()
    for gs in singles:
        spx.gneb_step(gs, n_it)
    e1.record()
    torch.cuda.synchronize()
    ms_1 = e0.elapsed_time(e1)
    out["per_instance"] = {"ms_per_iteration": ms_1 / n_it, "spin_image_iterations_per_s": spin_images * n_it / (ms_1 / 1e3),
                           "batched_speedup": ms_1 / ms,
                           "what": "each lattice its own GNEB object, stepped one after another on one stream"}
    log(f"[bench] per-instance GNEB: {ms_1 / n_it:.3f} ms per iteration (batched {ms / n_it:.3f} ms)")
    del singles
    # -- the string method on the same batch: force step + geodesic reparameterisation
    spx.gneb_set_params(g, vp_dt=0.01, ci_mode=4, tol_force=0.0)
    spx.gneb_step(g, 3)
    torch.cuda.synchronize()
    e0.record()
    spx.gneb_step(g, n_it)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    rate_s = spin_images * n_it / (ms_s / 1e3)
    out["string_method"] = {"ms_per_iteration": ms_s / n_it, "spin_image_iterations_per_s": rate_s,
                            "bytes_per_spin_image_iteration": STRING_BYTES,
                            "GBps_algorithmic": rate_s * STRING_BYTES / 1e9,
                            "hbm_frac": rate_s * STRING_BYTES / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] string method: {rate_s:.3e} spin-image-iterations/s ({ms_s / n_it:.2f} ms per iteration)")
    out["config"] = {"workload": "sc_frustrated_gneb", "lattices": [list((L, L, L)) for L in sizes], "images": 32,
                     "spin_images": spin_images, "shells_throughput": [1.0, -0.164, -0.082],
                     "parallelism": "single GPU, ragged batch: one launch per instance and pass, the instances on parallel graph branches"}
    del g, hams, imgs
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_gneb_baseline(args.cpu_seconds)
    out["hbm_copy_GBps"] = copy_bandwidth()
    out["net_forward"] = net_forward_roofline()
    if args.no_learned:
        print(json.dumps(out), flush=True)
        return
    out["learned_init"] = {fam: learned_experiment(fam, args) for fam in args.families.split(",")}
    print(json.dumps(out), flush=True)


# useful flops of the path corrector's forward per site: four 3^3
# convolutions 10 -> 16 -> 16 -> 16 -> 3 channels, two flops per product
NET_FLOP_PER_SITE = 2 * 27 * (10 * 16 + 16 * 16 + 16 * 16 + 16 * 3)
# HBM bytes per site of one BF16 forward with per-image end states: the input
# pass reads S_g, S_A, S_B (72) and writes the BF16 activations (32); each
# hidden layer reads and writes 32; the last reads 32 and writes u (12); the
# head reads u and S_g (36) and writes S_hat (24).  At 97 flop per byte the
# forward sits below the MFMA ridge (2500 / 8000 = 312 flop per byte): HBM
# bounds it.
NET_BYTES_PER_SITE = 104 + 3 * 64 + 44 + 60


def net_forward_roofline(L=(64, 64, 64), batch=16, reps=10):
    """The path corrector's forward (dilation 1, 2, 4, 8) on a batch of
    64^3 images with random parameters and states, FP32 on the vector ALUs and
    BF16 implicit GEMMs on the matrix cores.  The BF16 form's roofline is
    HBM's (its bytes per site above); its rate of useful flops (the padding
    of channels to 16 and of the 27 taps to 28 not counted) is also given
    against the dense BF16 MFMA peak."""
    import torch

    from paper_2605_26016_amd import pathinit, spx
    N = L[0] * L[1] * L[2]
    gen = torch.Generator(device="cuda").manual_seed(7)

    def unit():
        v = torch.randn((batch, 3, N), dtype=torch.float64, device="cuda", generator=gen)
        return v / v.norm(dim=1, keepdim=True)

    Sg, SA, SB = unit(), unit(), unit()
    t = torch.linspace(0.1, 0.9, batch, dtype=torch.float32, device="cuda")
    p = torch.from_numpy(pathinit.init_params(1)).float().cuda()
    out = torch.empty((batch, 3, N), dtype=torch.float64, device="cuda")
    res = {"images": batch, "lattice": list(L), "dilation": [1, 2, 4, 8],
           "flop_per_site_useful": NET_FLOP_PER_SITE}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for prec in ("fp32", "bf16"):
        net = spx.Net(dilation=(1, 2, 4, 8))
        spx.net_set_precision(net, prec)
        spx.net_forward(net, p, L, batch, Sg, SA, SB, t, out)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            spx.net_forward(net, p, L, batch, Sg, SA, SB, t, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[prec + "_ms"] = ms
        res[prec + "_TFLOPs"] = batch * N * NET_FLOP_PER_SITE / ms / 1e9
        del net
    gbs = batch * N * NET_BYTES_PER_SITE / res["bf16_ms"] / 1e6
    res["mfma_frac"] = round(res["bf16_TFLOPs"] / MFMA_BF16_PEAK_TFLOPS, 4)
    traffic = measured_traffic("net_forward_bf16", f"net_forward_{L[0]}x{L[1]}x{L[2]}_x{batch}", None, None)
    res["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "bytes_per_site": NET_BYTES_PER_SITE,
                       "kernel": "BF16 network forward (k_net_input_bf16, 4 x k_conv_mfma, k_net_head)"}
    log(f"[bench] network forward 64^3 x {batch}: FP32 {res['fp32_ms']:.3f} ms, BF16 MFMA {res['bf16_ms']:.3f} ms "
        f"({res['bf16_TFLOPs']:.1f} TFLOP/s, {gbs:.0f} GB/s)")
    return res


# Monte Carlo per attempted update: the spin is read (as a neighbour) and
# written once per sweep at the least
MC_BYTES = 48
MC_SHELLS = ((1.0,), (1.0, 0.3), (1.0, 0.3, 0.1), (1.0, 0.3, 0.1, 0.05), (1.0, 0.3, 0.1, 0.05, 0.02))


def mc_workload(args):
    """FP64 heat-bath and Metropolis Monte Carlo on sc 200^3 (Methods, Monte
    Carlo sampling): attempted spin updates/s for 1 .. 5 exchange shells, and
    the colour count each needs.  The headline value is heat-bath with one
    shell."""
    import torch

    from paper_2605_26016_amd import spx
    from workloads import random_sphere_device
    L, T = 200, 500.0
    N = L ** 3
    S = random_sphere_device(N, 3)
    n = max(1, args.steps)
    table = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for J in MC_SHELLS:
        h = spx.setup_hamiltonian((L, L, L), J_shell=J, field_prec="fp64", B=(0.0, 0.0, 1.0))
        C, _ = spx.mc_colouring(h)
        row = {"shells": len(J), "colours": C}
        for method in ("heat_bath", "metropolis"):
            spx.mc_sweep(h, S, T, seed=1, sweep0=0, n_sweeps=args.warmup if len(J) == 1 else 2, method=method)
            torch.cuda.synchronize()
            e0.record()
            spx.mc_sweep(h, S, T, seed=1, sweep0=1000, n_sweeps=n if len(J) == 1 else max(1, n // 10),
                         method=method)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (n if len(J) == 1 else max(1, n // 10))
            row[method] = {"ms_per_sweep": ms, "updates_per_s": N / (ms / 1e3)}
        table.append(row)
        log(f"[bench] MC {len(J)} shell(s), {C} colours: heat-bath {row['heat_bath']['updates_per_s']:.3e}, "
            f"Metropolis {row['metropolis']['updates_per_s']:.3e} updates/s")
        del h
    head = table[0]["heat_bath"]
    rate = head["updates_per_s"]
    out = {"metric": "attempted spin updates/s (heat-bath Monte Carlo, FP64)", "value": rate,
           "unit": "spin-updates/s", "n_gpus": 1, "steps": n, "warmup": args.warmup,
           "ms_per_step": head["ms_per_sweep"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic (seeded random spins)",
           "config": {"workload": "sc200_mc", "cells": [L, L, L], "spins": N, "T_K": T, "B_T": [0.0, 0.0, 1.0],
                      "shells": [list(J) for J in MC_SHELLS], "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "achieved": rate * MC_BYTES / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": rate * MC_BYTES / 1e9 / HBM_PEAK_GBS,
                        "traffic": measured_traffic("mc_heat_bath_1shell", "sc200_mc", None, None),
                        "kernel": "k_mc_colour_cm (heat-bath, one shell, 2 colours)",
                        "bytes_per_update_algorithmic": MC_BYTES},
           "table": table}
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_mc_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


# static minimiser iteration, per spin: field pass (24 B in, 24 B out) +
# force pass (read S, b, u_prev, F_prev; write F) + update pass (read S, F;
# write S, u, F_prev): 48 + 120 + 120 B, plus the L-BFGS two-loop passes
MIN_BYTES = {"vp": 48 + 120 + 144, "bb": 48 + 120 + 120, "lbfgs": 48 + 120 + 120, "adam": 48 + 72 + 192}


def min_workload(args):
    """FP64 static minimisers on sc 200^3 with a fixed number of iterations
    (Methods, static optimisation): spin-site updates/s (spins x iterations /
    time) for 1 .. 5 exchange shells; the headline value is velocity
    projection with one shell."""
    import torch

    from paper_2605_26016_amd import spx
    from workloads import random_sphere_device
    L = 200
    N = L ** 3
    n = max(1, args.steps // 10)
    table = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for J in MC_SHELLS:
        h = spx.setup_hamiltonian((L, L, L), J_shell=J, field_prec="fp64", K=0.1, B=(0.0, 0.0, 1.0))
        row = {"shells": len(J)}
        for method, kw in (("vp", dict(dt=0.1)), ("bb", dict(dt=0.02)), ("lbfgs", dict(dt=0.02, history=5)),
                           ("adam", dict(dt=0.01))):
            S = random_sphere_device(N, 3)
            mn = spx.min_create(h, method=method, max_step=0.2, **kw)
            spx.min_step(mn, S, 2)
            torch.cuda.synchronize()
            e0.record()
            spx.min_step(mn, S, n)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n
            row[method] = {"ms_per_iteration": ms, "updates_per_s": N / (ms / 1e3)}
            del mn, S
        table.append(row)
        log(f"[bench] minimisers, {len(J)} shell(s): " +
            ", ".join(f"{k} {row[k]['updates_per_s']:.3e}" for k in ("vp", "bb", "lbfgs", "adam")))
        del h
    head = table[0]["vp"]
    rate = head["updates_per_s"]
    out = {"metric": "spin-site updates/s (static minimisation, fixed iterations, FP64)", "value": rate,
           "unit": "spin-iterations/s", "n_gpus": 1, "steps": n, "warmup": 2,
           "ms_per_step": head["ms_per_iteration"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded random spins)",
           "config": {"workload": "sc200_min", "cells": [L, L, L], "spins": N, "K_meV": 0.1, "B_T": [0.0, 0.0, 1.0],
                      "shells": [list(J) for J in MC_SHELLS], "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "achieved": rate * MIN_BYTES["vp"] / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": rate * MIN_BYTES["vp"] / 1e9 / HBM_PEAK_GBS,
                        "traffic": measured_traffic("min_vp_iteration", "sc200_min", None, None),
                        "kernel": "velocity-projection iteration (field, force, update)",
                        "bytes_per_spin_iteration": MIN_BYTES["vp"]},
           "table": table, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def pairlist_workload(args):
    """The pair-list backend against the lattice engine on the same sc 200^3
    nearest-neighbour model (the paper's backend comparison): field
    evaluations/s and Heun spin-steps/s, FP64 and FP32 field.  The headline
    value is the FP32-field pair-list Heun throughput."""
    import numpy as np
    import torch

    from paper_2605_26016_amd import spx
    from workloads import random_sphere_device
    L = 200
    N = L ** 3
    idx = np.arange(N, dtype=np.int64)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    tgt, src = [], []
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        tgt.append(idx)
        src.append((x + d[0]) % L + L * (((y + d[1]) % L) + L * ((z + d[2]) % L)))
    tgt, src = np.concatenate(tgt), np.concatenate(src)
    J = np.ones(len(tgt))
    S0 = random_sphere_device(N, 3)
    n = max(1, args.steps // 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    table = {}
    for backend in ("pairlist", "lattice"):
        for prec in ("fp64", "fp32"):
            if backend == "pairlist":
                h = spx.setup_pairlist(N, tgt, src, J, field_prec=prec)
            else:
                h = spx.setup_hamiltonian((L, L, L), J_shell=(1.0,), field_prec=prec)
            b = torch.empty((3, N), dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
            S = S0.clone()
            ms_f = timed(lambda: spx.eval_field(h, S, b))
            ms_h = timed(lambda: spx.llg_heun_step(h, S, alpha=0.1, dt_fs=0.1, temperature_K=0.0, n_steps=1))
            table[f"{backend}_{prec}"] = {"field_ms": ms_f, "fields_per_s": N / (ms_f / 1e3), "heun_ms": ms_h,
                                          "spin_steps_per_s": N / (ms_h / 1e3)}
            log(f"[bench] {backend} {prec}: field {N / (ms_f / 1e3):.3e}/s, Heun {N / (ms_h / 1e3):.3e} spin-steps/s")
            del h, b, S
    head = table["pairlist_fp32"]
    # pair-list field contract bytes per site: the spin array read once 24 B
    # (each spin as some site's source), 6 sources (4 B index + 4 B FP32
    # coupling), row pointer 8 B, FP32 field out 12 B
    pl_bytes = 24 + 6 * 8 + 8 + 12
    out = {"metric": "spin updates/s (field+Heun), pair-list backend, sc 200^3 nearest neighbours",
           "value": head["spin_steps_per_s"], "unit": "spin-steps/s", "n_gpus": 1, "steps": n, "warmup": 1,
           "ms_per_step": head["heun_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 field (f64 state)", "data": "synthetic (seeded random spins)",
           "config": {"workload": "sc200_pairlist", "cells": [L, L, L], "spins": N, "pairs": int(len(tgt)),
                      "parallelism": "single GPU"},
           "roofline": {"bound": "hbm", "achieved": head["fields_per_s"] * pl_bytes / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": head["fields_per_s"] * pl_bytes / 1e9 / HBM_PEAK_GBS,
                        "traffic": measured_traffic("pl_field_fp32", "sc200_pairlist", None, None),
                        "kernel": "k_pl_field<float> (pair-list FP32 field)",
                        "bytes_per_site_algorithmic": pl_bytes},
           "table": table, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def cpu_mc_baseline(seconds):
    """The FP64 oracle's heat-bath sweeps on sc 48^3 (one shell)."""
    import oracle
    from tests.helpers import oracle_model
    from workloads import Workload, random_sphere
    w = Workload(name="mc", L=(48, 48, 48), J_shell=(1.0,), B=(0.0, 0.0, 1.0))
    m = oracle_model(w)
    S = random_sphere(w.N, 3)
    col = oracle.mc_colouring(m)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.mc_sweeps(m, S, 500.0, 1, sweep0=n, n_sweeps=1, method=0, colouring=col)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or el * (n + 1) / n > 2.5 * seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.N * n / el, "unit": "spin-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} heat-bath sweeps of sc 48^3 (one shell), {el:.1f} s"}


def cpu_gneb_baseline(seconds):
    """FP64 oracle GNEB iterations on the 48^3 x 32-image instance."""
    import oracle
    from tests.helpers import oracle_model
    from workloads import hopfion_texture, sc_frustrated_gneb, uniform_state
    w = sc_frustrated_gneb((48, 48, 48), shells="config3")
    m = oracle_model(w)
    st = oracle.GnebState(oracle.geodesic_path(hopfion_texture(w.L), uniform_state(w.N), 32), ci_mode=1,
                          ci_on_below=1e-2)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.gneb_iterate(m, st)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or el * (n + 1) / n > 2.5 * seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 32 * w.N * n / el, "unit": "spin-image-iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} GNEB iteration(s) of the 48^3 x 32-image instance, FP64 oracle, {el:.1f} s"}


def learned_experiment(family, args):
    """Learned versus geodesic initial paths on held-out end states of one
    family (see pathinit.learned_vs_geodesic)."""
    from paper_2605_26016_amd import pathinit
    tr = None
    if args.train_sizes:
        tr = tuple((int(e.split(":")[0]), float(e.split(":")[1]) if ":" in e else 1.0)
                   for e in args.train_sizes.split(","))
    te = tuple(int(e) for e in args.test_sizes.split(",")) if args.test_sizes else None
    dil = tuple(int(v) for v in args.dilation.split(",")) if args.dilation else None
    damp = tuple(float(v) for v in args.damping.split(",")) if args.damping else ()
    return pathinit.learned_vs_geodesic(family, n_train=args.n_train, n_test=args.n_test, epochs=args.epochs,
                                        lr=args.lr, max_iter=args.max_iter, train_sizes=tr, test_sizes=te,
                                        n_img_test=args.test_images, dilation=dil, endpoint_tol=args.endpoint_tol,
                                        damping=damp, log=log)


def heun_workload(args, w, steps=None, warmup=None, cpu=True):
    """Field + (stochastic) Heun throughput of one lattice workload; returns
    the JSON record.  The timed region replays the library's captured Heun
    graphs (the production path) and is bracketed by HIP events on the launch
    stream; per-kernel durations come from a separate pass of direct launches
    with events around every launch."""
    import numpy as np
    import torch

    from paper_2605_26016_amd import spx
    from workloads import random_sphere_device

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    log(f"[bench] workload {w.name}: {w.N} spins, {warmup} warmup + {steps} timed Heun steps")
    stream = torch.cuda.current_stream()
    h = spx.setup_hamiltonian(w.L, cell=w.cell, sub_frac=w.frac, mu=w.mu, periodic=w.periodic,
                              J_shell=w.J_shell, D_shell=w.D_shell, K=(w.K if w.K else None),
                              K_axis=w.K_axis, B=w.B, dipolar=w.dipolar, field_prec=w.field_prec,
                              autotune=0 if args.no_autotune else 1, tune_cache_path=args.tune_cache)
    info = spx.get_info(h)
    log(f"[bench] engine {info.stencil_engine} shape {info.shape} zchunk {info.zchunk} "
        f"heun_field {info.heun_field} tile_rows {info.tile_rows} tuned {info.tuned} "
        f"({info.tuned_step_us:.1f} us/step while tuning), "
        f"library workspace {info.workspace_bytes / 2**30:.2f} GiB")
    if w.N > 200_000_000:
        # too large to draw on the host in reasonable time: torch's seeded device generator
        S = random_sphere_device(w.N, w.init_seed)
        data = "synthetic (seeded uniform random start drawn on the device, Philox noise)"
    else:
        S = torch.from_numpy(w.initial_state()).cuda()
        data = "synthetic (seeded start, Philox noise)" if w.T_K > 0 else "synthetic (seeded start)"
    params = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed)
    spx.llg_heun_step(h, S, step0=0, n_steps=warmup, **params)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    fused = info.heun_field == 8
    kinds = ("heun_predict", "heun_correct", "noise")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    spx.llg_heun_step(h, S, step0=warmup, n_steps=steps, **params)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"[bench] timed region: {gpu_ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall)")
    # per-kernel durations: a separate pass with events around every launch
    spx.set_kernel_timing(h, True)
    for k in kinds:
        spx.get_kernel_times(h, k)  # reset
    n_kt = min(steps, 10 if w.N > 100_000_000 else 100)
    spx.llg_heun_step(h, S, step0=warmup + steps, n_steps=n_kt, **params)
    torch.cuda.synchronize()
    spx.set_kernel_timing(h, False)
    kt = {k: spx.get_kernel_times(h, k) for k in kinds}
    t = max(gpu_ms / 1e3, 1e-12)
    value = w.N * steps / t
    nrm = torch.sqrt((S * S).sum(0))
    assert float((nrm - 1).abs().max()) < 1e-12, "state left the unit sphere"
    del nrm

    bps = dict(BYTES_PER_SPIN)
    if fused:
        bps = {"heun_predict": BYTES_FUSED}  # kind 0 times the one fused launch
    kernels = {}
    for k, (cnt, tot) in kt.items():
        if cnt == 0:
            continue
        avg = tot / cnt / 1e3
        name = "heun_fused" if (fused and k == "heun_predict") else k
        kernels[name] = {"launches": cnt, "avg_us": avg * 1e6}
        if k in bps:
            kernels[name]["GBps_algorithmic"] = bps[k] * w.N / avg / 1e9
    if fused:
        # one fused launch per step (plus one step-counter node per 16-step
        # graph): the kernel's average duration over the timed region is the
        # region divided by its launches
        dom = "heun_fused"
        avg_s = t / steps
        achieved = BYTES_FUSED * w.N / avg_s / 1e9
        kname = "k_heun_fused (predictor + corrector, one pass)"
        timing = ("HIP events around the timed region of graph-replayed steps on the launch stream, "
                  "one fused launch per step; per-launch events in a separate pass: "
                  f"{kernels['heun_fused']['avg_us']:.1f} us")
        bpl = BYTES_FUSED
        step_bytes = BYTES_FUSED
    else:
        # the dominant kernel: the stage with the larger summed time in the
        # per-launch pass
        dom = max(("heun_predict", "heun_correct"), key=lambda k: kt[k][1])
        achieved = kernels[dom]["GBps_algorithmic"]
        kname = {("heun_predict", 2): "k_zmarch (predictor instantiation)",
                 ("heun_correct", 2): "k_zmarch (corrector instantiation)",
                 ("heun_predict", 1): "k_heun_predict", ("heun_correct", 1): "k_heun_correct"}
        if info.stencil_engine == 2 and info.heun_field in (5, 6):
            kname[("heun_predict", 2)] = "k_zmarch<ZM_BIL> + k_heun_pre (predictor sweep)"
            if info.heun_field == 5:
                kname[("heun_correct", 2)] = "k_zmarch<ZM_BIL> + k_heun_post (corrector sweep)"
        kname = kname.get((dom, info.stencil_engine), dom)
        timing = "HIP events around every launch in a separate pass of direct launches after the timed region"
        bpl = BYTES_PER_SPIN[dom]
        step_bytes = sum(BYTES_PER_SPIN.values())
    traffic = measured_traffic(dom, w.name, info.heun_field, info.zchunk, info.tile_rows)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
            "bytes_per_spin_algorithmic": bpl, "bytes_per_launch_algorithmic": bpl * w.N,
            "kernel_timing": timing}
    cpu_rec = None
    if cpu and not args.no_cpu_baseline:
        log("[bench] timing the FP64 CPU oracle on a bounded sample ...")
        cpu_rec = cpu_baseline(w, args.cpu_seconds)
        log(f"[bench] cpu oracle: {cpu_rec['value']:.3e} spin-steps/s on {cpu_rec['cores']} threads")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": gpu_ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 field + f64 state" if w.field_prec == "fp32" else "f64",
        "data": data,
        "config": {"workload": w.name, "lattice": "bcc (2 sublattices)" if w.n_sub == 2 else "sc",
                   "cells": list(w.L), "spins": w.N, "shells": w.n_shells, "T_K": w.T_K,
                   "alpha": w.alpha, "dt_fs": w.dt_fs, "field_prec": w.field_prec,
                   "parallelism": "single GPU", "stencil_engine": info.stencil_engine,
                   "zchunk": info.zchunk, "heun_mode": info.heun_field, "tile_rows": info.tile_rows},
        "roofline": roof,
        "cpu_baseline": cpu_rec,
        "kernels": kernels,
        "step_effective_GBps": step_bytes * w.N * steps / t / 1e9,
        "hbm_frac_step": step_bytes * w.N * steps / t / 1e9 / HBM_PEAK_GBS,
        # the rate against the two-sweep roofline (120 B per spin-step at 8 TB/s)
        "two_sweep_roofline_frac": value / (HBM_PEAK_GBS * 1e9 / TWO_SWEEP_BYTES),
        "device": torch.cuda.get_device_name(0),
    }
    # the same steps with direct launches instead of the captured graph
    spx.set_heun_graph(h, False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_direct = min(steps, 20 if w.N > 100_000_000 else steps)
    e0.record(stream)
    spx.llg_heun_step(h, S, step0=warmup, n_steps=n_direct, **params)
    e1.record(stream)
    torch.cuda.synchronize()
    spx.set_heun_graph(h, True)
    out["direct_launch_ms_per_step"] = e0.elapsed_time(e1) / n_direct
    # energy of the final state (deterministic two-level reduction)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    spx.energy(h, S, E)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        spx.energy(h, S, E)
    e1.record(stream)
    torch.cuda.synchronize()
    out["energy"] = {"ms": e0.elapsed_time(e1) / 10, "meV_per_spin": float(E.item()) / w.N}
    if args.calibrate_copy:
        src = torch.empty_like(S).copy_(S)
        dst = torch.empty_like(S)
        for _ in range(4):
            spx.stream_probe(0, src, dst, src.numel() * 8)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 4 copies of {src.numel() * 8} bytes")
        del src, dst
    del S, h
    torch.cuda.empty_cache()
    return out


def headline(args):
    """The N = 1 line: the billion-spin sc 1024^3 stochastic workload, with the
    bcc 128^3 five-shell workload as a secondary record (same metric)."""
    from workloads import WORKLOADS
    out = heun_workload(args, WORKLOADS["sc1024_nn_stochastic_mixed"]())
    out["hbm_copy_GBps"] = copy_bandwidth()
    sec = heun_workload(args, WORKLOADS["bcc128_5shell_stochastic_mixed"](), steps=max(args.steps, 200),
                        warmup=max(args.warmup, 20), cpu=False)
    keep = ("value", "unit", "steps", "warmup", "ms_per_step", "config", "roofline", "kernels",
            "step_effective_GBps", "hbm_frac_step", "two_sweep_roofline_frac", "direct_launch_ms_per_step",
            "energy")
    out["secondary"] = {k: sec[k] for k in keep}
    print(json.dumps(out), flush=True)


def copy_bandwidth(nbytes=4 << 30, reps=5):
    """Attainable HBM bandwidth from the library's streaming probe over 4 GiB
    buffers (far beyond the on-die caches): copy (read + write bytes), read
    only and write only, each event-timed over `reps` passes."""
    import torch

    from paper_2605_26016_amd import spx
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    res = {}
    for kind, name, mult in ((0, "copy", 2.0), (1, "read", 1.0), (2, "write", 1.0)):
        spx.stream_probe(kind, a, b, nbytes)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            spx.stream_probe(kind, a, b, nbytes)
        e1.record()
        torch.cuda.synchronize()
        res[name] = round(mult * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    log(f"[bench] streaming probe over 4 GiB: copy {res['copy']} GB/s, read {res['read']} GB/s, "
        f"write {res['write']} GB/s")
    return res


def field_workload(args, w):
    """Field-only evaluations of the sc 256^3 chiral magnet: the FP32 stencil
    (J + DMI + Zeeman), the stencil plus the zero-padded FFT dipolar field,
    and the dense 7^3 window in BF16/FP16 MFMA and FP32 direct form against
    its FP64 evaluation."""
    import numpy as np
    import torch

    from paper_2605_26016_amd import spx

    stream = torch.cuda.current_stream()
    S = torch.from_numpy(w.initial_state()).cuda()
    b32 = torch.empty((3, w.N), dtype=torch.float32, device="cuda")

    def timed(h, out, reps):
        spx.eval_field(h, S, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            spx.eval_field(h, S, out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(args.steps, 1)
    common = dict(cell=w.cell, mu=w.mu, periodic=w.periodic, B=w.B)
    h = spx.setup_hamiltonian(w.L, J_shell=w.J_shell, D_shell=w.D_shell, dipolar=0, field_prec="fp32", **common)
    ms_st = timed(h, b32, reps)
    del h
    h = spx.setup_hamiltonian(w.L, J_shell=w.J_shell, D_shell=w.D_shell, dipolar=1, field_prec="fp32", **common)
    ms_dip = timed(h, b32, reps)
    del h
    log(f"[bench] stencil {ms_st * 1e3:.1f} us, stencil + dipolar FFT {ms_dip:.3f} ms")
    from workloads import dense7_couplings
    ab, dl, J9 = dense7_couplings(mu=w.mu[0], a=w.cell[0][0])
    b64 = torch.empty((3, w.N), dtype=torch.float64, device="cuda")
    h = spx.setup_hamiltonian(w.L, bonds=(ab, dl, J9), field_prec="fp64", **common)
    ms64 = timed(h, b64, 2)
    del h
    ref_max = float(b64.abs().max())
    dense = {}
    # bf16 / fp16: the MFMA window; fp32_direct: the FP32 direct window on the
    # vector ALUs (the plain path the MFMA forms are compared with);
    # fp32_gather: the generic gather kernel on the same bond table
    for name, prec, backend in (("bf16", "bf16", 2), ("fp16", "fp16", 2), ("fp32_direct", "fp32", 2),
                                ("fp32_gather", "fp32", 1)):
        h = spx.setup_hamiltonian(w.L, bonds=(ab, dl, J9), field_prec=prec, backend=backend, **common)
        ms = timed(h, b32, reps if name != "fp32_gather" else max(reps // 20, 2))
        err = float((b32.double() - b64).abs().max()) / ref_max
        tf = DENSE_FLOP_PER_SITE * w.N / ms / 1e9
        dense[name] = {"ms": ms, "fields_per_s": w.N / ms * 1e3, "TFLOPs_algorithmic": tf,
                       "max_rel_error_vs_fp64": err}
        log(f"[bench] K7 dense {name}: {ms:.3f} ms, {tf:.1f} TFLOP/s, error vs FP64 {err:.2e}")
        del h
    fd = dense["fp32_direct"]
    fd["frac_of_fp32_peak"] = fd["TFLOPs_algorithmic"] / FP32_VECTOR_PEAK_TFLOPS
    fd["frac_of_unpacked_fp32_peak"] = fd["TFLOPs_algorithmic"] / (FP32_VECTOR_PEAK_TFLOPS / 2)
    for name in ("bf16", "fp16"):
        dense[name]["speedup_over_fp32_direct"] = fd["ms"] / dense[name]["ms"]
    dense["fp64_direct_ms"] = ms64
    mf = dense["bf16"]
    roof = {"bound": "mfma", "achieved": round(mf["TFLOPs_algorithmic"], 2), "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(mf["TFLOPs_algorithmic"] / MFMA_BF16_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("dense_mfma_bf16", "sc256_chiral_dipolar_field", None, None),
            "kernel": "k_dense_mfma (BF16)",
            "flop_per_site_algorithmic": DENSE_FLOP_PER_SITE}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_field_baseline(w, args.cpu_seconds)
    out = {"metric": "field evaluations/s (sc 256^3 chiral magnet + dipolar FFT); dense 7^3 MFMA TFLOP/s",
           "value": w.N / ms_dip * 1e3, "unit": "fields/s", "n_gpus": 1, "steps": reps, "warmup": 1,
           "ms_per_step": ms_dip, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 field (f64 state); dense window bf16/fp16 MFMA with f32 accumulation",
           "data": "synthetic (seeded uniform random spins)",
           "config": {"workload": w.name, "cells": list(w.L), "spins": w.N, "boundary": "open",
                      "parallelism": "single GPU"},
           "roofline": roof,
           "stencil_only": {"ms": ms_st, "fields_per_s": w.N / ms_st * 1e3,
                            "GBps_algorithmic": FIELD_BYTES * w.N / ms_st / 1e6,
                            "hbm_frac": FIELD_BYTES * w.N / ms_st / 1e6 / HBM_PEAK_GBS},
           "stencil_plus_dipolar_fft_ms": ms_dip,
           "dipolar": dipolar_traffic(w.L, ms_dip - ms_st, zsym=bool(
               np.all(np.asarray(w.cell, np.float64).reshape(3, 3)[[0, 1, 2, 2], [2, 2, 0, 1]] == 0.0))),
           "dense_7cubed": dense, "cpu_baseline": cpu,
           "hbm_copy_GBps": copy_bandwidth(), "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)


def dipolar_traffic(L, ms, zsym=True):
    """Contract bytes of one pruned dipolar evaluation (each array read or
    written once per pass: pad, x-row R2C, y columns, fused z pass with the
    dipole spectrum, inverse y, C2R, crop) and the rate they imply.  With a
    cell whose third vector is along z (zsym) the fused pass reads the
    spectrum only for kz <= Pz / 2.  With Px = 512 the x-row passes read the
    spins and write the x spectra directly (and back), with no padded real
    rows in between."""
    Lx, Ly, Lz = L
    P = [1 << (2 * v - 1).bit_length() for v in L]
    H = P[0] // 2 + 1
    rows = 3 * Ly * Lz
    R, X = rows * P[0] * 4, rows * H * 8
    Y = 3 * Lz * P[1] * H * 8
    kz_read = P[2] // 2 + 1 if (zsym and P[2] == 512) else P[2]
    kern = 6 * kz_read * P[1] * H * 4
    N = Lx * Ly * Lz
    if P[0] == 512:
        total = (3 * N * 8 + X) + (X + Y) + (Y + kern + Y) + (Y + X) + (X + 3 * N * 4)
    else:
        total = (3 * N * 8 + R) + (R + X) + (X + Y) + (Y + kern + Y) + (Y + X) + (X + R) + (3 * N * 4 * 2)
    return {"ms": ms, "contract_bytes": total, "GBps": total / (ms / 1e3) / 1e9,
            "hbm_frac": total / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, "padded": P}


def cpu_field_baseline(w, seconds):
    """FP64 oracle field (J + DMI + Zeeman, no dipolar) on the full lattice."""
    import oracle
    from tests.helpers import oracle_model
    ws = w.scaled(w.L)
    ws.dipolar = 0
    m = oracle_model(ws)
    S = ws.initial_state()
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.field(m, S)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or el * (n + 1) / n > 2.5 * seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.N * n / el, "unit": "fields/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full-lattice short-range field evaluation(s), FP64 oracle, {el:.1f} s (dipolar excluded)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="headline",
                    help="headline (sc 1024^3 with bcc 128^3 as secondary), or one workload name")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (shared by repeated runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run 4 plain device copies of 3N doubles (a known byte "
                         "count for scaling hardware traffic counters)")
    ap.add_argument("--no-learned", action="store_true", help="GNEB workload: throughput only")
    ap.add_argument("--train-sizes", default=None,
                    help="learned init: training lattice edges and shares, e.g. 48:0.8,64:0.2 "
                         "(default: the family's own)")
    ap.add_argument("--test-sizes", default=None, help="learned init: test lattice edges, e.g. 48,64,96")
    ap.add_argument("--dilation", default=None,
                    help="learned init: per-layer dilation of the network, e.g. 1,2,4,8 (default: the family's own)")
    ap.add_argument("--test-images", type=int, default=32, help="learned init: images per test path")
    ap.add_argument("--endpoint-tol", type=float, default=2e-4,
                    help="learned init: max |F| (meV) of the relaxed end states")
    ap.add_argument("--n-train", type=int, default=200)
    ap.add_argument("--n-test", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--lr", type=float, default=2e-3, help="initial Adam step of the path net (cosine decay to lr/20)")
    ap.add_argument("--families", default="skyrmion,hopfion")
    ap.add_argument("--max-iter", type=int, default=30000)
    ap.add_argument("--damping", default="",
                    help="learned init: further factors for the network's correction, e.g. 0.6,0.3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_26016_amd import spx
    from workloads import WORKLOADS

    torch.cuda.set_device(0)
    if args.workload == "sc200_mc":
        mc_workload(args)
    elif args.workload == "sc200_min":
        min_workload(args)
    elif args.workload == "sc200_pairlist":
        pairlist_workload(args)
    elif args.workload == "sc_frustrated_gneb":
        gneb_workload(args)
    elif args.workload == "sc256_chiral_dipolar_field":
        field_workload(args, WORKLOADS[args.workload]())
    elif args.workload == "headline":
        headline(args)
    else:
        out = heun_workload(args, WORKLOADS[args.workload]())
        out["hbm_copy_GBps"] = copy_bandwidth()
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
