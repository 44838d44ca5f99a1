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
KERNEL_SOURCES = ["paper_2605_26016_amd/csrc/spx_kernels.hip", "paper_2605_26016_amd/csrc/spx_device.hpp",
                  "paper_2605_26016_amd/csrc/spx_stencil.hip", "paper_2605_26016_amd/csrc/spx_stencil.hpp",
                  "paper_2605_26016_amd/csrc/spx_internal.hpp"]
# corrector kernel name per stencil engine (1 gather, 2 z-march)
CORRECT_KERNEL = {1: "k_heun_correct", 2: "k_zmarch (corrector instantiation)"}


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


# GNEB algorithmic HBM bytes per spin-image-iteration of the three passes
# (FP64, 24 B per spin vector): pass A reads S_n, S_n+1 and writes F (72 B);
# pass B reads S_n-1, S_n, S_n+1, F, v (120 B); pass C reads S_n-1, S_n, S_n+1,
# F and writes v, S' (144 B).  Neighbour reuse inside an image is on chip.
GNEB_BYTES = 336


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
                             "unit": "GB/s", "frac": rate * GNEB_BYTES / 1e9 / HBM_PEAK_GBS, "traffic": None,
                             "kernel": "GNEB iteration (passes A, B, C + reductions)",
                             "bytes_per_spin_image_iteration": GNEB_BYTES}})
    out["config"] = {"workload": "sc_frustrated_gneb", "lattices": [list((L, L, L)) for L in sizes], "images": 32,
                     "spin_images": spin_images, "shells_throughput": [1.0, -0.164, -0.082],
                     "parallelism": "single GPU, ragged batch in one launch per pass"}
    del g, hams, imgs
    log(f"[bench] batched GNEB: {rate:.3e} spin-image-iterations/s")
    if args.no_learned:
        print(json.dumps(out), flush=True)
        return
    out["learned_init"] = {fam: learned_experiment(fam, args) for fam in args.families.split(",")}
    print(json.dumps(out), flush=True)


def learned_experiment(family, args):
    """Train the path corrector on GNEB-converged paths of one family and
    compare GNEB from the learned and the geodesic initial path on held-out
    end states.  hopfion: four-shell frustrated sc exchange (J1 = 1 meV,
    J2/J1 = 0.188, J3/J1 = -0.274, J4/J1 = -0.161), open L^3, VP-relaxed
    seeded hopfion -> FM.  skyrmion: sc monolayer film, J = 1 meV, bulk DMI
    0.3 meV, B = 1.4 T, periodic in plane, relaxed seeded skyrmion -> FM,
    trained on 32^2 and evaluated on a ragged batch of 48^2, 64^2, 96^2 films
    with 32 images."""
    import numpy as np
    import torch

    from paper_2605_26016_amd import pathinit, spx
    from workloads import hopfion_texture, skyrmion_texture, uniform_state

    t0 = time.perf_counter()
    if family == "hopfion":
        J = dict(J_shell=(1.0, 0.188, -0.274, -0.161))
        Ltr = (args.gneb_L,) * 3
        Lte = [Ltr]
        per = (0, 0, 0)
        n_tr_img, n_te_img = 16, 16
        n_train, n_test = args.n_train, args.n_test

        def seed_state(L, s):
            rng = np.random.default_rng(s)
            m = min(L) / 6
            return hopfion_texture(L, R0=m * (1 + 0.2 * rng.uniform(-1, 1)), width=m * (1 + 0.2 * rng.uniform(-1, 1)),
                                   center_offset=rng.uniform(-2, 2, 3))
    else:
        J = dict(J_shell=(1.0,), D_shell=(0.3,), B=(0.0, 0.0, 1.4))
        Ltr = (32, 32, 1)
        Lte = [(48, 48, 1), (64, 64, 1), (96, 96, 1)]
        per = (1, 1, 0)
        n_tr_img, n_te_img = 16, 32
        n_train, n_test = args.n_train, 3 * max(1, args.n_test // 3)

        def seed_state(L, s):
            rng = np.random.default_rng(s)
            return skyrmion_texture(L, R=3.0 * (1 + 0.3 * rng.uniform(-1, 1)), center=tuple(rng.uniform(-3, 3, 2)))

    hams = {}

    def ham(L):
        if L not in hams:
            hams[L] = spx.setup_hamiltonian(L, periodic=per, field_prec="fp64", **J)
        return hams[L]

    def endpoints(L, seeds):
        h = ham(L)
        st = [torch.from_numpy(seed_state(L, s)).cuda() for s in seeds]
        rel, _, _ = pathinit.minimize(h, st, tol=2e-4, max_iter=30000, vp_dt=0.2)
        return [r for r in rel if int((r[2] < 0).sum()) > 0]   # textures that survived relaxation

    def paths(L, A, n_img):
        N = L[0] * L[1] * L[2]
        fm = torch.from_numpy(uniform_state(N)).cuda()
        Ys = []
        for a in A:
            Y = torch.zeros((n_img, 3, N), dtype=torch.float64, device="cuda")
            Y[0] = a
            Y[-1] = fm
            Ys.append(Y)
        return Ys

    A_tr = endpoints(Ltr, range(1000, 1000 + n_train))
    Y_tr = paths(Ltr, A_tr, n_tr_img)
    geo = [y.clone() for y in Y_tr]
    gg = spx.gneb_create([ham(Ltr)] * len(geo), geo)
    spx.gneb_init_path(gg)
    res_tr = pathinit.converge([ham(Ltr)] * len(Y_tr), Y_tr, tol=1e-3, max_iter=args.max_iter, chunk=1000)
    ok = [k for k in range(len(Y_tr)) if res_tr.converged[k]]
    log(f"[bench] {family}: {len(ok)}/{len(Y_tr)} training paths converged (median "
        f"{int(np.median(res_tr.iterations))} iterations), {time.perf_counter() - t0:.1f} s")
    data = pathinit.build_samples(Ltr, [geo[k] for k in ok], [Y_tr[k] for k in ok])
    p, net, hist = pathinit.train(data, epochs=args.epochs, batch=16, lr=1e-3)
    log(f"[bench] {family}: trained, loss {hist[0]:.3e} -> {hist[-1]:.3e}, {time.perf_counter() - t0:.1f} s")
    Hs, Yp = [], []
    per_size = max(1, n_test // len(Lte))
    for i, L in enumerate(Lte):
        A = endpoints(L, range(5000 + 100 * i, 5000 + 100 * i + per_size))
        Yp += paths(L, A, n_te_img)
        Hs += [ham(L)] * len(A)
    Yl = [y.clone() for y in Yp]
    rp = pathinit.converge(Hs, Yp, tol=1e-3, max_iter=args.max_iter, chunk=250)
    rl = pathinit.converge(Hs, Yl, tol=1e-3, max_iter=args.max_iter, chunk=250, method=1, net=net, params=p)
    both = [k for k in range(len(Yp)) if rp.converged[k] and rl.converged[k]]
    dbar = np.abs(rl.barrier - rp.barrier)
    same = [k for k in both if dbar[k] <= 0.1]
    it_p = float(np.mean(rp.iterations[same])) if same else None
    it_l = float(np.mean(rl.iterations[same])) if same else None
    return {"lattice_train": list(Ltr), "lattices_test": [list(L) for L in Lte], "images_train": n_tr_img,
            "images_test": n_te_img, "train_paths": len(ok), "test_paths": len(Yp),
            "test_converged_both": len(both), "same_channel_within_0.1meV": len(same),
            "iterations_geodesic": rp.iterations.tolist(), "iterations_learned": rl.iterations.tolist(),
            "barrier_geodesic_meV": np.round(rp.barrier, 4).tolist(),
            "barrier_learned_meV": np.round(rl.barrier, 4).tolist(),
            "mean_iterations_geodesic_same_channel": it_p, "mean_iterations_learned_same_channel": it_l,
            "iteration_ratio_learned_over_geodesic": (it_l / it_p) if same else None,
            "max_barrier_difference_same_channel_meV": float(np.max(dbar[same])) if same else None,
            "train_loss_first_last": [hist[0], hist[-1]], "seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bcc128_5shell_stochastic_mixed")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (shared by repeated runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run 4 plain device copies of 3N doubles (a known byte "
                         "count for scaling hardware traffic counters)")
    ap.add_argument("--no-learned", action="store_true", help="GNEB workload: throughput only")
    ap.add_argument("--gneb-L", type=int, default=32)
    ap.add_argument("--n-train", type=int, default=200)
    ap.add_argument("--n-test", type=int, default=12)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--families", default="skyrmion,hopfion")
    ap.add_argument("--max-iter", type=int, default=30000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_26016_amd import spx
    from workloads import WORKLOADS

    if args.workload == "sc_frustrated_gneb":
        torch.cuda.set_device(0)
        gneb_workload(args)
        return
    w = WORKLOADS[args.workload]()
    log(f"[bench] workload {w.name}: {w.N} spins, {args.warmup} warmup + {args.steps} timed Heun steps")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    h = spx.setup_hamiltonian(w.L, cell=w.cell, sub_frac=w.frac, mu=w.mu, periodic=w.periodic,
                              J_shell=w.J_shell, D_shell=w.D_shell, K=(w.K if w.K else None),
                              K_axis=w.K_axis, B=w.B, dipolar=w.dipolar, field_prec=w.field_prec,
                              autotune=0 if args.no_autotune else 1, tune_cache_path=args.tune_cache)
    info = spx.get_info(h)
    log(f"[bench] engine {info.stencil_engine} shape {info.shape} zchunk {info.zchunk} "
        f"heun_field {info.heun_field} tuned {info.tuned} ({info.tuned_step_us:.1f} us/step while tuning)")
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
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": CORRECT_KERNEL.get(info.stencil_engine, "k_heun_correct"),
            "bytes_per_launch_algorithmic": BYTES_PER_SPIN[dom] * w.N}
    step_bytes = sum(BYTES_PER_SPIN.values())
    if args.calibrate_copy:
        src = torch.empty_like(S).copy_(S)
        dst = torch.empty_like(S)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 4 copies of {src.numel() * 8} bytes")
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
                   "parallelism": "single GPU", "stencil_engine": info.stencil_engine,
                   "zchunk": info.zchunk, "heun_field": info.heun_field},
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
