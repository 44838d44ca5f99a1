"""Training and evaluation driver of the learned initial-path corrector.

Orchestration only: every step runs in libspx.so kernels (damped-LLG endpoint
relaxation, batched GNEB, network forward/backward/Adam).  The data are
minimum-energy paths the method itself produces: for each pair of end states
the batched GNEB is converged from the geodesic path, and each movable image
of the converged path becomes a training target for its geodesic guess at the
same reaction coordinate t = n / (n_img - 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import spx


def relax(h, S, n_steps, dt_fs=4.0, alpha=1.0, chunk=1000):
    """Damped zero-temperature LLG (Heun) relaxation of S in place."""
    done = 0
    while done < n_steps:
        k = min(chunk, n_steps - done)
        spx.llg_heun_step(h, S, alpha=alpha, dt_fs=dt_fs, temperature_K=0.0, n_steps=k, step0=done)
        done += k


@dataclass
class PathResult:
    iterations: np.ndarray       # per instance
    converged: np.ndarray
    barrier: np.ndarray          # E_CI - E_0 (meV), or max(E) - E_0 without a climbing image
    max_force: np.ndarray
    seconds: float
    spin_image_iters: float      # sum over instances of N * n_img * iterations


def converge(hams, images, tol=1e-3, ci_on_below=1e-2, max_iter=20000, chunk=500, spring_k=1.0, vp_dt=0.1,
             vp_mass=1.0, method=0, net=None, params=None, log=None, what="") -> PathResult:
    """Batched GNEB over all instances from the geodesic (method 0) or learned
    (method 1) initial path until every instance has converged or max_iter.
    log: called with a progress line every 5000 iterations."""
    import time
    import torch
    g = spx.gneb_create(hams, images, spring_k=spring_k, vp_dt=vp_dt, vp_mass=vp_mass, ci_mode=1,
                        ci_on_below=ci_on_below, tol_force=tol)
    spx.gneb_init_path(g, method=method, net=net, params=params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    n = len(hams)
    while done < max_iter:
        spx.gneb_step(g, min(chunk, max_iter - done))
        done += min(chunk, max_iter - done)
        conv = [spx.gneb_get_stats(g, k)["converged"] for k in range(n)]
        if all(conv):
            break
        if log and done % 5000 < chunk:
            log(f"[path-init] {what}: {done} iterations, {sum(conv)}/{n} converged, "
                f"{time.perf_counter() - t0:.0f} s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = [spx.gneb_get_stats(g, k) for k in range(n)]
    its = np.array([s["iterations"] for s in st])
    bar = []
    for s in st:
        ci = s["ci_index"]
        e = s["E"]
        bar.append((e[ci] if ci >= 0 else e.max()) - e[0])
    work = float(sum(int(images[k].shape[0]) * int(images[k].shape[2]) * int(its[k]) for k in range(n)))
    return PathResult(its, np.array([s["converged"] for s in st]), np.array(bar),
                      np.array([s["max_force"] for s in st]), el, work)


def init_params(seed=0):
    """He-scaled FP32 parameters for the 10-16-16-16-3 network, last layer
    scaled by 0.1 so the untrained network starts close to the identity map."""
    ch = (10, 16, 16, 16, 3)
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(4):
        fan = ch[l] * 27
        s = math.sqrt(2.0 / fan) * (0.1 if l == 3 else 1.0)
        parts.append(rng.standard_normal(ch[l + 1] * ch[l] * 27) * s)
        parts.append(np.zeros(ch[l + 1]))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == spx.net_nparams()
    return p


@dataclass
class PathData:
    """Training samples on one lattice size: geodesic guess, end images,
    reaction coordinate and converged image, all on the device."""
    dims: tuple
    Sg: "torch.Tensor"
    SA: "torch.Tensor"
    SB: "torch.Tensor"
    t: "torch.Tensor"
    Sstar: "torch.Tensor"


def build_samples(dims, geodesic_paths, converged_paths) -> PathData:
    """geodesic_paths / converged_paths: lists of device tensors [n_img][3][P]."""
    import torch
    Sg, SA, SB, t, Ss = [], [], [], [], []
    for geo, conv in zip(geodesic_paths, converged_paths):
        n_img = geo.shape[0]
        for n in range(1, n_img - 1):
            Sg.append(geo[n])
            SA.append(conv[0])
            SB.append(conv[-1])
            Ss.append(conv[n])
            t.append(n / (n_img - 1))
    return PathData(tuple(dims), torch.stack(Sg).contiguous(), torch.stack(SA).contiguous(),
                    torch.stack(SB).contiguous(), torch.tensor(t, dtype=torch.float32, device="cuda"),
                    torch.stack(Ss).contiguous())


def train(data, epochs=30, batch=16, lr=1e-3, seed=0, params=None, log=None, lr_final=None, dilation=(1, 1, 1, 1),
          log_every=1):
    """Adam on the mean over images and sites of |S_hat - S*|^2; the step
    size decays from lr to lr_final (default lr) on a cosine over the run.
    data: one PathData or a list of them (lattice sizes); every batch comes
    from one of them, and an epoch visits every sample once in shuffled
    batch order."""
    import torch
    sets = data if isinstance(data, (list, tuple)) else [data]
    net = spx.Net(dilation=dilation)
    p = torch.from_numpy(init_params(seed) if params is None else params).cuda()
    n = p.numel()
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    lr_end = lr if lr_final is None else lr_final
    n_steps = epochs * sum((d.Sg.shape[0] + batch - 1) // batch for d in sets)
    for ep in range(epochs):
        plan = []
        for k, d in enumerate(sets):
            order = rng.permutation(d.Sg.shape[0])
            plan += [(k, order[b0:b0 + batch]) for b0 in range(0, len(order), batch)]
        rng.shuffle(plan)
        tot = 0.0
        nb = 0
        for k, sel in plan:
            data = sets[k]
            idx = torch.from_numpy(sel).cuda()
            B = int(idx.numel())
            Sg = data.Sg.index_select(0, idx).contiguous()
            SA = data.SA.index_select(0, idx).contiguous()
            SB = data.SB.index_select(0, idx).contiguous()
            Ss = data.Sstar.index_select(0, idx).contiguous()
            tt = data.t.index_select(0, idx).contiguous()
            spx.net_backward(net, p, data.dims, B, Sg, SA, SB, tt, Ss, grad, loss)
            lr_k = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * step / max(n_steps, 1)))
            step += 1
            spx.net_adam_step(p, grad, m, v, step, lr=lr_k)
            tot += loss.item()
            nb += 1
        hist.append(tot / max(nb, 1))
        if log and (ep % log_every == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return p, net, hist


def minimize(h, states, tol=1e-4, max_iter=20000, chunk=1000, vp_dt=0.1, vp_mass=1.0):
    """Relax each state ([3][N] device tensors, same Hamiltonian) to a local
    minimum by velocity projection with the exponential-map retraction (the
    batched GNEB object in minimisation mode, all states in one launch).
    Returns (relaxed states, iterations, max force)."""
    import torch
    M = len(states)
    Y = torch.stack([states[0]] + list(states) + [states[0]]).contiguous()
    g = spx.gneb_create([h], [Y], spring_k=0.0, vp_dt=vp_dt, vp_mass=vp_mass, ci_mode=3, tol_force=tol)
    done = 0
    while done < max_iter:
        k = min(chunk, max_iter - done)
        spx.gneb_step(g, k)
        done += k
        if spx.gneb_get_stats(g)["converged"]:
            break
    s = spx.gneb_get_stats(g)
    return [Y[1 + m].clone() for m in range(M)], s["iterations"], s["max_force"]


def learned_vs_geodesic(family, n_train=200, n_test=12, epochs=150, lr=2e-3, max_iter=30000, train_sizes=None,
                        test_sizes=None, n_img_train=16, n_img_test=32, dilation=None, endpoint_tol=2e-4,
                        damping=(), log=None):
    """Train the path corrector on GNEB-converged paths of one family and
    compare GNEB from the learned and the geodesic initial path on held-out
    end states.

    hopfion: four-shell frustrated sc exchange (J1 = 1 meV, J2/J1 = 0.188,
    J3/J1 = -0.274, J4/J1 = -0.161), open L^3, VP-relaxed seeded hopfion ->
    FM; train_sizes default ((48, 0.8), (64, 0.2)): lattice edge and share of
    the n_train training pairs; test on 48^3, 64^3 and 96^3.
    skyrmion: sc monolayer film, J = 1 meV, bulk DMI 0.3 meV, B = 1.4 T,
    periodic in plane, relaxed seeded skyrmion -> FM; trained on 32^2 films,
    tested on 48^2, 64^2 and 96^2 films.

    End states are relaxed by velocity projection to max |F| < endpoint_tol
    (meV).  n_img_train images per training path, n_img_test per test path; the
    test pairs are dealt evenly over test_sizes and run as one ragged batch.
    dilation: per-layer dilation of the network (default (1, 2, 4, 8) for
    hopfions, whose torus radius L/6 exceeds the 9-cell field of undilated
    layers, and (1, 1, 1, 1) for skyrmion films).  Both GNEB runs use the same
    optimiser settings; a pair counts when both converge to max |F| < 1e-3
    meV with barriers within 0.1 meV (same channel).  End states are drawn by
    the seeded texture generators (training seeds 1000.., test seeds 5000..).
    damping: further factors lambda for the correction (the last layer's
    weights and bias scaled by lambda, so the tangent update u is scaled
    exactly); GNEB runs again from each damped learned path and the same
    statistics are reported per lambda."""
    import time

    import torch

    from workloads import hopfion_texture, skyrmion_texture, uniform_state

    log = log or (lambda *a: None)

    t0 = time.perf_counter()
    if family == "hopfion":
        J = dict(J_shell=(1.0, 0.188, -0.274, -0.161))
        per = (0, 0, 0)
        train_sizes = train_sizes or ((48, 0.8), (64, 0.2))
        test_sizes = test_sizes or (48, 64, 96)
        dilation = dilation or (1, 2, 4, 8)

        def lat(L):
            return (L, L, L)

        def seed_state(L, s):
            rng = np.random.default_rng(s)
            m = min(L) / 6
            return hopfion_texture(L, R0=m * (1 + 0.2 * rng.uniform(-1, 1)), width=m * (1 + 0.2 * rng.uniform(-1, 1)),
                                   center_offset=rng.uniform(-2, 2, 3))
    else:
        J = dict(J_shell=(1.0,), D_shell=(0.3,), B=(0.0, 0.0, 1.4))
        per = (1, 1, 0)
        train_sizes = train_sizes or ((32, 1.0),)
        test_sizes = test_sizes or (48, 64, 96)
        dilation = dilation or (1, 1, 1, 1)

        def lat(L):
            return (L, L, 1)

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
        rel, _, _ = minimize(h, st, tol=endpoint_tol, max_iter=60000, vp_dt=0.2)
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

    # -- training data: converged paths per lattice size
    sets, n_ok, its_tr, bar_tr = [], 0, [], []
    for i, (edge, share) in enumerate(train_sizes):
        L = lat(edge)
        n_L = max(1, int(round(n_train * share)))
        A_tr = endpoints(L, range(1000 + 2000 * i, 1000 + 2000 * i + n_L))
        Y_tr = paths(L, A_tr, n_img_train)
        geo = [y.clone() for y in Y_tr]
        gg = spx.gneb_create([ham(L)] * len(geo), geo)
        spx.gneb_init_path(gg)
        del gg
        res_tr = converge([ham(L)] * len(Y_tr), Y_tr, tol=1e-3, max_iter=max_iter, chunk=1000, log=log,
                          what=f"{family} training {edge}")
        ok = [k for k in range(len(Y_tr)) if res_tr.converged[k]]
        n_ok += len(ok)
        its_tr += res_tr.iterations.tolist()
        bar_tr += np.round(res_tr.barrier, 4).tolist()
        log(f"[path-init] {family} {L}: {len(ok)}/{len(Y_tr)} training paths converged (median "
            f"{int(np.median(res_tr.iterations))} iterations, barriers {np.min(res_tr.barrier):.3f} .. "
            f"{np.max(res_tr.barrier):.3f} meV), {time.perf_counter() - t0:.1f} s")
        if ok:
            sets.append(build_samples(L, [geo[k] for k in ok], [Y_tr[k] for k in ok]))
        del Y_tr, geo
    p, net, hist = train(sets, epochs=epochs, batch=16, lr=lr, lr_final=lr / 20, dilation=dilation,
                         log=lambda m: log(f"[path-init] {family} {m}"), log_every=10)
    log(f"[path-init] {family}: trained, loss {hist[0]:.3e} -> {hist[-1]:.3e}, {time.perf_counter() - t0:.1f} s")
    del sets
    # -- held-out pairs on every test size, one ragged batch per initial path
    Hs, Yp, size_of = [], [], []
    per_size = max(1, n_test // len(test_sizes))
    for i, edge in enumerate(test_sizes):
        L = lat(edge)
        A = endpoints(L, range(5000 + 100 * i, 5000 + 100 * i + per_size))
        Yp += paths(L, A, n_img_test)
        Hs += [ham(L)] * len(A)
        size_of += [edge] * len(A)
    Yl = [y.clone() for y in Yp]
    rp = converge(Hs, Yp, tol=1e-3, max_iter=max_iter, chunk=250, log=log, what=f"{family} test geodesic")
    rl = converge(Hs, Yl, tol=1e-3, max_iter=max_iter, chunk=250, method=1, net=net, params=p, log=log,
                  what=f"{family} test learned")
    # the same learned initial paths with the network in BF16 on the matrix
    # cores: the initial path's cost and distance from the FP32 one, and GNEB
    # from it (the endpoints of the relaxed buffers are the original ones)
    import torch
    Yf = [y.clone() for y in Yl]
    Yb = [y.clone() for y in Yl]
    gf = spx.gneb_create(Hs, Yf)
    gb = spx.gneb_create(Hs, Yb)
    init_ms = {}
    for prec, g in (("fp32", gf), ("bf16", gb)):
        spx.net_set_precision(net, prec)
        spx.gneb_init_path(g, method=1, net=net, params=p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            spx.gneb_init_path(g, method=1, net=net, params=p)
        e1.record()
        torch.cuda.synchronize()
        init_ms[prec] = e0.elapsed_time(e1) / 10
    d_bf16 = max(float((a - b).abs().max()) for a, b in zip(Yf, Yb))
    del gf, gb, Yf
    rb = converge(Hs, Yb, tol=1e-3, max_iter=max_iter, chunk=250, method=1, net=net, params=p, log=log,
                  what=f"{family} test learned bf16")
    spx.net_set_precision(net, "fp32")
    log(f"[path-init] {family}: initial paths of the test batch {init_ms['fp32']:.2f} ms FP32, "
        f"{init_ms['bf16']:.2f} ms BF16 MFMA, max |dS| {d_bf16:.2e}")
    # damped corrections: the last layer (3 x 16 x 27 weights and 3 biases,
    # the end of the parameter vector) scaled by lambda
    n_last = 3 * 16 * 27 + 3
    damped = {}
    for lam in damping:
        pl = p.clone()
        pl[-n_last:] *= float(lam)
        Yd = [y.clone() for y in Yl]
        rd = converge(Hs, Yd, tol=1e-3, max_iter=max_iter, chunk=250, method=1, net=net, params=pl, log=log,
                      what=f"{family} test learned x{lam}")
        sd = [k for k in range(len(Yp)) if rp.converged[k] and rd.converged[k]
              and abs(rd.barrier[k] - rp.barrier[k]) <= 0.1]
        ip = float(np.mean(rp.iterations[sd])) if sd else None
        idd = float(np.mean(rd.iterations[sd])) if sd else None
        damped[str(lam)] = {"same_channel_within_0.1meV": len(sd), "converged": int(np.sum(rd.converged)),
                            "mean_iterations_geodesic_same_channel": ip,
                            "mean_iterations_learned_same_channel": idd,
                            "iteration_ratio_learned_over_geodesic": (idd / ip) if sd else None,
                            "iterations_learned": rd.iterations.tolist(),
                            "barrier_learned_meV": np.round(rd.barrier, 4).tolist()}
        log(f"[path-init] {family}: correction x{lam}: {len(sd)}/{len(Yp)} test pairs in the same channel; "
            f"iterations learned {idd} vs geodesic {ip}")
        del Yd
    both = [k for k in range(len(Yp)) if rp.converged[k] and rl.converged[k]]
    dbar = np.abs(rl.barrier - rp.barrier)
    same = [k for k in both if dbar[k] <= 0.1]
    it_p = float(np.mean(rp.iterations[same])) if same else None
    it_l = float(np.mean(rl.iterations[same])) if same else None
    same_b = [k for k in range(len(Yp)) if rp.converged[k] and rb.converged[k] and abs(rb.barrier[k] - rp.barrier[k]) <= 0.1]
    it_pb = float(np.mean(rp.iterations[same_b])) if same_b else None
    it_b = float(np.mean(rb.iterations[same_b])) if same_b else None
    log(f"[path-init] {family}: {len(same)}/{len(Yp)} test pairs in the same channel; iterations learned "
        f"{it_l} vs geodesic {it_p}")
    return {"lattices_train": [list(lat(e)) for e, _ in train_sizes], "train_share": [sh for _, sh in train_sizes],
            "lattices_test": [list(lat(e)) for e in test_sizes], "test_lattice_edge": size_of,
            "images_train": n_img_train, "images_test": n_img_test, "dilation": list(dilation),
            "train_paths": n_ok, "train_iterations": its_tr, "train_barriers_meV": bar_tr, "test_paths": len(Yp),
            "test_converged_both": len(both), "same_channel_within_0.1meV": len(same),
            "iterations_geodesic": rp.iterations.tolist(), "iterations_learned": rl.iterations.tolist(),
            "barrier_geodesic_meV": np.round(rp.barrier, 4).tolist(),
            "barrier_learned_meV": np.round(rl.barrier, 4).tolist(),
            "mean_iterations_geodesic_same_channel": it_p, "mean_iterations_learned_same_channel": it_l,
            "iteration_ratio_learned_over_geodesic": (it_l / it_p) if same else None,
            "max_barrier_difference_same_channel_meV": float(np.max(dbar[same])) if same else None,
            "damped": damped,
            "init_ms_test_batch": {"fp32": init_ms["fp32"], "bf16_mfma": init_ms["bf16"]},
            "init_bf16_vs_fp32_max_dS": d_bf16, "iterations_learned_bf16": rb.iterations.tolist(),
            "same_channel_bf16_within_0.1meV": len(same_b),
            "mean_iterations_geodesic_same_channel_bf16": it_pb,
            "mean_iterations_learned_bf16_same_channel": it_b,
            "train_loss_first_last": [hist[0], hist[-1]], "seconds": time.perf_counter() - t0}
