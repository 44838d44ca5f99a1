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
             vp_mass=1.0, method=0, net=None, params=None) -> PathResult:
    """Batched GNEB over all instances from the geodesic (method 0) or learned
    (method 1) initial path until every instance has converged or max_iter."""
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


def train(data: PathData, epochs=30, batch=16, lr=1e-3, seed=0, params=None, log=None, lr_final=None):
    """Adam on the mean over images and sites of |S_hat - S*|^2; the step
    size decays from lr to lr_final (default lr) on a cosine over the run."""
    import torch
    net = spx.Net()
    p = torch.from_numpy(init_params(seed) if params is None else params).cuda()
    n = p.numel()
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    ns = data.Sg.shape[0]
    step = 0
    hist = []
    lr_end = lr if lr_final is None else lr_final
    n_steps = epochs * ((ns + batch - 1) // batch)
    for ep in range(epochs):
        order = rng.permutation(ns)
        tot = 0.0
        nb = 0
        for b0 in range(0, ns, batch):
            idx = torch.from_numpy(order[b0:b0 + batch]).cuda()
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
        if log:
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


def learned_vs_geodesic(family, n_train=200, n_test=12, epochs=150, lr=2e-3, max_iter=30000, hopfion_L=32,
                        skyrmion_train_L=32, skyrmion_test_L=(48, 64, 96), log=None):
    """Train the path corrector on GNEB-converged paths of one family and
    compare GNEB from the learned and the geodesic initial path on held-out
    end states.  hopfion: four-shell frustrated sc exchange (J1 = 1 meV,
    J2/J1 = 0.188, J3/J1 = -0.274, J4/J1 = -0.161), open L^3, VP-relaxed
    seeded hopfion -> FM (16 images).  skyrmion: sc monolayer film, J = 1 meV,
    bulk DMI 0.3 meV, B = 1.4 T, periodic in plane, relaxed seeded skyrmion ->
    FM, trained on skyrmion_train_L^2 films (16 images) and evaluated on a
    ragged batch of skyrmion_test_L^2 films (32 images).  Both GNEB runs use
    the same optimiser settings; a pair counts when both converge to max |F| <
    1e-3 meV with barriers within 0.1 meV (same channel).  End states are
    drawn by the seeded texture generators (training seeds 1000.., test seeds
    5000..)."""
    import time

    import torch

    from workloads import hopfion_texture, skyrmion_texture, uniform_state

    log = log or (lambda *a: None)

    t0 = time.perf_counter()
    if family == "hopfion":
        J = dict(J_shell=(1.0, 0.188, -0.274, -0.161))
        Ltr = (hopfion_L,) * 3
        Lte = [Ltr]
        per = (0, 0, 0)
        n_tr_img, n_te_img = 16, 16

        def seed_state(L, s):
            rng = np.random.default_rng(s)
            m = min(L) / 6
            return hopfion_texture(L, R0=m * (1 + 0.2 * rng.uniform(-1, 1)), width=m * (1 + 0.2 * rng.uniform(-1, 1)),
                                   center_offset=rng.uniform(-2, 2, 3))
    else:
        J = dict(J_shell=(1.0,), D_shell=(0.3,), B=(0.0, 0.0, 1.4))
        Ltr = (skyrmion_train_L, skyrmion_train_L, 1)
        Lte = [(L, L, 1) for L in skyrmion_test_L]
        per = (1, 1, 0)
        n_tr_img, n_te_img = 16, 32
        n_test = len(Lte) * max(1, n_test // len(Lte))

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
        rel, _, _ = minimize(h, st, tol=2e-4, max_iter=30000, vp_dt=0.2)
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
    res_tr = converge([ham(Ltr)] * len(Y_tr), Y_tr, tol=1e-3, max_iter=max_iter, chunk=1000)
    ok = [k for k in range(len(Y_tr)) if res_tr.converged[k]]
    log(f"[path-init] {family}: {len(ok)}/{len(Y_tr)} training paths converged (median "
        f"{int(np.median(res_tr.iterations))} iterations), {time.perf_counter() - t0:.1f} s")
    data = build_samples(Ltr, [geo[k] for k in ok], [Y_tr[k] for k in ok])
    p, net, hist = train(data, epochs=epochs, batch=16, lr=lr, lr_final=lr / 20)
    log(f"[path-init] {family}: trained, loss {hist[0]:.3e} -> {hist[-1]:.3e}, {time.perf_counter() - t0:.1f} s")
    Hs, Yp = [], []
    per_size = max(1, n_test // len(Lte))
    for i, L in enumerate(Lte):
        A = endpoints(L, range(5000 + 100 * i, 5000 + 100 * i + per_size))
        Yp += paths(L, A, n_te_img)
        Hs += [ham(L)] * len(A)
    Yl = [y.clone() for y in Yp]
    rp = converge(Hs, Yp, tol=1e-3, max_iter=max_iter, chunk=250)
    rl = converge(Hs, Yl, tol=1e-3, max_iter=max_iter, chunk=250, method=1, net=net, params=p)
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
