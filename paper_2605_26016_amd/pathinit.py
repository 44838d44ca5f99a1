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


def train(data: PathData, epochs=30, batch=16, lr=1e-3, seed=0, params=None, log=None):
    """Adam on the mean over images and sites of |S_hat - S*|^2."""
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
            step += 1
            spx.net_adam_step(p, grad, m, v, step, lr=lr)
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
