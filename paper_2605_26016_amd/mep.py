"""Minimum-energy-path workflow on the batched GNEB (Methods, minimum-energy
paths, and the annihilation-path pipeline of the hopfion study):

  - several trial paths are relaxed together, as the ragged instances of one
    spx_gneb object: the string method first (mode 4: force step + geodesic
    reparameterisation), then climbing-image GNEB; the channels come back
    sorted by barrier;
  - the saddle region of a path is refined locally: the band of images around
    the highest one is resampled to more images along its geodesic arc and
    relaxed by climbing-image GNEB with the band's end images pinned;
  - a long path is cut into segments that share their end images, the
    segments are refined together (one instance each, ends pinned) and
    assembled again.

Every numerical step runs in libspx (spx_gneb_* calls); this module only
places images in device buffers and sequences the calls.
"""
from dataclasses import dataclass

import numpy as np

from . import spx


@dataclass
class PathResult:
    images: "object"          # device tensor [n_img][3][N], FP64 (the relaxed path)
    energies: np.ndarray      # meV per image
    barrier: float            # max_n E_n - E_0 (meV)
    saddle: int               # index of the highest-energy image
    max_force: float          # max |F| per spin of the last iteration (meV)
    string_iterations: int
    gneb_iterations: int
    converged: bool


def _run(g, n_inst, max_iter, chunk):
    """Step until every instance has converged or max_iter iterations ran."""
    done = 0
    while done < max_iter:
        n = min(chunk, max_iter - done)
        spx.gneb_step(g, n)
        done += n
        if all(spx.gneb_get_stats(g, k)["converged"] for k in range(n_inst)):
            break


def _result(g, k, images, string_iterations):
    s = spx.gneb_get_stats(g, k)
    E = np.asarray(s["E"], dtype=np.float64)
    top = int(np.argmax(E))
    return PathResult(images=images, energies=E, barrier=float(E[top] - E[0]), saddle=top,
                      max_force=float(s["max_force"]), string_iterations=string_iterations,
                      gneb_iterations=int(s["iterations"]), converged=bool(s["converged"]))


def relax_trials(ham, trials, *, string_dt=0.05, string_tol=1e-4, string_iter=5000, spring_k=1.0,
                 vp_dt=0.1, vp_mass=1.0, ci_mode=1, ci_on_below=1e-2, ci_tol=1e-6, gneb_iter=20000,
                 chunk=200):
    """Relax trial paths (device tensors [n_img][3][N] of one lattice, end images
    pinned, updated in place) by the string method to max |F_perp| <
    string_tol, then by GNEB with a climbing image (ci_mode 1: switched on
    below ci_on_below; 2: from the start) to max |F| < ci_tol.  A tolerance of
    0 runs the full iteration count.  Returns one PathResult per trial, lowest
    barrier first."""
    n = len(trials)
    g = spx.gneb_create([ham] * n, list(trials), vp_dt=string_dt, ci_mode=4, tol_force=string_tol)
    _run(g, n, string_iter, chunk)
    s_it = [int(spx.gneb_get_stats(g, k)["iterations"]) for k in range(n)]
    spx.gneb_set_params(g, spring_k=spring_k, vp_dt=vp_dt, vp_mass=vp_mass, ci_mode=ci_mode,
                        ci_on_below=ci_on_below, tol_force=ci_tol)
    _run(g, n, gneb_iter, chunk)
    out = [_result(g, k, trials[k], s_it[k]) for k in range(n)]
    spx.gneb_destroy(g)
    return sorted(out, key=lambda r: r.barrier)


def upsample_indices(n_old, n_new):
    """Indices of the old images that fill n_new slots in order, each old image
    at least once (n_new >= n_old): the duplicated path has the same geodesic
    arc, and an equal-spacing redistribution of it is the arc resampled."""
    if n_new < n_old:
        raise ValueError("upsampling needs n_new >= n_old")
    return np.rint(np.linspace(0.0, n_old - 1, n_new)).astype(np.int64)


def resample(images, n_new):
    """A new device path of n_new images spread evenly along the geodesic arc
    of `images` (end images kept): the duplicated path, redistributed."""
    import torch
    idx = torch.as_tensor(upsample_indices(images.shape[0], n_new), device=images.device)
    return images.index_select(0, idx).contiguous()


def refine_saddle(ham, path, saddle=None, *, half_width=1, n_local=9, spring_k=1.0, vp_dt=0.1, vp_mass=1.0,
                  tol=5e-6, max_iter=50000, chunk=500):
    """Local climbing-image refinement of the saddle region: images saddle -
    half_width .. saddle + half_width of `path` (default saddle: the image
    with the highest energy) are resampled to n_local images along their
    geodesic arc, and the band is relaxed by climbing-image GNEB (climbing
    image from the start) with its end images pinned, to max |F| < tol."""
    M = path.shape[0]
    if saddle is None:
        g0 = spx.gneb_create([ham], [path.clone()], ci_mode=0)
        spx.gneb_step(g0, 1)
        saddle = int(np.argmax(spx.gneb_get_stats(g0)["E"]))
        spx.gneb_destroy(g0)
    lo, hi = max(0, saddle - half_width), min(M - 1, saddle + half_width)
    band = resample(path[lo:hi + 1], max(n_local, hi - lo + 1))
    g = spx.gneb_create([ham], [band], spring_k=spring_k, vp_dt=vp_dt, vp_mass=vp_mass, ci_mode=2, tol_force=tol)
    spx.gneb_redistribute(g)
    _run(g, 1, max_iter, chunk)
    r = _result(g, 0, band, 0)
    spx.gneb_destroy(g)
    return r


def split(path, cuts):
    """Segments of `path` between the image indices in cuts (first 0, last
    n_img - 1); neighbouring segments share their end image."""
    cuts = list(cuts)
    if cuts[0] != 0 or cuts[-1] != path.shape[0] - 1 or any(b - a < 2 for a, b in zip(cuts, cuts[1:])):
        raise ValueError("cuts must run from 0 to n_img - 1 with at least one movable image per segment")
    return [path[a:b + 1].clone() for a, b in zip(cuts, cuts[1:])]


def assemble(segments):
    """One path from segments that share their end images (each shared image
    appears once)."""
    import torch
    for a, b in zip(segments, segments[1:]):
        if not torch.equal(a[-1], b[0]):
            raise ValueError("segments must share their end images")
    return torch.cat([segments[0]] + [s[1:] for s in segments[1:]], dim=0)


def refine_segments(ham, path, cuts, *, spring_k=1.0, vp_dt=0.1, vp_mass=1.0, ci_mode=1, ci_on_below=1e-2,
                    tol=1e-6, max_iter=20000, chunk=200):
    """Cut `path` at the image indices `cuts`, refine every segment by GNEB
    (one instance each, all in one batched object, end images pinned) and
    assemble the refined path.  Returns (path, [PathResult per segment])."""
    segs = split(path, cuts)
    g = spx.gneb_create([ham] * len(segs), segs, spring_k=spring_k, vp_dt=vp_dt, vp_mass=vp_mass, ci_mode=ci_mode,
                        ci_on_below=ci_on_below, tol_force=tol)
    _run(g, len(segs), max_iter, chunk)
    res = [_result(g, k, segs[k], 0) for k in range(len(segs))]
    spx.gneb_destroy(g)
    return assemble(segs), res
