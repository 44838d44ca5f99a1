"""FP64 NumPy/SciPy reference for the open-boundary dipolar field via FFT.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is the textbook
zero-padded linear convolution (Methods, reciprocal-space convolution for long
range dipolar fields): the dipole tensor
    T_ab(r) = (mu0/4pi) mu_B^2 (3 rhat_a rhat_b - delta_ab) / |r|^3,  T(0) = 0,
is sampled on a grid of 2L per axis holding every displacement in
[-(L-1), L-1], the spins are zero-padded to the same grid, and the product of
spectra is transformed back and cropped.  It uses pocketfft (scipy.fft) in
float64 and is itself checked against the direct O(N^2) sum of the C oracle.
Single-sublattice lattices only.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import constants


def _workers():
    """Threads for the transforms (pocketfft splits independent 1-D
    transforms between threads; every transform's arithmetic is unchanged)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def dipole_kernel(L, cell):
    """Real-space dipole tensor on the (2Lz, 2Ly, 2Lx) grid; returns dict of
    the six components xx, xy, xz, yy, yz, zz (meV / mu_B^2 units of mu_i mu_j).
    Evaluated one z plane at a time (the same formula per grid point)."""
    Lx, Ly, Lz = (int(v) for v in L)
    cell = np.asarray(cell, np.float64).reshape(3, 3)
    pref = constants()[3]

    def disp(Lk):
        k = np.arange(2 * Lk)
        d = np.where(k < Lk, k, k - 2 * Lk).astype(np.float64)
        d[Lk] = 0.0  # never reached by a displacement in [-(L-1), L-1]
        valid = np.ones(2 * Lk, bool)
        valid[Lk] = False
        return d, valid

    dx, vx = disp(Lx)
    dy, vy = disp(Ly)
    dz, vz = disp(Lz)
    names = {"xx": (0, 0), "xy": (0, 1), "xz": (0, 2), "yy": (1, 1), "yz": (1, 2), "zz": (2, 2)}
    comp = {k: np.zeros((2 * Lz, 2 * Ly, 2 * Lx)) for k in names}
    DY, DX = np.meshgrid(dy, dx, indexing="ij")
    vyx = vy[:, None] & vx[None, :]
    for iz in range(2 * Lz):
        r = DX[..., None] * cell[0] + DY[..., None] * cell[1] + dz[iz] * cell[2]
        rn = np.sqrt((r * r).sum(-1))
        ok = vyx & vz[iz] & (rn > 0)
        inv3 = np.zeros_like(rn)
        inv3[ok] = 1.0 / rn[ok] ** 3
        rh = np.zeros_like(r)
        rh[ok] = r[ok] / rn[ok][:, None]
        for k, (a, b) in names.items():
            comp[k][iz] = pref * (3.0 * rh[..., a] * rh[..., b] - (1.0 if a == b else 0.0)) * inv3
    return comp


def dipolar_field_fft(L, cell, mu, S):
    """b_dip (meV), shape (3, N), for a single-sublattice open sample."""
    Lx, Ly, Lz = (int(v) for v in L)
    S = np.asarray(S, np.float64).reshape(3, Lz, Ly, Lx)
    ker = dipole_kernel(L, cell)
    shape = (2 * Lz, 2 * Ly, 2 * Lx)
    nw = _workers()
    Sh = [sfft.rfftn(S[c], s=shape, workers=nw) for c in range(3)]
    Kh = {}
    for k in list(ker):
        Kh[k] = sfft.rfftn(ker.pop(k), workers=nw)
    idx = {(0, 0): "xx", (0, 1): "xy", (0, 2): "xz", (1, 0): "xy", (1, 1): "yy", (1, 2): "yz",
           (2, 0): "xz", (2, 1): "yz", (2, 2): "zz"}
    out = np.zeros((3, Lz, Ly, Lx))
    m = float(mu)
    for a in range(3):
        acc = sum(Kh[idx[(a, b)]] * Sh[b] for b in range(3))
        full = sfft.irfftn(acc, s=shape, workers=nw)
        out[a] = m * m * full[:Lz, :Ly, :Lx]
    return out.reshape(3, -1)
