"""Seeded synthetic inputs and workload descriptions.

This module holds no arithmetic of the method: it only draws the initial spin
states (NumPy PCG64 streams) and lists the lattice/model parameters of the
benchmark workloads as plain data.  Both the HIP path's tests and the oracle's
tests take their inputs from here, so that the two sides see identical bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


# ---------------------------------------------------------------- spin states
def random_sphere(N: int, seed: int) -> np.ndarray:
    """Uniform random unit vectors, shape (3, N): z ~ U[-1,1], phi ~ U[0,2pi)."""
    g = np.random.Generator(np.random.PCG64(seed))
    z = g.uniform(-1.0, 1.0, N)
    phi = g.uniform(0.0, 2.0 * np.pi, N)
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.ascontiguousarray(np.stack([r * np.cos(phi), r * np.sin(phi), z]))


def random_sphere_device(N: int, seed: int, device="cuda"):
    """Uniform random unit vectors drawn on a torch device, shape (3, N),
    FP64: z ~ U[-1,1], phi ~ U[0,2pi) from torch's seeded generator of that
    device.  For lattices too large to draw on the host (1024^3 spins); the
    same bits are then copied to whoever checks them."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    S = torch.empty((3, N), dtype=torch.float64, device=device)
    z = S[2]
    z.uniform_(-1.0, 1.0, generator=g)
    phi = S[0]
    phi.uniform_(0.0, 2.0 * np.pi, generator=g)
    r = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
    S[1].copy_(torch.sin(phi)).mul_(r)
    S[0].copy_(torch.cos(phi)).mul_(r)
    del r
    return S


def fm_tilt(N: int, seed: int, eps: float = 0.1) -> np.ndarray:
    """Ferromagnet along +z plus a seeded Gaussian tilt: (eps gx, eps gy, 1)/norm."""
    g = np.random.Generator(np.random.PCG64(seed))
    gx = g.standard_normal(N)
    gy = g.standard_normal(N)
    v = np.stack([eps * gx, eps * gy, np.ones(N)])
    return np.ascontiguousarray(v / np.sqrt((v * v).sum(0)))


def uniform_state(N: int, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    return np.ascontiguousarray(np.repeat(d[:, None], N, axis=1))


def hopfion_texture(L: Sequence[int], R0: Optional[float] = None, width: Optional[float] = None,
                    center_offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Toroidal Hopf-map-like seed texture of Hopf index 1 on an L^3 simple
    cubic grid, shape (3, N).  The core circle of radius R0 (default L/6) lies
    in the xy plane through the centre; rho is the distance to that circle,
    Theta = pi * max(0, 1 - rho/width) (width defaults to R0),
    Phi = azimuth + poloidal angle; spins far from the torus point along +z."""
    Lx, Ly, Lz = (int(v) for v in L)
    R0 = float(min(Lx, Ly, Lz)) / 6.0 if R0 is None else float(R0)
    w = R0 if width is None else float(width)
    cx = (Lx - 1) / 2.0 + center_offset[0]
    cy = (Ly - 1) / 2.0 + center_offset[1]
    cz = (Lz - 1) / 2.0 + center_offset[2]
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    X, Y, Z = x - cx, y - cy, z - cz
    rxy = np.sqrt(X * X + Y * Y)
    rho = np.sqrt((rxy - R0) ** 2 + Z * Z)
    theta = np.pi * np.clip(1.0 - rho / w, 0.0, 1.0)
    phi = np.arctan2(Y, X) + np.arctan2(Z, rxy - R0)
    S = np.stack([np.cos(phi) * np.sin(theta), np.sin(phi) * np.sin(theta), np.cos(theta)])
    return np.ascontiguousarray(S.reshape(3, -1))


# ---------------------------------------------------------------- workloads
SC_CELL = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


@dataclass
class Workload:
    """Lattice + Hamiltonian + dynamics parameters of one benchmark case."""
    name: str
    L: tuple
    n_sub: int = 1
    frac: tuple = ((0.0, 0.0, 0.0),)
    cell: tuple = SC_CELL
    periodic: tuple = (1, 1, 1)
    mu: tuple = (1.0,)
    J_shell: tuple = (1.0,)
    D_shell: Optional[tuple] = None
    K: float = 0.0
    K_axis: tuple = (0.0, 0.0, 1.0)
    B: tuple = (0.0, 0.0, 0.0)
    dipolar: int = 0
    alpha: float = 0.1
    dt_fs: float = 0.1
    T_K: float = 0.0
    n_steps: int = 100
    init: str = "random"
    init_seed: int = 1
    philox_seed: int = 1001
    field_prec: str = "fp64"
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.n_sub * self.L[0] * self.L[1] * self.L[2])

    @property
    def n_shells(self) -> int:
        return len(self.J_shell)

    def initial_state(self) -> np.ndarray:
        if self.init == "random":
            return random_sphere(self.N, self.init_seed)
        if self.init == "fm_tilt":
            return fm_tilt(self.N, self.init_seed)
        if self.init == "fm":
            return uniform_state(self.N)
        raise ValueError(self.init)

    def scaled(self, L) -> "Workload":
        """Same physics on a different lattice size (parity-test sizes)."""
        d = dict(self.__dict__)
        d["L"] = tuple(int(v) for v in L)
        return Workload(**d)


def sc_nn_fp64(L=(32, 32, 32)) -> Workload:
    """sc 32^3, NN J = 1 meV, K = 0.1 meV along z, deterministic Heun,
    alpha 0.1, dt 0.1 fs, 100 steps, FP64 throughout."""
    return Workload(name="sc32_nn_fp64_heun", L=L, J_shell=(1.0,), K=0.1, alpha=0.1, dt_fs=0.1,
                    T_K=0.0, n_steps=100, init="random", init_seed=1, philox_seed=1001,
                    field_prec="fp64")


BCC_FRAC = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.5))


def bcc_5shell_stochastic(L=(128, 128, 128)) -> Workload:
    """bcc as two sublattices, shells 1-5 J = 1.33, 0.75, -0.05, -0.10, 0.07
    meV, K = 0.005 meV along z, FM + tilt start, stochastic Heun at 300 K,
    alpha 0.05, dt 0.1 fs, FP32 field / FP64 state, 1000 steps."""
    return Workload(name="bcc128_5shell_stochastic_mixed", L=L, n_sub=2, frac=BCC_FRAC,
                    mu=(1.0, 1.0), J_shell=(1.33, 0.75, -0.05, -0.10, 0.07), K=0.005,
                    alpha=0.05, dt_fs=0.1, T_K=300.0, n_steps=1000, init="fm_tilt",
                    init_seed=2, philox_seed=1002, field_prec="fp32")


def sc_chiral_dipolar(L=(256, 256, 256)) -> Workload:
    """sc 256^3 chiral magnet, a = 0.4 nm, mu = 2, J = 1 meV, bulk DMI 0.3 meV
    along bonds, B = 0.5 T along z, open boundaries, dipolar via zero-padded FFT."""
    a = 0.4
    return Workload(name="sc256_chiral_dipolar_field", L=L, cell=((a, 0, 0), (0, a, 0), (0, 0, a)),
                    periodic=(0, 0, 0), mu=(2.0,), J_shell=(1.0,), D_shell=(0.3,),
                    B=(0.0, 0.0, 0.5), dipolar=1, init="random", init_seed=3, philox_seed=1003,
                    field_prec="fp32")


def sc_billion(L=(1024, 1024, 1024)) -> Workload:
    """sc 1024^3, J = 1 meV NN, K = 0.1 meV, stochastic Heun at 50 K, alpha 0.1,
    dt 0.1 fs, 100 steps, FP64 state with FP32 field."""
    return Workload(name="sc1024_nn_stochastic_mixed", L=L, J_shell=(1.0,), K=0.1, alpha=0.1,
                    dt_fs=0.1, T_K=50.0, n_steps=100, init="random", init_seed=4,
                    philox_seed=1004, field_prec="fp32")


def sc_frustrated_gneb(L=(48, 48, 48), shells="paper4") -> Workload:
    """Frustrated sc exchange for the hopfion GNEB workload, open boundaries.
    shells='config3': J1 = 1.0, J2 = -0.164, J3 = -0.082 meV;
    shells='paper4': J1 = 1 meV with the four-shell ratios 0.188, -0.274, -0.161."""
    J = (1.0, -0.164, -0.082) if shells == "config3" else (1.0, 0.188, -0.274, -0.161)
    return Workload(name="sc_frustrated_gneb", L=L, periodic=(0, 0, 0), J_shell=J,
                    init="hopfion", init_seed=5, field_prec="fp64")


WORKLOADS = {
    "sc32_nn_fp64_heun": sc_nn_fp64,
    "bcc128_5shell_stochastic_mixed": bcc_5shell_stochastic,
    "sc256_chiral_dipolar_field": sc_chiral_dipolar,
    "sc1024_nn_stochastic_mixed": sc_billion,
    "sc_frustrated_gneb": sc_frustrated_gneb,
}


def skyrmion_texture(L: Sequence[int], R: float, center=(0.0, 0.0), helicity: float = 0.5 * np.pi) -> np.ndarray:
    """Isolated skyrmion seed in every xy layer of an L grid, shape (3, N):
    core down, background +z, polar angle 2 atan(R / r), in-plane angle
    azimuth + helicity (pi/2: Bloch type)."""
    Lx, Ly, Lz = (int(v) for v in L)
    cx = (Lx - 1) / 2.0 + center[0]
    cy = (Ly - 1) / 2.0 + center[1]
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    X, Y = x - cx, y - cy
    r = np.sqrt(X * X + Y * Y)
    theta = 2.0 * np.arctan2(R, r)
    phi = np.arctan2(Y, X) + helicity
    S = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    return np.ascontiguousarray(S.reshape(3, -1))


# (mu0/4pi) mu_B^2 in meV nm^3 from the SI values (CODATA 2018 mu_B, exact e)
DIPOLE_PREFACTOR_MEV_NM3 = 1.0e-7 * 9.2740100783e-24 ** 2 / 1.602176634e-22 * 1.0e27


def dense7_couplings(J=1.0, D=0.3, mu=2.0, a=0.4, dipolar=True):
    """Input coupling table of the dense 7^3 window (simple cubic, lattice
    constant a nm, moment mu mu_B): J + bulk DMI (D along the bond) on the six
    nearest-neighbour offsets and, when dipolar is True, the dipole tensor
    (mu0/4pi) mu_B^2 mu^2 (3 r r - 1)/r^3 on every other offset of the window
    (the near field a dense convolution holds).  Returns (ab [n][2],
    delta [n][3], J [n][3][3]) in meV, offsets in (dz, dy, dx) loop order."""
    pref = DIPOLE_PREFACTOR_MEV_NM3 * mu * mu
    ab, dl, Js = [], [], []
    for dz in range(-3, 4):
        for dy in range(-3, 4):
            for dx in range(-3, 4):
                if dx == dy == dz == 0:
                    continue
                r = np.array([dx, dy, dz], float) * a
                rn = np.linalg.norm(r)
                u = r / rn
                if abs(dx) + abs(dy) + abs(dz) == 1:
                    Dv = D * u
                    T = J * np.eye(3) + np.array([[0, Dv[2], -Dv[1]], [-Dv[2], 0, Dv[0]], [Dv[1], -Dv[0], 0]])
                elif dipolar:
                    T = pref * (3 * np.outer(u, u) - np.eye(3)) / rn ** 3
                else:
                    continue
                ab.append((0, 0))
                dl.append((dx, dy, dz))
                Js.append(T)
    return np.array(ab, np.int32), np.array(dl, np.int32), np.array(Js)
