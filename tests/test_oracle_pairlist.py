"""Pins of the oracle's pair-list Hamiltonian (Methods, pair-list backend):

  - a regular lattice written out as an explicit pair list (every bond of
    every site, wrapped on periodic axes and dropped at open faces, built here
    in Python from the lattice's bond table) gives the lattice oracle's field,
    energy and stochastic Heun trajectory;
  - for a disordered list with reciprocal couplings (J_ji = J_ij^T),
    per-site moments and anisotropies, the field is minus the gradient of an
    energy written here as an explicit pair sum (central differences);
  - at zero damping and temperature the Heun trajectory of that disordered
    system conserves its energy to the method's O(dt^2).
"""
import numpy as np
import pytest

import oracle
from tests.helpers import oracle_model
from workloads import Workload, bcc_5shell_stochastic, random_sphere

MU_B = 5.7883818060e-2


def lattice_to_pairlist(w):
    m = oracle_model(w)
    Lx, Ly, Lz = w.L
    M = Lx * Ly * Lz
    ti, sj, J = [], [], []
    for a in range(w.n_sub):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    i = a * M + x + Lx * (y + Ly * z)
                    for p in range(m.n_bonds):
                        if m.b_a[p] != a:
                            continue
                        d = m.b_delta[3 * p:3 * p + 3]
                        r = [x + d[0], y + d[1], z + d[2]]
                        keep = True
                        for k in range(3):
                            if not 0 <= r[k] < w.L[k]:
                                if not w.periodic[k]:
                                    keep = False
                                r[k] %= w.L[k]
                        if keep:
                            ti.append(i)
                            sj.append(m.b_b[p] * M + r[0] + Lx * (r[1] + Ly * r[2]))
                            J.append(np.asarray(m.b_J[9 * p:9 * p + 9]).reshape(3, 3))
    mu = np.repeat(np.asarray(w.mu, np.float64), M)
    K = Kax = None
    if w.K:
        K = np.full(w.N, w.K)
        Kax = np.tile(np.asarray(w.K_axis, np.float64), (w.N, 1))
    return oracle.PairList(w.N, ti, sj, np.array(J), mu=mu, K=K, K_axis=Kax, B=w.B)


CASES = [Workload(name="sc", L=(4, 3, 5), periodic=(1, 0, 1), J_shell=(1.0, -0.3, 0.1), D_shell=(0.4, 0.0, 0.0),
                  K=0.2, K_axis=(0.0, 0.6, 0.8), B=(1.0, -2.0, 0.5)),
         bcc_5shell_stochastic((3, 3, 3))]
CASES[1].periodic = (1, 1, 0)


@pytest.mark.parametrize("w", CASES, ids=["sc3shell_dmi", "bcc5shell"])
def test_lattice_as_pairlist_matches_the_lattice(w):
    pl = lattice_to_pairlist(w)
    m = oracle_model(w)
    S = random_sphere(w.N, 4)
    b_lat = oracle.field(m, S)
    b_pl = oracle.pl_field(pl, S)
    assert np.max(np.abs(b_pl - b_lat)) < 1e-12 * max(1.0, np.max(np.abs(b_lat)))
    np.testing.assert_allclose(oracle.pl_energy(pl, S)[[0, 1, 2, 4]], oracle.energy(m, S)[[0, 1, 2, 4]],
                               rtol=1e-12, atol=1e-12)
    kw = dict(alpha=0.1, dt_fs=0.2, T_K=150.0, seed=7, step0=3, n_steps=4)
    ref = oracle.heun(m, S, **kw)
    got = oracle.pl_heun(pl, S, **kw)
    assert np.max(np.abs(got - ref)) < 1e-12


def disordered(N=40, P=300, seed=3):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, N, P)
    j = (i + rng.integers(1, N, P)) % N                       # no self-coupling
    J = rng.normal(0.0, 1.0, (P, 3, 3))
    ti = np.concatenate([i, j])
    sj = np.concatenate([j, i])
    JJ = np.concatenate([J, np.transpose(J, (0, 2, 1))])       # reciprocal entries
    mu = rng.uniform(0.5, 3.0, N)
    K = rng.uniform(-0.5, 0.5, N)
    ax = rng.normal(size=(N, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    return oracle.PairList(N, ti, sj, JJ, mu=mu, K=K, K_axis=ax, B=(0.3, -0.2, 1.1)), (ti, sj, JJ, mu, K, ax)


def pair_sum_energy(parts, B, S):
    ti, sj, JJ, mu, K, ax = parts
    e = -0.5 * np.einsum("pa,pab,pb->", S[:, ti].T, JJ, S[:, sj].T)
    e -= np.sum(mu * MU_B * (np.asarray(B) @ S))
    e -= np.sum(K * np.einsum("ci,ic->i", S, ax) ** 2)
    return e


def test_disordered_field_is_minus_the_energy_gradient():
    pl, parts = disordered()
    S = random_sphere(pl.N, 5)
    b = oracle.pl_field(pl, S)
    h = 1e-6
    for i in (0, 7, 19, 33):
        for c in range(3):
            Sp, Sm = S.copy(), S.copy()
            Sp[c, i] += h
            Sm[c, i] -= h
            g = (pair_sum_energy(parts, pl.B, Sp) - pair_sum_energy(parts, pl.B, Sm)) / (2 * h)
            assert abs(b[c, i] + g) < 1e-6 * max(1.0, abs(g)), (i, c, b[c, i], -g)
    assert abs(oracle.pl_energy(pl, S)[4] - pair_sum_energy(parts, pl.B, S)) < 1e-10


def test_disordered_heun_conserves_energy_without_damping():
    pl, parts = disordered(N=30, P=120, seed=8)
    S = random_sphere(pl.N, 6)
    E0 = oracle.pl_energy(pl, S)[4]
    drift = []
    for dt in (0.2, 0.1):
        X = oracle.pl_heun(pl, S, alpha=0.0, dt_fs=dt, n_steps=int(round(40 / dt)))
        drift.append(abs(oracle.pl_energy(pl, X)[4] - E0))
    assert drift[0] < 1e-3 * abs(E0)
    assert drift[1] < drift[0] / 3.0                           # second order in dt


def empty_list(N=37, seed=9):
    rng = np.random.default_rng(seed)
    ax = rng.normal(size=(N, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    mu, K = rng.uniform(0.5, 3.0, N), rng.uniform(-0.5, 0.5, N)
    e = np.zeros(0, np.int64)
    return oracle.PairList(N, e, e, np.zeros((0, 3, 3)), mu=mu, K=K, K_axis=ax, B=(0.3, -0.2, 1.1))


def test_empty_list_field_and_energy_are_the_onsite_closed_forms():
    # no couplings: each site sees its own Zeeman field mu muB B and the
    # anisotropy field 2 K (a.S) a, and the energy is the sum of -mu muB B.S
    # and -K (a.S)^2
    pl = empty_list()
    S = random_sphere(pl.N, 3)
    proj = np.einsum("ci,ic->i", S, pl.K_axis.reshape(-1, 3))
    want = MU_B * pl.mu[None, :] * pl.B[:, None] + 2.0 * pl.K[None, :] * proj[None, :] * pl.K_axis.reshape(-1, 3).T
    assert np.max(np.abs(oracle.pl_field(pl, S) - want)) < 1e-14
    t = oracle.pl_energy(pl, S)
    assert abs(t[4] - (-np.sum(MU_B * pl.mu * (pl.B @ S)) - np.sum(pl.K * proj ** 2))) < 1e-12
    assert t[0] == 0.0
