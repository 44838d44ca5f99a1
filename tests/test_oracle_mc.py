"""Pins of the oracle's Monte Carlo (Methods, Monte Carlo sampling) against
closed forms and brute force:

  - the colouring: no bond joins two sites of one colour (site by site in
    Python), and no valid colouring of the same linear form uses fewer colours
    (exhaustive search in Python on small lattices);
  - a free spin in a field b: the heat-bath draw gives <S.b^> = L(x) =
    coth x - 1/x and <(S.b^)^2> = 1 - 2 L(x)/x with x = beta |b|, and the
    cosine passes a Kolmogorov-Smirnov test against exp(x c) on [-1, 1];
    Metropolis reaches the same averages;
  - Metropolis with uniaxial anisotropy K: <S_z^2> equals the ratio of the
    integrals of c^2 exp(beta K c^2) and exp(beta K c^2) over [-1, 1];
  - the open classical Heisenberg chain: bond variables are independent, so
    <S_i.S_i+1> = L(beta J) and <S_0.S_r> = L(beta J)^r, for both methods;
  - heat-bath with anisotropy is refused.

Averages are checked to 4.5 standard errors (batch means for correlated
samples); the seeds are fixed, so the tests are deterministic.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from tests.helpers import oracle_model
from workloads import Workload, random_sphere

K_B = 8.617333262e-2   # meV/K
MU_B = 5.7883818060e-2  # meV/T


def langevin(x):
    return 1.0 / np.tanh(x) - 1.0 / x


def colour_of(L, C, coef, x, y, z, a):
    return (x + coef[0] * y + coef[1] * z + coef[2 + a]) % C


def valid(w, C, coef):
    m = oracle_model(w)
    Lx, Ly, Lz = w.L
    for a in range(w.n_sub):
        for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
            c0 = colour_of(w.L, C, coef, x, y, z, a)
            for p in range(m.n_bonds):
                if m.b_a[p] != a:
                    continue
                d = m.b_delta[3 * p:3 * p + 3]
                r = [x + d[0], y + d[1], z + d[2]]
                ok = True
                for k in range(3):
                    if not 0 <= r[k] < w.L[k]:
                        if not w.periodic[k]:
                            ok = False
                        r[k] %= w.L[k]
                if ok and colour_of(w.L, C, coef, *r, m.b_b[p]) == c0:
                    return False
    return True


@pytest.mark.parametrize("w,expect", [
    (Workload(name="sc4", L=(4, 4, 4)), 2),
    (Workload(name="sc5x4x4", L=(5, 4, 4)), 5),
    (Workload(name="chain", L=(6, 1, 1), periodic=(0, 0, 0)), 2),
    (Workload(name="sc2sh", L=(4, 4, 4), J_shell=(1.0, 0.5)), None),
    (Workload(name="open", L=(3, 3, 3), periodic=(0, 0, 0), J_shell=(1.0, 0.5, 0.2)), None),
])
def test_colouring_is_valid_and_minimal(w, expect):
    m = oracle_model(w)
    C, coef = oracle.mc_colouring(m)
    assert C >= 2 and valid(w, C, coef)
    if expect is not None:
        assert C == expect
    for Cs in range(2, C):                      # nothing smaller of the same form works
        for ky, kz in itertools.product(range(Cs), repeat=2):
            assert not valid(w, Cs, [ky, kz, 0]), (Cs, ky, kz)


def free_spin(b_meV, T_K):
    """1x1x1 open lattice, no exchange, Zeeman field giving the reduced field b (mu = 1)."""
    w = Workload(name="spin", L=(1, 1, 1), periodic=(0, 0, 0), J_shell=(0.0,), B=tuple(np.asarray(b_meV) / MU_B))
    return w, oracle_model(w)


def sample(m, S, T_K, n, method, seed, proj=None, burn=0):
    col = oracle.mc_colouring(m)
    out = []
    for k in range(burn + n):
        oracle.mc_sweeps(m, S, T_K, seed, sweep0=k, n_sweeps=1, method=method, colouring=col)
        if k >= burn:
            out.append(proj(S))
    return np.array(out)


def mean_err(x, batches=50):
    x = np.asarray(x)
    b = x[: len(x) // batches * batches].reshape(batches, -1).mean(axis=1)
    return x.mean(), b.std(ddof=1) / np.sqrt(batches)


@pytest.mark.parametrize("x", [0.5, 2.0, 8.0])
def test_heat_bath_free_spin_follows_the_langevin_function(x):
    T = 10.0
    bhat = np.array([0.3, -0.5, 0.81])
    bhat /= np.linalg.norm(bhat)
    w, m = free_spin(x * K_B * T * bhat, T)
    S = np.array([[1.0], [0.0], [0.0]])
    c = sample(m, S, T, 40000, 0, 11, proj=lambda s: float(s[:, 0] @ bhat))
    mu, se = c.mean(), c.std() / np.sqrt(len(c))       # heat-bath draws of a free spin are independent
    assert abs(mu - langevin(x)) < 4.5 * se
    c2 = (c * c).mean()
    assert abs(c2 - (1 - 2 * langevin(x) / x)) < 4.5 * (c * c).std() / np.sqrt(len(c))
    cdf = lambda t: (np.exp(x * t) - np.exp(-x)) / (np.exp(x) - np.exp(-x))
    assert stats.kstest(c, cdf).pvalue > 1e-3


def test_metropolis_free_spin_follows_the_langevin_function():
    T, x = 10.0, 2.0
    w, m = free_spin((0.0, 0.0, x * K_B * T), T)
    S = np.array([[0.0], [0.0], [1.0]])
    c = sample(m, S, T, 60000, 1, 12, proj=lambda s: float(s[2, 0]), burn=100)
    mu, se = mean_err(c)
    assert abs(mu - langevin(x)) < 4.5 * se


def test_metropolis_uniaxial_anisotropy():
    T, K = 10.0, 1.5 * K_B * 10.0                      # beta K = 1.5
    w = Workload(name="ani", L=(1, 1, 1), periodic=(0, 0, 0), J_shell=(0.0,), K=K)
    m = oracle_model(w)
    bk = K / (K_B * T)
    num = integrate.quad(lambda c: c * c * np.exp(bk * c * c), -1, 1)[0]
    den = integrate.quad(lambda c: np.exp(bk * c * c), -1, 1)[0]
    S = np.array([[1.0], [0.0], [0.0]])
    z2 = sample(m, S, T, 60000, 1, 13, proj=lambda s: float(s[2, 0] ** 2), burn=100)
    mu, se = mean_err(z2)
    assert abs(mu - num / den) < 4.5 * se


@pytest.mark.parametrize("method,bj", [(0, 1.0), (0, 2.5), (1, 1.0)])
def test_open_heisenberg_chain_bond_and_pair_correlations(method, bj):
    n, J = 8, 1.0
    T = J / (bj * K_B)
    w = Workload(name="chain", L=(n, 1, 1), periodic=(0, 0, 0), J_shell=(J,))
    m = oracle_model(w)
    S = random_sphere(n, 5)
    nn = lambda s: float(np.mean(np.sum(s[:, :-1] * s[:, 1:], axis=0)))
    r3 = lambda s: float(np.mean([s[:, i] @ s[:, i + 3] for i in range(n - 3)]))
    runs = 30000 if method == 0 else 60000
    col = oracle.mc_colouring(m)
    a1, a3 = [], []
    for k in range(runs + 200):
        oracle.mc_sweeps(m, S, T, 21 + method, sweep0=k, n_sweeps=1, method=method, colouring=col)
        if k >= 200:
            a1.append(nn(S))
            a3.append(r3(S))
    L1 = langevin(bj)
    mu1, se1 = mean_err(a1)
    mu3, se3 = mean_err(a3)
    assert abs(mu1 - L1) < 4.5 * se1, (mu1, L1, se1)
    assert abs(mu3 - L1 ** 3) < 4.5 * se3, (mu3, L1 ** 3, se3)


def test_heat_bath_refuses_anisotropy_and_keeps_the_state():
    w = Workload(name="ani", L=(2, 2, 2), J_shell=(1.0,), K=0.5)
    m = oracle_model(w)
    S = random_sphere(w.N, 3)
    S0 = S.copy()
    assert oracle.mc_sweeps(m, S, 10.0, 1, method=0) == -1
    assert np.array_equal(S, S0)
