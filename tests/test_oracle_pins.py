"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (closed forms, invariants, brute force, textbook special cases).

Each test names the passage of the paper (Methods) it pins.  None of these
tests touches the HIP library.
"""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import max_rel, oracle_lattice, oracle_model
from workloads import (BCC_FRAC, Workload, bcc_5shell_stochastic, fm_tilt, random_sphere,
                       sc_chiral_dipolar, uniform_state)

MU_B, K_B, GAMMA, DIP = None, None, None, None


@pytest.fixture(scope="module", autouse=True)
def _consts(oracle_mod):
    global MU_B, K_B, GAMMA, DIP
    MU_B, K_B, GAMMA, DIP = oracle.constants()


# ---------------------------------------------------------------- constants
def test_constants_match_paper_and_codata():
    # Methods: mu_B ~ 5.7884e-2 meV/T
    assert abs(MU_B - 5.7884e-2) < 5e-7
    # mu0/4pi mu_B^2 in meV nm^3 from SI values: 1e-7 * muB_J^2 / meV_J * 1e27
    assert abs(DIP - 5.36815e-5) / 5.36815e-5 < 1e-5
    # k_B = R / N_A in meV/K (gas constant / Avogadro, independent route)
    assert abs(K_B - 8.314462618 / 6.02214076e23 / 1.602176634e-22) < 1e-10
    # gamma = g_e mu_B / hbar (free-electron g), in rad/(fs T)
    g_e, muB_J, hbar = 2.00231930436256, 9.2740100783e-24, 1.054571817e-34
    assert abs(GAMMA - g_e * muB_J / hbar * 1e-15) / GAMMA < 1e-9


# ---------------------------------------------------------------- shells and bond tables
def _bond_counts(n_sub, frac, n_shells):
    lat = oracle.Lattice((4, 4, 4), np.eye(3), frac, mu=np.ones(n_sub))
    m = oracle.Model(lat, n_shells=n_shells, J_shell=np.arange(1, n_shells + 1, dtype=float))
    return m, np.bincount(m.b_shell, minlength=n_shells)


def test_sc_shell_counts():
    # simple cubic coordination numbers 6, 12, 8, 6, 24 at r^2 = 1, 2, 3, 4, 5
    lat = oracle.Lattice((4, 4, 4), np.eye(3), [0, 0, 0])
    d = oracle.shell_distances(lat, 5)
    np.testing.assert_allclose(d ** 2, [1, 2, 3, 4, 5], rtol=0, atol=1e-12)
    _, c = _bond_counts(1, [0, 0, 0], 5)
    assert list(c) == [6, 12, 8, 6, 24]


def test_bcc_shell_counts_and_windows():
    # bcc: 8, 6, 12, 24, 8 neighbours at r^2/a^2 = 0.75, 1, 2, 2.75, 3 (per site,
    # two sublattices -> doubled counts in the directed table)
    lat = oracle.Lattice((4, 4, 4), np.eye(3), BCC_FRAC, mu=[1, 1])
    d = oracle.shell_distances(lat, 5)
    np.testing.assert_allclose(d ** 2, [0.75, 1, 2, 2.75, 3], atol=1e-12)
    m, c = _bond_counts(2, BCC_FRAC, 5)
    assert list(c) == [16, 12, 24, 48, 16]
    delta = m.b_delta.reshape(-1, 3)
    for (a, b), (lo, hi, cnt) in {(0, 0): (-1, 1, 26), (1, 1): (-1, 1, 26),
                                  (0, 1): (-2, 1, 32), (1, 0): (-1, 2, 32)}.items():
        sel = (m.b_a == a) & (m.b_b == b)
        assert sel.sum() == cnt
        assert delta[sel].min() == lo and delta[sel].max() == hi


def test_bond_table_reciprocity():
    # Methods: J_ji^{beta alpha} = J_ij^{alpha beta}, D_ji = -D_ij
    lat = oracle.Lattice((4, 4, 4), np.eye(3), BCC_FRAC, mu=[1, 1])
    m = oracle.Model(lat, n_shells=2, J_shell=[1.0, 0.5], D_shell=[0.3, -0.2])
    d = m.b_delta.reshape(-1, 3)
    J = m.b_J.reshape(-1, 3, 3)
    for p in range(m.n_bonds):
        q = [k for k in range(m.n_bonds) if m.b_a[k] == m.b_b[p] and m.b_b[k] == m.b_a[p]
             and np.all(d[k] == -d[p])]
        assert len(q) == 1
        np.testing.assert_allclose(J[q[0]], J[p].T, atol=1e-15)


# ---------------------------------------------------------------- field: brute force
@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_field_matches_bruteforce_sc_dmi_periodic(L):
    w = Workload(name="t", L=(L, L, L), J_shell=(1.0, -0.3), D_shell=(0.4, 0.1))
    m = oracle_model(w)
    S = random_sphere(w.N, 11 + L)
    b = oracle.field(m, S)
    bb, _ = oracle.bruteforce(m, S)
    assert max_rel(b, bb) < 1e-13


@pytest.mark.parametrize("L", [(1, 1, 1), (2, 3, 2), (4, 4, 4)])
def test_field_matches_bruteforce_bcc_5shell(L):
    w = bcc_5shell_stochastic(L)
    w.K = 0.0
    m = oracle_model(w)
    S = random_sphere(w.N, 7)
    assert max_rel(oracle.field(m, S), oracle.bruteforce(m, S)[0]) < 1e-13


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 0, 1)])
def test_field_matches_bruteforce_open(per):
    w = Workload(name="t", L=(5, 4, 6), periodic=per, J_shell=(1.0, 0.2, -0.1), D_shell=(0.3, 0.0, 0.05))
    m = oracle_model(w)
    S = random_sphere(w.N, 5)
    assert max_rel(oracle.field(m, S), oracle.bruteforce(m, S)[0]) < 1e-13


def test_pair_energy_equals_half_field_form():
    # Methods: ordered-pair form with 1/2 equals the unordered pair sum
    for per, L in (((1, 1, 1), (3, 3, 3)), ((0, 0, 0), (4, 3, 5)), ((1, 1, 1), (1, 1, 1))):
        w = Workload(name="t", L=L, periodic=per, J_shell=(1.0, -0.4), D_shell=(0.3, 0.2))
        m = oracle_model(w)
        S = random_sphere(w.N, 3)
        e = oracle.energy(m, S)
        _, ep = oracle.bruteforce(m, S)
        assert abs(e[0] - ep) < 1e-12 * max(1.0, abs(ep))


# ---------------------------------------------------------------- field: closed forms
def test_fm_closed_form_sc_and_bcc():
    w = Workload(name="t", L=(4, 4, 4), J_shell=(1.0,), K=0.1)
    m = oracle_model(w)
    S = uniform_state(w.N)
    b = oracle.field(m, S)
    np.testing.assert_allclose(b[2], 6 * 1.0 + 2 * 0.1, rtol=0, atol=1e-13)
    np.testing.assert_allclose(b[:2], 0.0, atol=1e-13)
    e = oracle.energy(m, S)
    assert abs(e[4] / w.N - (-0.5 * 6.0 - 0.1)) < 1e-13
    wb = bcc_5shell_stochastic((3, 3, 3))
    mb = oracle_model(wb)
    Sb = uniform_state(wb.N)
    bb = oracle.field(mb, Sb)
    zJ = 8 * 1.33 + 6 * 0.75 + 12 * -0.05 + 24 * -0.10 + 8 * 0.07
    assert abs(zJ - 12.7) < 1e-12
    np.testing.assert_allclose(bb[2], zJ + 2 * 0.005, atol=1e-12)
    eb = oracle.energy(mb, Sb)
    assert abs(eb[4] / wb.N - (-0.5 * zJ - 0.005)) < 1e-12


@pytest.mark.parametrize("m_wind", [1, 2, 3])
def test_helix_closed_form_dmi(m_wind):
    # S(x) = (0, cos qx, sin qx): b = (4J + 2J cos q + 2D sin q) S, pins the wrap,
    # the DMI sign and the tensor layout (Methods, DMI tensor)
    L = 12
    J, D = 1.0, 0.3
    q = 2 * np.pi * m_wind / L
    w = Workload(name="t", L=(L, 5, 4), J_shell=(J,), D_shell=(D,))
    mo = oracle_model(w)
    x = np.tile(np.arange(L), 5 * 4).astype(float)
    S = np.stack([np.zeros_like(x), np.cos(q * x), np.sin(q * x)])
    b = oracle.field(mo, S)
    lam = 4 * J + 2 * J * np.cos(q) + 2 * D * np.sin(q)
    np.testing.assert_allclose(b, lam * S, atol=1e-13)
    e = oracle.energy(mo, S)
    assert abs(e[0] / w.N + 0.5 * lam) < 1e-13


def test_helix_is_stationary_under_heun():
    L = 10
    q = 2 * np.pi / L
    w = Workload(name="t", L=(L, 3, 3), J_shell=(1.0,), D_shell=(0.3,))
    mo = oracle_model(w)
    x = np.tile(np.arange(L), 9).astype(float)
    S = np.stack([np.zeros_like(x), np.cos(q * x), np.sin(q * x)])
    S2 = oracle.heun(mo, S, alpha=0.1, dt_fs=1.0, n_steps=5)
    assert np.max(np.abs(S2 - S)) < 1e-14


def test_zeeman_and_anisotropy_terms():
    w = Workload(name="t", L=(3, 2, 2), J_shell=(0.0,), mu=(2.0,), K=0.7, K_axis=(0.6, 0.0, 0.8),
                 B=(0.3, -0.2, 1.5))
    m = oracle_model(w)
    S = random_sphere(w.N, 9)
    b, parts = oracle.field(m, S, terms=True)
    n = np.array([0.6, 0.0, 0.8])
    sn = n @ S
    np.testing.assert_allclose(parts["aniso"], 2 * 0.7 * sn * n[:, None], atol=1e-14)
    np.testing.assert_allclose(parts["zeeman"], 2.0 * MU_B * np.array([0.3, -0.2, 1.5])[:, None]
                               * np.ones(w.N), atol=1e-14)
    e = oracle.energy(m, S)
    assert abs(e[2] - (-0.7 * np.sum(sn ** 2))) < 1e-12
    assert abs(e[1] - (-2.0 * MU_B * np.sum(np.array([0.3, -0.2, 1.5]) @ S))) < 1e-12


def test_zeeman_field_is_minus_gradient():
    # B_eff = -(1/(mu mu_B)) dH/dS: finite-difference check of the full field
    w = Workload(name="t", L=(3, 3, 2), periodic=(1, 0, 1), J_shell=(1.0, -0.2), D_shell=(0.3, 0.1),
                 K=0.2, K_axis=(0.0, 0.6, 0.8), B=(0.1, 0.2, 0.3), mu=(1.5,))
    m = oracle_model(w)
    S = random_sphere(w.N, 2)
    b = oracle.field(m, S)
    h = 1e-6
    for i in (0, 5, w.N - 1):
        for c in range(3):
            Sp, Sm = S.copy(), S.copy()
            Sp[c, i] += h
            Sm[c, i] -= h
            g = (oracle.energy(m, Sp)[4] - oracle.energy(m, Sm)[4]) / (2 * h)
            assert abs(-g - b[c, i]) < 1e-7


# ---------------------------------------------------------------- dipolar
def test_dipolar_two_dipole_closed_forms():
    # a pair of dipoles a distance r apart: field on one from the other is
    # pref mu mu (3 rhat(rhat.S) - S)/r^3: +2/r^3 along the axis, -1/r^3 across
    a = 0.4
    from oracle import Lattice
    lat = Lattice((2, 1, 1), np.eye(3) * a, [0, 0, 0], periodic=(0, 0, 0), mu=[2.0])
    S = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    b = oracle.dipolar_direct(lat, S, [0])
    assert abs(b[0, 0] - DIP * 4 * 2 / a ** 3) < 1e-15 and abs(b[1, 0]) < 1e-18
    S = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 1.0]])
    b = oracle.dipolar_direct(lat, S, [0])
    assert abs(b[2, 0] - DIP * 4 * (-1) / a ** 3) < 1e-15


def test_dipolar_cubic_symmetry_zero_at_centre():
    # uniformly magnetised odd sc cube: the dipole sum at the centre vanishes
    from oracle import Lattice
    L = 7
    lat = Lattice((L, L, L), np.eye(3) * 0.4, [0, 0, 0], periodic=(0, 0, 0), mu=[2.0])
    for d in ((0, 0, 1), (1, 1, 1), (0.3, -0.5, 0.8)):
        S = uniform_state(lat.N, d)
        c = (L // 2) * (1 + L + L * L)
        b = oracle.dipolar_direct(lat, S, [c])
        b_edge = oracle.dipolar_direct(lat, S, [0])
        assert np.max(np.abs(b)) < 1e-12 * np.max(np.abs(b_edge))


@pytest.mark.parametrize("L", [(4, 4, 4), (6, 5, 3)])
def test_dipolar_fft_matches_direct(L):
    from oracle import Lattice
    from oracle.dipolar_fft import dipolar_field_fft
    cell = np.eye(3) * 0.4
    lat = Lattice(L, cell, [0, 0, 0], periodic=(0, 0, 0), mu=[2.0])
    S = random_sphere(lat.N, 13)
    direct = oracle.dipolar_direct(lat, S, np.arange(lat.N))
    fft = dipolar_field_fft(L, cell, 2.0, S)
    assert max_rel(fft, direct) < 1e-12


def test_dipolar_energy_pair_reciprocity():
    # E_dip = -1/2 sum S.b_dip equals the unordered pair sum of H_dip
    w = Workload(name="t", L=(3, 3, 2), periodic=(0, 0, 0), J_shell=(0.0,), mu=(2.0,),
                 cell=((0.4, 0, 0), (0, 0.4, 0), (0, 0, 0.4)), dipolar=1)
    m = oracle_model(w)
    S = random_sphere(w.N, 21)
    e = oracle.energy(m, S)[3]
    pos = []
    for i in range(w.N):
        x, y, z = i % 3, (i // 3) % 3, i // 9
        pos.append(np.array([x, y, z]) * 0.4)
    ep = 0.0
    for i in range(w.N):
        for j in range(i + 1, w.N):
            r = pos[j] - pos[i]
            rn = np.linalg.norm(r)
            u = r / rn
            ep -= DIP * 4.0 * (3 * (S[:, i] @ u) * (S[:, j] @ u) - S[:, i] @ S[:, j]) / rn ** 3
    assert abs(e - ep) < 1e-12 * abs(ep)


# ---------------------------------------------------------------- Philox / noise
def test_philox_statistics_and_counter_sensitivity():
    blocks = np.array([oracle.philox([i, 0, 7, 0], [123, 456]) for i in range(4096)])
    u = (blocks.astype(np.float64) + 0.5) / 2 ** 32
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005
    # one-bit changes of counter or key give unrelated outputs
    b0 = oracle.philox([0, 0, 0, 0], [0, 0])
    for ctr, key in (([1, 0, 0, 0], [0, 0]), ([0, 0, 0, 1 << 31], [0, 0]), ([0, 0, 0, 0], [1, 0])):
        b1 = oracle.philox(ctr, key)
        assert np.all(b0 != b1)


def test_thermal_eta_moments():
    eta = oracle.thermal_eta(seed=99, step=3, N=200000)
    assert np.all(np.abs(eta.mean(axis=1)) < 0.01)
    assert np.all(np.abs(eta.var(axis=1) - 1.0) < 0.015)
    c = np.corrcoef(eta)
    assert np.max(np.abs(c - np.eye(3))) < 0.01
    # fourth moment of a standard normal is 3
    assert np.all(np.abs((eta ** 4).mean(axis=1) - 3.0) < 0.1)
    eta2 = oracle.thermal_eta(seed=99, step=4, N=200000)
    assert abs(np.corrcoef(eta[0], eta2[0])[0, 1]) < 0.01


# ---------------------------------------------------------------- LLG / Heun
def _single_spin_model(B=1.0, alpha=0.01, mu=1.0):
    w = Workload(name="t", L=(1, 1, 1), J_shell=(0.0,), mu=(mu,), B=(0.0, 0.0, B))
    return oracle_model(w)


def _analytic_precession(t, B, alpha):
    gp = GAMMA / (1 + alpha ** 2)
    phi = gp * B * t
    th = 2 * np.arctan(np.tan(np.pi / 4) * np.exp(-alpha * gp * B * t))
    return np.stack([np.cos(phi) * np.sin(th), np.sin(phi) * np.sin(th), np.cos(th)])


def _rmse_single_spin(dt, B=1.0, alpha=0.01, t_total=500000.0, sample=1000.0):
    m = _single_spin_model(B, alpha)
    S = np.array([[1.0], [0.0], [0.0]])
    per = int(round(sample / dt))
    errs = []
    for k in range(1, int(t_total / sample) + 1):
        S = oracle.heun(m, S, alpha=alpha, dt_fs=dt, n_steps=per)
        ref = _analytic_precession(k * sample, B, alpha)
        errs.append(np.sum((S[:, 0] - ref) ** 2))
    return math.sqrt(np.mean(errs))


def test_single_spin_precession_second_order():
    # Fig. 2a benchmark: B = 1 T along z, alpha = 0.01, S0 = x, 500 ps sampled
    # every 1 ps; Heun's global error is O(dt^2)
    e1 = _rmse_single_spin(50.0)
    e2 = _rmse_single_spin(25.0)
    assert e1 < 5e-3
    assert 3.6 < e1 / e2 < 4.4


def test_zero_damping_energy_drift_second_order():
    w = Workload(name="t", L=(4, 4, 4), J_shell=(1.0, -0.1), D_shell=(0.2, 0.0), K=0.3)
    m = oracle_model(w)
    S0 = fm_tilt(w.N, 4, eps=0.5)
    E0 = oracle.energy(m, S0)[4]
    drifts = []
    # asymptotic regime (omega dt ~ 1e-3): halving dt quarters the drift
    for dt in (0.1, 0.05):
        S = oracle.heun(m, S0, alpha=0.0, dt_fs=dt, n_steps=int(round(100 / dt)))
        drifts.append(abs(oracle.energy(m, S)[4] - E0))
    assert drifts[0] > 0
    assert 3.6 < drifts[0] / drifts[1] < 4.6


def test_damped_energy_decreases_and_norm_preserved():
    w = Workload(name="t", L=(4, 4, 4), J_shell=(1.0, 0.2), K=0.1, B=(0, 0, 1.0))
    m = oracle_model(w)
    S = random_sphere(w.N, 8)
    E = oracle.energy(m, S)[4]
    for _ in range(10):
        S = oracle.heun(m, S, alpha=0.5, dt_fs=1.0, n_steps=5)
        assert np.max(np.abs(np.sqrt((S * S).sum(0)) - 1)) < 1e-14
        E2 = oracle.energy(m, S)[4]
        assert E2 <= E + 1e-12
        E = E2


def _langevin_mz(T, B=10.0, alpha=0.5, dt=5.0, N=4096, burn=3000, meas=3000, seed=77):
    m = _single_spin_model_many(N, B)
    S = uniform_state(N)
    S = oracle.heun(m, S, alpha=alpha, dt_fs=dt, T_K=T, seed=seed, step0=0, n_steps=burn)
    acc = 0.0
    chunk = 100
    for k in range(meas // chunk):
        S = oracle.heun(m, S, alpha=alpha, dt_fs=dt, T_K=T, seed=seed, step0=burn + k * chunk,
                        n_steps=chunk)
        acc += S[2].mean()
    return acc / (meas // chunk)


def _single_spin_model_many(N, B):
    w = Workload(name="t", L=(N, 1, 1), J_shell=(0.0,), B=(0.0, 0.0, B))
    return oracle_model(w)


def test_stochastic_heun_reaches_langevin_function():
    # Brown / stochastic LLG: non-interacting spins equilibrate to
    # <S_z> = coth x - 1/x, x = mu mu_B B / (k_B T).  With alpha = 0.5 this
    # pins sigma's factor 2 and the absence of a (1+alpha^2) factor.
    for T in (2.0, 6.0):
        x = MU_B * 10.0 / (K_B * T)
        ref = 1 / math.tanh(x) - 1 / x
        got = _langevin_mz(T)
        assert abs(got - ref) < 0.006, (T, got, ref)


def test_stochastic_same_noise_both_stages_and_reproducible():
    w = Workload(name="t", L=(4, 4, 4), J_shell=(1.0,), K=0.1)
    m = oracle_model(w)
    S = random_sphere(w.N, 1)
    a = oracle.heun(m, S, alpha=0.1, dt_fs=0.1, T_K=300, seed=5, step0=10, n_steps=3)
    b = oracle.heun(m, S, alpha=0.1, dt_fs=0.1, T_K=300, seed=5, step0=10, n_steps=3)
    assert np.array_equal(a, b)
    # resume: 2 steps + 1 step from the saved step counter == 3 steps
    c = oracle.heun(m, S, alpha=0.1, dt_fs=0.1, T_K=300, seed=5, step0=10, n_steps=2)
    c = oracle.heun(m, c, alpha=0.1, dt_fs=0.1, T_K=300, seed=5, step0=12, n_steps=1)
    assert np.array_equal(a, c)


# ---------------------------------------------------------------- manifold geometry / GNEB
def test_geodesic_distance_uniform_rotation():
    N = 50
    S = random_sphere(N, 3)
    th = 0.37
    c, s = math.cos(th), math.sin(th)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    # rotate each spin about its own perpendicular axis by th: use the exp map
    # construction with an explicit unit tangent
    t = np.cross(S.T, np.array([0.3, 0.5, 0.8])).T
    t /= np.sqrt((t * t).sum(0))
    S2 = c * S + s * t
    assert abs(oracle.image_distance(S, S2) - math.sqrt(N) * th) < 1e-12
    del R


def test_geodesic_path_properties():
    N = 40
    SA = random_sphere(N, 1)
    SB = random_sphere(N, 2)
    SA[:, 0] = [0, 0, 1.0]
    SB[:, 0] = [0, 0, -1.0]   # antipodal
    SA[:, 1] = SB[:, 1]       # parallel
    n_img = 9
    P = oracle.geodesic_path(SA, SB, n_img)
    np.testing.assert_allclose(P[0], SA, atol=1e-15)
    np.testing.assert_allclose(P[-1], SB, atol=1e-12)
    ang = np.arctan2(np.linalg.norm(np.cross(SA.T, SB.T), axis=1), (SA * SB).sum(0))
    for n in range(n_img - 1):
        d = np.arctan2(np.linalg.norm(np.cross(P[n].T, P[n + 1].T), axis=1), (P[n] * P[n + 1]).sum(0))
        np.testing.assert_allclose(d, ang / (n_img - 1), atol=1e-12)
        # each spin stays on the great circle through SA and SB
    # antipodal rule: -z -> +z via x, first image tilts toward +x
    Q = oracle.geodesic_path(-SA[:, :1], SA[:, :1], 3)
    np.testing.assert_allclose(Q[1][:, 0], [1.0, 0.0, 0.0], atol=1e-15)


def _sw_model(K=1.0, h=0.3, L=(1, 1, 1), J=0.0):
    B = 2 * K * h / MU_B
    w = Workload(name="t", L=L, J_shell=(J,), K=K, B=(0, 0, B))
    return oracle_model(w)


def test_gneb_stoner_wohlfarth_barrier_and_saddle():
    # macrospin E(theta) = -K cos^2 theta - mu mu_B B cos theta, h = mu mu_B B/(2K):
    # saddle at cos theta* = -h, barrier from theta = pi is K (1 - h)^2
    K, h = 1.0, 0.3
    m = _sw_model(K, h)
    SA = np.array([[0.0], [0.0], [-1.0]])
    SB = np.array([[0.0], [0.0], [1.0]])
    st = oracle.GnebState(oracle.geodesic_path(SA, SB, 9), k_spring=1.0, dt=0.2, mass=1.0,
                          ci_mode=1, ci_on_below=1e-2)
    for it in range(4000):
        E, dist, fmax, ci = oracle.gneb_iterate(m, st)
        if ci >= 0 and fmax < 1e-9:
            break
    assert ci >= 0 and fmax < 1e-9
    Sci = st.Y[ci][:, 0]
    assert abs(Sci[2] - (-h)) < 1e-6
    barrier = E[ci] - E[0]
    assert abs(barrier - K * (1 - h) ** 2) < 1e-8
    # the path stays on the great circle in the xz plane
    assert np.max(np.abs(st.Y[:, 1, 0])) < 1e-12


def test_gneb_coherent_rotation_block():
    # strongly exchange-coupled periodic 3^3 block: coherent rotation, barrier N K (1-h)^2
    K, h = 0.1, 0.2
    m = _sw_model(K, h, L=(3, 3, 3), J=5.0)
    N = 27
    SA = uniform_state(N, (0, 0, -1))
    SB = uniform_state(N, (0, 0, 1))
    st = oracle.GnebState(oracle.geodesic_path(SA, SB, 7), k_spring=1.0, dt=0.3, mass=1.0,
                          ci_mode=2)
    for it in range(3000):
        E, dist, fmax, ci = oracle.gneb_iterate(m, st)
        if fmax < 1e-9:
            break
    assert abs((E[ci] - E[0]) - N * K * (1 - h) ** 2) < 1e-7
    # springs act on each side of the climbing image separately: equal spacing
    # among the segments left of it and among those right of it
    np.testing.assert_allclose(dist[:ci], dist[0], rtol=1e-6)
    np.testing.assert_allclose(dist[ci:], dist[-1], rtol=1e-6)
    assert abs(dist.sum() - math.sqrt(N) * math.pi) < 1e-6


def test_gneb_minimisation_mode_relaxes_images_to_their_basins():
    # static minimisation: images relax independently of springs and tangent;
    # macrospin images with cos theta > -h fall into theta = 0, the others into pi
    K, h = 1.0, 0.3
    m = _sw_model(K, h)
    SA = np.array([[0.0], [0.0], [-1.0]])
    SB = np.array([[0.0], [0.0], [1.0]])
    Y0 = oracle.geodesic_path(SA, SB, 9)
    out = []
    for k in (0.0, 7.0):
        st = oracle.GnebState(Y0.copy(), k_spring=k, dt=0.2, mass=1.0, ci_mode=3)
        for it in range(3000):
            E, dist, fmax, ci = oracle.gneb_iterate(m, st)
            if fmax < 1e-10:
                break
        assert ci == -1 and fmax < 1e-10
        out.append(st.Y.copy())
    np.testing.assert_array_equal(out[0], out[1])
    for n in range(9):
        want = 1.0 if Y0[n][2, 0] > -h else -1.0
        assert abs(out[0][n][2, 0] - want) < 1e-9, n


# ---------------------------------------------------------------- net
def test_net_single_channel_conv_is_correlation():
    # one input / output channel, 3^3 kernel, zero padding == scipy correlate
    from scipy.ndimage import correlate
    rng = np.random.default_rng(0)
    L = (5, 4, 3)
    ch = (1, 1, 1, 1, 1)
    n = oracle.net_nparams(ch)
    assert n == 4 * 28
    # identity layers 2..4 (centre tap 1, bias 0) are not identities after SiLU,
    # so check layer 1 alone via a net whose last three layers are linear in
    # the SiLU output: compare the pre-activation saved by the forward pass
    p = np.zeros(n)
    k1 = rng.standard_normal(27)
    p[:27] = k1
    p[27] = 0.25
    x = rng.standard_normal((1, L[0] * L[1] * L[2]))
    _, act = oracle.net_forward(L, p, x, ch=ch, want_act=True)
    xr = x.reshape(L[2], L[1], L[0])
    ref = correlate(xr, k1.reshape(3, 3, 3), mode="constant", cval=0.0) + 0.25
    np.testing.assert_allclose(act[0], ref.reshape(-1), atol=1e-12)
    # layer 2 input is SiLU(layer-1 output)
    p2 = p.copy()
    p2[28 + 13] = 1.0  # centre tap of layer 2
    _, act2 = oracle.net_forward(L, p2, x, ch=ch, want_act=True)
    silu = ref * (1 / (1 + np.exp(-ref)))
    np.testing.assert_allclose(act2[1], silu.reshape(-1), atol=1e-12)


def test_net_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    L = (4, 3, 3)
    P = L[0] * L[1] * L[2]
    ch = (10, 4, 4, 4, 3)
    n = oracle.net_nparams(ch)
    params = rng.standard_normal(n) * 0.2
    Sg = random_sphere(P, 1)
    Ss = random_sphere(P, 2)
    x = np.concatenate([Sg, Ss, random_sphere(P, 3), np.full((1, P), 0.4)])
    loss, g = oracle.net_backward(L, params, x, Sg, Ss, ch=ch)
    h = 1e-6
    idx = rng.choice(n, 40, replace=False)
    for k in idx:
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp = oracle.net_predict_loss(oracle.net_forward(L, pp, x, ch=ch), Sg, Ss)[1]
        lm = oracle.net_predict_loss(oracle.net_forward(L, pm, x, ch=ch), Sg, Ss)[1]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, fd, g[k])
    lf = oracle.net_predict_loss(oracle.net_forward(L, params, x, ch=ch), Sg, Ss)[1]
    assert abs(lf - loss) < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_net_dilated_layer_is_correlation_with_spread_kernel(d):
    # a layer dilated by d equals scipy's correlation with the 3^3 kernel
    # spread onto a (2d+1)^3 grid (taps at 0, d, 2d, zeros between), zero
    # padding; the later layers see its SiLU output (checked as above)
    from scipy.ndimage import correlate
    rng = np.random.default_rng(5)
    L = (9, 7, 8)
    ch = (1, 1, 1, 1, 1)
    n = oracle.net_nparams(ch)
    p = np.zeros(n)
    k1 = rng.standard_normal(27)
    p[:27] = k1
    p[27] = -0.5
    x = rng.standard_normal((1, L[0] * L[1] * L[2]))
    _, act = oracle.net_forward(L, p, x, ch=ch, want_act=True, dil=(d, 1, 1, 1))
    big = np.zeros((2 * d + 1,) * 3)
    big[::d, ::d, ::d] = k1.reshape(3, 3, 3)
    ref = correlate(x.reshape(L[2], L[1], L[0]), big, mode="constant", cval=0.0) - 0.5
    np.testing.assert_allclose(act[0], ref.reshape(-1), atol=1e-12)
    # layer 2 dilated too: its pre-activation is the spread correlation of
    # the SiLU of layer 1
    p2 = p.copy()
    k2 = rng.standard_normal(27)
    p2[28:55] = k2
    _, act2 = oracle.net_forward(L, p2, x, ch=ch, want_act=True, dil=(d, d + 1, 1, 1))
    big2 = np.zeros((2 * (d + 1) + 1,) * 3)
    big2[::d + 1, ::d + 1, ::d + 1] = k2.reshape(3, 3, 3)
    silu = ref * (1 / (1 + np.exp(-ref)))
    ref2 = correlate(silu, big2, mode="constant", cval=0.0)
    np.testing.assert_allclose(act2[1], ref2.reshape(-1), atol=1e-12)


def test_net_dilated_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    L = (7, 6, 5)
    P = L[0] * L[1] * L[2]
    ch = (10, 4, 4, 4, 3)
    dil = (2, 1, 3, 1)
    n = oracle.net_nparams(ch)
    params = rng.standard_normal(n) * 0.2
    Sg = random_sphere(P, 7)
    Ss = random_sphere(P, 8)
    x = np.concatenate([Sg, Ss, random_sphere(P, 9), np.full((1, P), 0.6)])
    loss, g = oracle.net_backward(L, params, x, Sg, Ss, ch=ch, dil=dil)
    h = 1e-6
    for k in rng.choice(n, 40, replace=False):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        lp = oracle.net_predict_loss(oracle.net_forward(L, pp, x, ch=ch, dil=dil), Sg, Ss)[1]
        lm = oracle.net_predict_loss(oracle.net_forward(L, pm, x, ch=ch, dil=dil), Sg, Ss)[1]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, fd, g[k])
    # dilation changes the result (the taps are not those of dilation 1)
    l1, _ = oracle.net_backward(L, params, x, Sg, Ss, ch=ch)
    assert abs(l1 - loss) > 1e-6


def _bf16_by_arithmetic(a):
    # float32 first, then the nearest number with 8 significant bits (numpy's
    # round is half-to-even): an arithmetic rounding, not the oracle's bit form
    f = np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    m, e = np.frexp(f)
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def test_net_bf16_operands_are_rounded_to_nearest_even():
    # the quantised oracle mode (the BF16 form's emulated operands): layer 1's
    # pre-activation is the correlation of the rounded input with the rounded
    # kernel, ties included (the input holds exact halfway values)
    from scipy.ndimage import correlate
    rng = np.random.default_rng(8)
    L = (6, 5, 4)
    P = L[0] * L[1] * L[2]
    ch = (1, 1, 1, 1, 1)
    p = np.zeros(oracle.net_nparams(ch))
    k1 = rng.standard_normal(27)
    p[:27] = k1
    p[27] = 0.125
    x = rng.standard_normal((1, P))
    x[0, :8] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -9, 1.5 + 2 ** -8, 2 ** -130, 1e-3, 3.0]
    _, act = oracle.net_forward(L, p, x, ch=ch, want_act=True, bf16=True)
    assert _bf16_by_arithmetic(1 + 2 ** -8) == 1.0 and _bf16_by_arithmetic(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    xr = _bf16_by_arithmetic(x).reshape(L[2], L[1], L[0])
    ref = correlate(xr, _bf16_by_arithmetic(k1).reshape(3, 3, 3), mode="constant", cval=0.0) + 0.125
    np.testing.assert_allclose(act[0], ref.reshape(-1), atol=1e-12)
    # without rounding the result differs
    _, act0 = oracle.net_forward(L, p, x, ch=ch, want_act=True)
    assert np.max(np.abs(act0[0] - act[0])) > 1e-4


def test_net_zero_output_returns_geodesic_guess():
    L = (3, 3, 3)
    P = 27
    Sg = random_sphere(P, 4)
    shat, _ = oracle.net_predict_loss(np.zeros((3, P)), Sg)
    np.testing.assert_array_equal(shat, Sg)


def test_adam_first_step_is_lr_times_sign():
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    oracle.adam(w, g, m, v, 1, lr=0.1)
    np.testing.assert_allclose(w, [0.9, -1.9, 2.9], atol=1e-6)


def test_heun_site_offset_reproduces_a_slab_of_a_larger_lattice():
    # a z-slab of a periodic-in-xy lattice advanced alone (open in z) with the
    # noise counters offset by the slab's first global site equals the full
    # lattice's step on the planes at least two away from the slab faces
    w = Workload(name="t", L=(6, 5, 10), J_shell=(1.0,), K=0.1, alpha=0.1, dt_fs=0.5, T_K=50.0)
    m = oracle_model(w)
    S0 = random_sphere(w.N, 4)
    full = oracle.heun(m, S0, alpha=0.1, dt_fs=0.5, T_K=50.0, seed=1004, step0=3, n_steps=1)
    z0, nz, plane = 3, 6, 6 * 5
    ws = Workload(name="t", L=(6, 5, nz), periodic=(1, 1, 0), J_shell=(1.0,), K=0.1)
    slab = S0[:, z0 * plane:(z0 + nz) * plane]
    got = oracle.heun(oracle_model(ws), slab, alpha=0.1, dt_fs=0.5, T_K=50.0, seed=1004, step0=3, n_steps=1,
                      site0=z0 * plane)
    inner = slice(2 * plane, (nz - 2) * plane)
    np.testing.assert_array_equal(got[:, inner], full[:, (z0 + 2) * plane:(z0 + nz - 2) * plane])
    # without the offset the noise differs
    off = oracle.heun(oracle_model(ws), slab, alpha=0.1, dt_fs=0.5, T_K=50.0, seed=1004, step0=3, n_steps=1)
    assert np.max(np.abs(off[:, inner] - got[:, inner])) > 1e-6


def test_model_rejects_shell_lists_shorter_than_the_shell_count():
    lat = oracle_lattice(Workload(name="t", L=(3, 3, 3)))
    with pytest.raises(ValueError):
        oracle.Model(lat, n_shells=3, J_shell=(1.0, -0.3, 0.1), D_shell=(0.4,))
    with pytest.raises(ValueError):
        oracle.Model(lat, n_shells=2, J_shell=(1.0,))
