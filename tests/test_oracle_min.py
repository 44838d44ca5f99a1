"""Pins of the oracle's static minimisers (Methods, static optimisation):
velocity projection, Barzilai-Borwein, L-BFGS and Adam, each with the
exponential-map and the normalised retraction.

  - a free spin in a field turns to the field (E = -|b|, F = 0);
  - a periodic ferromagnet with anisotropy and a strong field along z, from
    random spins, reaches the uniform state, E = -N (3 J + K + h) (six
    neighbours, each bond counted once);
  - at the minimum an iteration changes nothing;
  - first steps in closed form: velocity projection from rest rotates a spin
    perpendicular to its field by |u| = dt^2 |F| / m under the exponential map
    and by atan |u| under the normalised retraction; a step longer than
    max_step is cut to max_step; Adam's first step has |u| = dt (to eps).
"""
import numpy as np
import pytest

import oracle
from tests.helpers import oracle_model
from workloads import Workload, random_sphere

MU_B = 5.7883818060e-2
METHODS = ["vp", "bb", "lbfgs", "adam"]
RETRACTIONS = ["exp", "norm"]
SETTINGS = {"vp": dict(dt=0.2), "bb": dict(dt=0.05), "lbfgs": dict(dt=0.05, hist=5), "adam": dict(dt=0.05)}


def free_spin(h=2.0, axis=(0.0, 0.0, 1.0)):
    w = Workload(name="s", L=(1, 1, 1), periodic=(0, 0, 0), J_shell=(0.0,), B=tuple(np.asarray(axis) * h / MU_B))
    return w, oracle_model(w)


def angle(a, b):
    return float(np.arctan2(np.linalg.norm(np.cross(a, b)), np.dot(a, b)))


def run(m, S, st, n, tol):
    for it in range(n):
        f = oracle.min_iterate(m, S, st)
        if f < tol:
            return it, f
    return n, f


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("retraction", RETRACTIONS)
def test_free_spin_turns_to_its_field(method, retraction):
    h = 2.0
    axis = np.array([0.3, -0.4, 0.866])
    axis /= np.linalg.norm(axis)
    w, m = free_spin(h, axis)
    S = np.array([[0.6], [0.8], [0.0]])
    st = oracle.MinState(1, method, retraction, max_step=0.5, **SETTINGS[method])
    it, f = run(m, S, st, 4000, 1e-10)
    assert f < 1e-10, (it, f)
    assert np.allclose(S[:, 0], axis, atol=1e-10)
    E = oracle.energy(m, S)[4]
    assert abs(E - (-h)) < 1e-12


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("retraction", RETRACTIONS)
def test_ferromagnet_reaches_the_uniform_ground_state(method, retraction):
    J, K, h = 1.0, 0.2, 6.0
    w = Workload(name="fm", L=(3, 3, 3), J_shell=(J,), K=K, B=(0.0, 0.0, h / MU_B))
    m = oracle_model(w)
    S = random_sphere(w.N, 9)
    st = oracle.MinState(w.N, method, retraction, max_step=0.3, **SETTINGS[method])
    it, f = run(m, S, st, 6000, 1e-9)
    assert f < 1e-9, (it, f)
    assert np.max(np.abs(S[2] - 1.0)) < 1e-9
    E = oracle.energy(m, S)[4]
    assert abs(E - (-w.N * (3 * J + K + h))) < 1e-9


@pytest.mark.parametrize("method", METHODS)
def test_an_iteration_at_the_minimum_changes_nothing(method):
    J, K, h = 1.0, 0.2, 3.0
    w = Workload(name="fm", L=(3, 3, 2), J_shell=(J,), K=K, B=(0.0, 0.0, h / MU_B))
    m = oracle_model(w)
    S = np.zeros((3, w.N))
    S[2] = 1.0
    st = oracle.MinState(w.N, method, "exp", **SETTINGS[method])
    for _ in range(3):
        f = oracle.min_iterate(m, S, st)
        assert f < 1e-14
    assert np.array_equal(S[2], np.ones(w.N)) and not S[:2].any()


@pytest.mark.parametrize("retraction,expect", [("exp", lambda u: u), ("norm", np.arctan)])
def test_first_velocity_projection_step(retraction, expect):
    h, dt, mass = 1.5, 0.4, 2.0
    w, m = free_spin(h, (0.0, 0.0, 1.0))
    S = np.array([[1.0], [0.0], [0.0]])
    S0 = S[:, 0].copy()
    st = oracle.MinState(1, "vp", retraction, dt=dt, mass=mass)
    oracle.min_iterate(m, S, st)
    u = dt * dt / mass * h
    assert abs(angle(S0, S[:, 0]) - expect(u)) < 1e-14
    assert abs(S[1, 0]) == 0.0 and S[2, 0] > 0          # turned towards +z in the xz plane


def test_max_step_cuts_a_long_step():
    w, m = free_spin(5.0, (0.0, 0.0, 1.0))
    S = np.array([[1.0], [0.0], [0.0]])
    st = oracle.MinState(1, "vp", "exp", dt=3.0, mass=1.0, max_step=0.25)
    oracle.min_iterate(m, S, st)
    assert abs(angle(np.array([1.0, 0.0, 0.0]), S[:, 0]) - 0.25) < 1e-14


def test_first_adam_step_has_length_dt():
    w, m = free_spin(1.0, (0.0, 0.0, 1.0))
    S = np.array([[1.0], [0.0], [0.0]])
    st = oracle.MinState(1, "adam", "exp", dt=0.1, eps=1e-12)
    oracle.min_iterate(m, S, st)
    assert abs(angle(np.array([1.0, 0.0, 0.0]), S[:, 0]) - 0.1) < 1e-11
