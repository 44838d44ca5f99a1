"""Pins of the oracle's string method and geodesic reparameterisation
(Methods, minimum-energy paths), checked against closed forms:

  - a geodesic path whose images sit at uneven t, reparameterised to equal
    spacing, is the geodesic path at equal t (the arc length of a geodesic
    path is linear in t), and to a spacing profile alpha it is the geodesic
    path at t = alpha;
  - on an arbitrary path every new image is a great-circle interpolation, at
    one common fraction f, of two consecutive old images, found by brute
    force, and sits at the requested arc length;
  - string relaxation followed by climbing-image GNEB finds the
    Stoner-Wohlfarth barrier of a macrospin with easy axis z and a transverse
    field h along x, K (1 - h/2K)^2, on the channel through +x; started on
    the long arc through -x, the path stays in the xz plane and climbs to the
    stationary point (-1, 0, 0): K (1 + h/2K)^2;
  - a periodic ferromagnet started on uniform states rotates coherently: the
    barrier is N times the macrospin's.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import oracle_model
from workloads import Workload, random_sphere

MU_B = 5.7883818060e-2  # meV/T


def macrospin_model(K=1.0, h=0.6, L=(1, 1, 1), J=0.0, periodic=(0, 0, 0)):
    w = Workload(name="sw", L=L, periodic=periodic, J_shell=(J,), K=K, K_axis=(0.0, 0.0, 1.0),
                 B=(h / MU_B, 0.0, 0.0))
    return w, oracle_model(w)


def sw_minima(K, h, N):
    th = np.arcsin(h / (2 * K))
    up = np.tile(np.array([[np.sin(th)], [0.0], [np.cos(th)]]), (1, N))
    dn = np.tile(np.array([[np.sin(th)], [0.0], [-np.cos(th)]]), (1, N))
    return th, up, dn


def bulge(Y, amp):
    """Push the interior images off their arc along y by amp sin(pi t)."""
    Y = Y.copy()
    M = Y.shape[0]
    for n in range(1, M - 1):
        Y[n, 1] += amp * np.sin(np.pi * n / (M - 1))
        Y[n] /= np.linalg.norm(Y[n], axis=0)
    return Y


def relax_string_then_ci(m, Y0, string_iters=5000, dt=0.1, string_tol=1e-7, ci_tol=1e-9, max_ci=20000):
    st = oracle.GnebState(Y0, k_spring=1.0, dt=dt, mass=1.0, ci_mode=4)
    fperp = []
    for _ in range(string_iters):
        E, dist, f, ci = oracle.gneb_iterate(m, st)
        fperp.append(f)
        if f < string_tol:
            break
    st.ci_mode, st.dt = 2, 0.1
    st.V[:] = 0.0
    for it in range(max_ci):
        E, dist, f, ci = oracle.gneb_iterate(m, st)
        if f < ci_tol:
            break
    E, dist, f, ci = oracle.gneb_iterate(m, st)
    return st, E, ci, fperp


def test_reparametrize_uneven_geodesic_path_gives_even_geodesic_path():
    N, M = 40, 7
    A, B = random_sphere(N, 3), random_sphere(N, 4)
    fine = oracle.geodesic_path(A, B, 4 * (M - 1) + 1)      # t = j / 24
    pick = [0, 1, 2, 3, 7, 12, 13, 20, 24]                   # uneven t, 9 images
    Y = fine[pick]
    even = oracle.reparametrize(Y, alpha=np.linspace(0.0, 1.0, len(pick)))
    ref = oracle.geodesic_path(A, B, len(pick))
    assert np.max(np.abs(even - ref)) < 1e-12
    # default spacing is the equal one
    assert np.max(np.abs(oracle.reparametrize(Y) - ref)) < 1e-12


def test_reparametrize_to_a_spacing_profile():
    N = 25
    A, B = random_sphere(N, 5), random_sphere(N, 6)
    Y = oracle.geodesic_path(A, B, 6)
    alpha = np.array([0.0, 0.05, 0.1, 0.3, 0.6, 1.0])
    out = oracle.reparametrize(Y, alpha)
    fine = oracle.geodesic_path(A, B, 21)                    # t = j / 20
    ref = fine[[0, 1, 2, 6, 12, 20]]
    assert np.max(np.abs(out - ref)) < 1e-12


def _angle(a, b):
    c = np.cross(a.T, b.T)
    return np.arctan2(np.linalg.norm(c, axis=1), np.sum(a * b, axis=0))


def test_reparametrize_arbitrary_path_by_brute_force():
    N, M = 30, 8
    rng = np.random.default_rng(9)
    A = random_sphere(N, 11)
    Y = np.zeros((M, 3, N))
    Y[0] = A
    for n in range(1, M):                                     # a wandering path of small steps
        step = Y[n - 1] + 0.25 * rng.standard_normal((3, N))
        Y[n] = step / np.linalg.norm(step, axis=0)
    alpha = np.array([0.0, 0.08, 0.2, 0.35, 0.5, 0.7, 0.9, 1.0])
    out = oracle.reparametrize(Y, alpha)
    assert np.array_equal(out[0], Y[0]) and np.array_equal(out[-1], Y[-1])
    d = np.array([np.sqrt(np.sum(_angle(Y[n], Y[n + 1]) ** 2)) for n in range(M - 1)])
    s = np.concatenate([[0.0], np.cumsum(d)])
    for n in range(1, M - 1):
        p = out[n]
        found = False
        for k in range(M - 1):
            a, b = Y[k], Y[k + 1]
            ab, ap, pb = _angle(a, b), _angle(a, p), _angle(p, b)
            if np.max(np.abs(ap + pb - ab)) > 1e-10:
                continue                                      # not on these arcs
            f = ap / np.where(ab > 0, ab, 1.0)
            if np.ptp(f[ab > 1e-6]) > 1e-9:
                continue                                      # not one common fraction
            f0 = float(np.median(f[ab > 1e-6]))
            assert abs(s[k] + f0 * d[k] - alpha[n] * s[-1]) < 1e-9
            found = True
            break
        assert found, n


@pytest.mark.parametrize("K,h", [(1.0, 0.6), (0.5, 0.2)])
def test_string_then_climbing_image_finds_the_stoner_wohlfarth_barrier(K, h):
    w, m = macrospin_model(K, h)
    th, up, dn = sw_minima(K, h, 1)
    Y0 = bulge(oracle.geodesic_path(up, dn, 9), 0.4)         # short arc through +x, pushed out of plane
    st, E, ci, fperp = relax_string_then_ci(m, Y0)
    assert fperp[-1] < 1e-6 < fperp[0]
    barrier = E[ci] - E[0]
    assert abs(barrier - K * (1 - h / (2 * K)) ** 2) < 1e-8
    S_ci = st.Y[ci][:, 0]
    assert np.allclose(S_ci, [1.0, 0.0, 0.0], atol=1e-7)     # the saddle sits on the equator at +x
    assert abs(E[0] - (-K - h * h / (4 * K))) < 1e-12


def test_string_on_the_long_arc_stays_in_plane_and_climbs_to_minus_x():
    K, h = 1.0, 0.6
    w, m = macrospin_model(K, h)
    th = np.arcsin(h / (2 * K))
    u = np.linspace(0.0, 1.0, 11)
    theta = th - u * (np.pi + 2 * th)                         # over the north pole, through -x
    Y0 = np.stack([np.stack([np.sin(theta), np.zeros_like(theta), np.cos(theta)])[:, n:n + 1]
                   for n in range(len(u))])
    st, E, ci, fperp = relax_string_then_ci(m, Y0)
    assert np.all(st.Y[:, 1, :] == 0.0)                       # y stays exactly zero
    assert abs((E[ci] - E[0]) - K * (1 + h / (2 * K)) ** 2) < 1e-8
    assert np.allclose(st.Y[ci][:, 0], [-1.0, 0.0, 0.0], atol=1e-7)


def test_coherent_rotation_of_a_periodic_ferromagnet():
    K, h, L = 0.8, 0.5, (3, 3, 3)
    w, m = macrospin_model(K, h, L=L, J=1.0, periodic=(1, 1, 1))
    N = w.N
    th, up, dn = sw_minima(K, h, N)
    Y0 = oracle.geodesic_path(up, dn, 7)
    Y0 = np.stack([bulge(Y0[:, :, i:i + 1], 0.3)[:, :, 0] for i in range(N)], axis=-1)  # same bulge everywhere
    st, E, ci, fperp = relax_string_then_ci(m, Y0)
    assert fperp[-1] < 1e-7 < fperp[0]
    assert abs((E[ci] - E[0]) - N * K * (1 - h / (2 * K)) ** 2) < 1e-7 * N
    # every image stays uniform
    assert np.max(np.abs(st.Y - st.Y[:, :, :1])) < 1e-10
