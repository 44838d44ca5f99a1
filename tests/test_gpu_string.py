"""GPU parity of the string method (GNEB mode 4) and the geodesic
reparameterisation (spx_gneb_redistribute, spx_gneb_set_spacing) against the
FP64 oracle, and the string -> climbing-image workflow on a macrospin with a
transverse field (Stoner-Wohlfarth barrier K (1 - h/2K)^2).

Tolerances: state after each iteration <= 1e-9 per component (FP64 on both
sides; the distance sums differ only in summation order); energies and
distances 1e-10 relative; reported perpendicular force 1e-9 relative;
redistribution 1e-12 per component; barrier 1e-8 meV.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import gpu_hamiltonian, oracle_model, require_gpu, to_dev
from workloads import Workload, random_sphere

pytestmark = pytest.mark.gpu

MU_B = 5.7883818060e-2  # meV/T


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def frustrated(L, periodic=(0, 0, 0), K=0.05, B=(0.0, 0.0, 0.3)):
    return Workload(name="t", L=L, periodic=periodic, J_shell=(1.0, 0.188, -0.274, -0.161), K=K, B=B,
                    field_prec="fp64")


def bulge(Y, amp):
    """Push every spin of the interior images off its arc along y by amp sin(pi t)."""
    Y = Y.copy()
    M = Y.shape[0]
    for n in range(1, M - 1):
        Y[n, 1] += amp * np.sin(np.pi * n / (M - 1))
        Y[n] /= np.linalg.norm(Y[n], axis=0)
    return Y


def wandering_path(N, M, seed, step=0.25):
    rng = np.random.default_rng(seed)
    Y = np.zeros((M, 3, N))
    Y[0] = random_sphere(N, seed)
    for n in range(1, M):
        s = Y[n - 1] + step * rng.standard_normal((3, N))
        Y[n] = s / np.linalg.norm(s, axis=0)
    return Y


@pytest.mark.parametrize("engine", [0, 1], ids=["zmarch", "gather"])
def test_string_iterations_match_oracle(engine):
    from paper_2605_26016_amd import spx
    w = frustrated((5, 4, 3))
    A, B = random_sphere(w.N, 21), random_sphere(w.N, 22)
    n_img = 7
    Y0 = bulge(oracle.geodesic_path(A, B, n_img), 0.3)
    Yd = to_dev(Y0)
    g = spx.gneb_create([gpu_hamiltonian(w, stencil_engine=engine)], [Yd], vp_dt=0.02, ci_mode=4)
    st = oracle.GnebState(Y0, dt=0.02, ci_mode=4)
    m = oracle_model(w)
    for it in range(10):
        E, dist, fperp, ci = oracle.gneb_iterate(m, st)
        spx.gneb_step(g, 1)
        s = spx.gneb_get_stats(g)
        err = float(np.max(np.abs(Yd.cpu().numpy() - st.Y)))
        assert err <= 1e-9, (it, err)
        np.testing.assert_allclose(s["E"], E, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(s["dist"], dist, rtol=1e-10, atol=1e-12)
        assert abs(s["max_force"] - fperp) <= 1e-9 * max(1.0, fperp)
        assert s["ci_index"] == -1 and s["iterations"] == it + 1


def test_string_graph_replay_ragged_batch_with_spacing_profile():
    import torch
    from paper_2605_26016_amd import spx
    cases = [(frustrated((4, 4, 4), periodic=(1, 1, 1)), 6, 31, None),
             (frustrated((5, 3, 2), K=0.2), 8, 32, np.array([0, 0.05, 0.15, 0.3, 0.5, 0.7, 0.9, 1.0]))]
    hams, bufs, refs = [], [], []
    for w, n_img, seed, alpha in cases:
        Y0 = bulge(oracle.geodesic_path(random_sphere(w.N, seed), random_sphere(w.N, seed + 50), n_img), 0.2)
        hams.append(gpu_hamiltonian(w))
        bufs.append(to_dev(Y0))
        refs.append((oracle_model(w), oracle.GnebState(Y0, dt=0.03, ci_mode=4, alpha=alpha)))
    g = spx.gneb_create(hams, bufs, vp_dt=0.03, ci_mode=4)
    spx.gneb_set_spacing(g, 1, cases[1][3])
    n_it = 9
    spx.gneb_step(g, n_it)                     # one captured graph, replayed
    torch.cuda.synchronize()
    for k, (m, st) in enumerate(refs):
        for _ in range(n_it):
            E, dist, fperp, ci = oracle.gneb_iterate(m, st)
        err = float(np.max(np.abs(bufs[k].cpu().numpy() - st.Y)))
        assert err <= 1e-9, (k, err)
        s = spx.gneb_get_stats(g, k)
        np.testing.assert_allclose(s["E"], E, rtol=1e-10)
        assert s["iterations"] == n_it


def test_redistribute_matches_oracle():
    import torch
    from paper_2605_26016_amd import spx
    w1, w2 = frustrated((4, 3, 3)), frustrated((3, 3, 2))
    Y1, Y2 = wandering_path(w1.N, 8, 41), wandering_path(w2.N, 5, 42, step=0.6)
    d1, d2 = to_dev(Y1), to_dev(Y2)
    g = spx.gneb_create([gpu_hamiltonian(w1), gpu_hamiltonian(w2)], [d1, d2], ci_mode=4)
    alpha = np.array([0.0, 0.08, 0.2, 0.35, 0.5, 0.7, 0.9, 1.0])
    spx.gneb_set_spacing(g, 0, alpha)
    spx.gneb_redistribute(g)
    torch.cuda.synchronize()
    assert np.max(np.abs(d1.cpu().numpy() - oracle.reparametrize(Y1, alpha))) <= 1e-12
    assert np.max(np.abs(d2.cpu().numpy() - oracle.reparametrize(Y2))) <= 1e-12
    # a second redistribution of an already redistributed path moves it only
    # by the chord-versus-arc difference, and keeps the end images
    spx.gneb_redistribute(g)
    torch.cuda.synchronize()
    got = d1.cpu().numpy()
    assert np.array_equal(got[0], Y1[0]) and np.array_equal(got[-1], Y1[-1])


def test_string_then_climbing_image_on_a_transverse_field_macrospin():
    from paper_2605_26016_amd import spx
    K, h = 1.0, 0.6
    w = Workload(name="sw", L=(1, 1, 1), periodic=(0, 0, 0), J_shell=(0.0,), K=K, B=(h / MU_B, 0.0, 0.0),
                 field_prec="fp64")
    th = np.arcsin(h / (2 * K))
    up = np.array([[np.sin(th)], [0.0], [np.cos(th)]])
    dn = np.array([[np.sin(th)], [0.0], [-np.cos(th)]])
    Yd = to_dev(bulge(oracle.geodesic_path(up, dn, 9), 0.4))
    g = spx.gneb_create([gpu_hamiltonian(w)], [Yd], vp_dt=0.1, ci_mode=4, tol_force=1e-7)
    spx.gneb_step(g, 5000)
    s = spx.gneb_get_stats(g)
    assert s["converged"] == 1 and s["iterations"] < 5000
    spx.gneb_set_params(g, spring_k=1.0, vp_dt=0.2, ci_mode=2, tol_force=1e-9)
    assert spx.gneb_get_stats(g)["iterations"] == 0
    spx.gneb_step(g, 20000)
    s = spx.gneb_get_stats(g)
    assert s["converged"] == 1
    ci = s["ci_index"]
    assert abs((s["E"][ci] - s["E"][0]) - K * (1 - h / (2 * K)) ** 2) < 1e-8
    assert np.allclose(Yd.cpu().numpy()[ci, :, 0], [1.0, 0.0, 0.0], atol=1e-7)


def test_spacing_profile_is_validated():
    from paper_2605_26016_amd import spx
    w = frustrated((3, 3, 3))
    Yd = to_dev(oracle.geodesic_path(random_sphere(w.N, 1), random_sphere(w.N, 2), 5))
    g = spx.gneb_create([gpu_hamiltonian(w)], [Yd], ci_mode=4)
    for bad in ([0.1, 0.3, 0.5, 0.7, 1.0], [0.0, 0.3, 0.2, 0.7, 1.0], [0.0, 0.3, 0.5, 0.7, 0.9]):
        with pytest.raises(spx.SpxError):
            spx.gneb_set_spacing(g, 0, np.array(bad))
    with pytest.raises(spx.SpxError):
        spx.gneb_set_spacing(g, 1, np.linspace(0, 1, 5))
    with pytest.raises(spx.SpxError):
        spx.gneb_set_params(g, ci_mode=5)
    with pytest.raises(spx.SpxError):
        spx.gneb_set_params(g, vp_dt=0.0)
