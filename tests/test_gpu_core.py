"""GPU parity of the core path (field, energy, Heun, thermal noise, dipolar)
against the FP64 CPU oracle, through the C ABI of libspx.so.

Tolerances (written per test):
  - FP64 field / energy / deterministic state: rounding-level (1e-12 relative);
  - FP32 field: max|b - b_ref| / max|b_ref| <= 1e-5;
  - one Heun step from identical FP64 state: max |S - S_ref| <= 1e-9 per
    component in mixed mode, 1e-12 in FP64;
  - Philox blocks and the derived uniforms: bit-exact;
  - Gaussian normals: within a few ulp (device vs host libm), checked at 1e-13.
"""
import json

import numpy as np
import pytest

import oracle
from tests.helpers import gpu_hamiltonian, max_rel, oracle_model, require_gpu, to_dev
from workloads import (Workload, bcc_5shell_stochastic, fm_tilt, random_sphere, sc_billion,
                       sc_chiral_dipolar, sc_nn_fp64, uniform_state)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    import torch
    torch.cuda.init()
    print("GPU:", torch.cuda.get_device_name(0), flush=True)


def gpu_field(w, S, prec=None, **kw):
    import torch
    h = gpu_hamiltonian(w, field_prec=prec, **kw)
    dt = torch.float64 if (prec or w.field_prec) == "fp64" else torch.float32
    b = torch.empty((3, w.N), dtype=dt, device="cuda")
    from paper_2605_26016_amd import spx
    spx.eval_field(h, to_dev(S), b)
    torch.cuda.synchronize()
    return b.double().cpu().numpy()


FIELD_CASES = [
    ("sc_nn_fp64_16", sc_nn_fp64((16, 16, 16)), "fp64", 1e-13),
    ("sc_nn_fp64_ragged", sc_nn_fp64((13, 7, 5)), "fp64", 1e-13),
    ("sc_nn_fp32_ragged", sc_nn_fp64((13, 7, 5)), "fp32", 1e-5),
    ("bcc_5shell_fp32", bcc_5shell_stochastic((8, 6, 5)), "fp32", 1e-5),
    ("bcc_5shell_fp64", bcc_5shell_stochastic((7, 5, 6)), "fp64", 1e-13),
    ("bcc_tiny_L1", bcc_5shell_stochastic((1, 1, 1)), "fp64", 1e-13),
    ("bcc_tiny_L2", bcc_5shell_stochastic((2, 3, 2)), "fp32", 1e-5),
    ("sc_dmi_open_fp32", Workload(name="t", L=(9, 8, 7), periodic=(0, 0, 0), J_shell=(1.0,),
                                  D_shell=(0.3,), B=(0.0, 0.0, 0.5), mu=(2.0,)), "fp32", 1e-5),
    ("sc_dmi_mixedbc_fp64", Workload(name="t", L=(9, 8, 7), periodic=(1, 0, 1), J_shell=(1.0, -0.2),
                                     D_shell=(0.3, 0.05), K=0.2, K_axis=(0.6, 0.0, 0.8),
                                     B=(0.1, -0.3, 0.5)), "fp64", 1e-13),
    ("sc_frustrated_open", Workload(name="t", L=(11, 10, 9), periodic=(0, 0, 0),
                                    J_shell=(1.0, 0.188, -0.274, -0.161)), "fp64", 1e-13),
    # several 64 x 8 tiles with ragged x and y tails; tile counts divisible by
    # 8 (XCD-contiguous tile order) at the default z chunk
    ("sc3_fp32_multitile", Workload(name="t", L=(100, 20, 32), periodic=(1, 0, 1),
                                    J_shell=(1.0, -0.3, 0.15), K=0.1, B=(0.2, 0.0, 0.4)), "fp32", 1e-5),
    ("sc3_fp64_multitile", Workload(name="t", L=(100, 20, 32), periodic=(0, 1, 1),
                                    J_shell=(1.0, -0.3, 0.15)), "fp64", 1e-13),
    ("sc4_fp32_multitile", Workload(name="t", L=(70, 9, 16), periodic=(1, 1, 0),
                                    J_shell=(1.0, 0.188, -0.274, -0.161)), "fp32", 1e-5),
    ("bcc_fp32_multitile", bcc_5shell_stochastic((65, 17, 32)), "fp32", 1e-5),
]


# engine: 1 = table-driven gather kernel, 0 = auto (z-march LDS engine when
# the bond table matches a built-in shell shape), plus a small z chunk that
# puts block boundaries inside the lattice
ENGINES = [dict(stencil_engine=1), dict(stencil_engine=0), dict(stencil_engine=0, zchunk=3)]


@pytest.mark.parametrize("eng", ENGINES, ids=["gather", "auto", "auto_z3"])
@pytest.mark.parametrize("name,w,prec,tol", FIELD_CASES, ids=[c[0] for c in FIELD_CASES])
def test_field_parity(name, w, prec, tol, eng):
    S = random_sphere(w.N, 31)
    ref = oracle.field(oracle_model(w), S)
    got = gpu_field(w, S, prec, **eng)
    assert max_rel(got, ref) <= tol, (name, max_rel(got, ref))


def test_zmarch_engine_selected_for_shell_shapes():
    from paper_2605_26016_amd import spx
    for w, prec, shape in ((sc_nn_fp64((8, 8, 8)), "fp64", 0), (bcc_5shell_stochastic((8, 8, 8)), "fp32", 3),
                           (Workload(name="t", L=(8, 8, 8), J_shell=(1.0, 0.2, 0.1)), "fp64", 1),
                           (Workload(name="t", L=(8, 8, 8), J_shell=(1.0, 0.2, 0.1, 0.3)), "fp32", 2),
                           (Workload(name="t", L=(8, 8, 8), J_shell=(1.0,), D_shell=(0.3,)), "fp32", 0)):
        info = spx.get_info(gpu_hamiltonian(w, field_prec=prec))
        assert info.stencil_engine == 2 and info.shape == shape, (w.J_shell, info.shape)
    w = Workload(name="t", L=(8, 8, 8), J_shell=(1.0, 0.2), D_shell=(0.3, 0.1))
    assert spx.get_info(gpu_hamiltonian(w, field_prec="fp32")).stencil_engine == 1
    # an isotropic nearest-neighbour table whose bonds of one shell differ in J
    # is not shell-uniform: it runs on the gather engine, still exactly
    import torch
    deltas = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)], np.int32)
    Jb = np.array([np.eye(3) * v for v in (1.0, 1.0, 0.5, 0.5, 0.8, 0.8)])
    ab = np.zeros((6, 2), np.int32)
    hb = spx.setup_hamiltonian((6, 5, 4), J_shell=None, bonds=(ab, deltas, Jb), field_prec="fp64")
    assert spx.get_info(hb).stencil_engine == 1
    lat = oracle.Lattice((6, 5, 4), np.eye(3), [0, 0, 0])
    mb = oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], deltas, Jb))
    S = random_sphere(lat.N, 8)
    bb = torch.empty((3, lat.N), dtype=torch.float64, device="cuda")
    spx.eval_field(hb, to_dev(S), bb)
    assert max_rel(bb.cpu().numpy(), oracle.field(mb, S)) < 1e-13
    with pytest.raises(spx.SpxError):
        gpu_hamiltonian(w, field_prec="fp32", stencil_engine=2)


def test_bond_table_matches_oracle():
    from paper_2605_26016_amd import spx
    for w in (bcc_5shell_stochastic((4, 4, 4)),
              Workload(name="t", L=(4, 4, 4), J_shell=(1.0, 0.5), D_shell=(0.3, -0.1))):
        h = gpu_hamiltonian(w)
        ab, dl, J = spx.get_bonds(h)
        m = oracle_model(w)
        ref = {(int(a), int(b), *map(int, m.b_delta[3 * p:3 * p + 3])): m.b_J[9 * p:9 * p + 9]
               for p, (a, b) in enumerate(zip(m.b_a, m.b_b))}
        got = {(int(ab[p, 0]), int(ab[p, 1]), *map(int, dl[p])): J[p].reshape(-1) for p in range(len(ab))}
        assert set(ref) == set(got)
        for k in ref:
            np.testing.assert_allclose(got[k], ref[k], atol=1e-15)


def test_explicit_general_tensor_bonds():
    # a full, non-symmetric 3x3 tensor per bond through the explicit bond list
    from paper_2605_26016_amd import spx
    import torch
    rng = np.random.default_rng(5)
    L = (6, 5, 7)
    deltas = [(1, 0, 0), (-1, 0, 0), (0, 2, 0), (0, -2, 0), (1, 1, -1), (-1, -1, 1)]
    Js = rng.standard_normal((3, 3, 3))
    J = [Js[0], Js[0].T, Js[1], Js[1].T, Js[2], Js[2].T]
    ab = np.zeros((6, 2), np.int32)
    h = spx.setup_hamiltonian(L, J_shell=None, bonds=(ab, np.array(deltas), np.array(J)), field_prec="fp64")
    lat = oracle.Lattice(L, np.eye(3), [0, 0, 0])
    m = oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], np.array(deltas), np.array(J)))
    S = random_sphere(lat.N, 3)
    b = torch.empty((3, lat.N), dtype=torch.float64, device="cuda")
    spx.eval_field(h, to_dev(S), b)
    assert max_rel(b.cpu().numpy(), oracle.field(m, S)) < 1e-13


ENERGY_CASES = [
    ("sc_fp64", sc_nn_fp64((12, 10, 9)), "fp64", 1e-12),
    ("bcc_fp32", bcc_5shell_stochastic((8, 8, 8)), "fp32", 1e-6),
    ("dmi_zeeman_open_fp64", Workload(name="t", L=(9, 8, 7), periodic=(0, 0, 0), J_shell=(1.0,),
                                      D_shell=(0.3,), B=(0.0, 0.0, 0.5), mu=(2.0,), K=0.1), "fp64", 1e-12),
]


@pytest.mark.parametrize("engine", [0, 1], ids=["auto", "gather"])
@pytest.mark.parametrize("name,w,prec,tol", ENERGY_CASES, ids=[c[0] for c in ENERGY_CASES])
def test_energy_parity(name, w, prec, tol, engine):
    # auto: the z-march field pass feeds the energy where a shell shape matches
    import torch
    from paper_2605_26016_amd import spx
    S = random_sphere(w.N, 41)
    ref = oracle.energy(oracle_model(w), S)
    h = gpu_hamiltonian(w, field_prec=prec, stencil_engine=engine)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    terms = torch.zeros(5, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S), E, terms)
    t = terms.cpu().numpy()
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(t - ref)) <= tol * scale, (t, ref)
    assert abs(E.item() - ref[4]) <= tol * scale
    # deterministic: bitwise identical on repeat
    E2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S), E2)
    assert E2.item() == E.item()


@pytest.mark.parametrize("L,setup", [((128, 64, 128), dict(stencil_engine=1)), ((97, 101, 103), dict(stencil_engine=1)),
                                     ((256, 128, 64), dict(zchunk=1)), ((197, 81, 61), dict(zchunk=1, field_prec="fp32"))],
                         ids=["gather_even", "gather_odd", "zmarch_4096_tiles", "zmarch_fp32_ragged"])
def test_energy_two_level_reduction(L, setup):
    # more than 8 x 256 partial quadruples (gather kernel: one per 256 sites;
    # z-march energy epilogue: one per 64 x 8 x zchunk tile): the sum goes
    # through the middle level of the fixed-order reduction (several
    # quadruples per middle block, a ragged last chunk for the odd extents)
    import torch
    from paper_2605_26016_amd import spx
    setup = dict(setup)
    prec = setup.pop("field_prec", "fp64")
    w = Workload(name="e2", L=L, J_shell=(1.0, -0.3), D_shell=(0.2, 0.0), K=0.1, K_axis=(0.0, 0.0, 1.0),
                 B=(0.0, 0.5, 2.0), field_prec=prec)
    if "zchunk" in setup:
        # an isotropic table (no DMI) has a z-march shape
        w.D_shell = None
    S = random_sphere(w.N, 43)
    ref = oracle.energy(oracle_model(w), S)
    h = gpu_hamiltonian(w, **setup)
    tol = 1e-12 if prec == "fp64" else 1e-6
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    terms = torch.zeros(5, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S), E, terms)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(terms.cpu().numpy() - ref)) <= tol * scale
    assert abs(E.item() - ref[4]) <= tol * scale
    E2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S), E2)
    assert E2.item() == E.item()


def gpu_heun(w, S, prec, setup=None, **kw):
    import torch
    from paper_2605_26016_amd import spx
    h = gpu_hamiltonian(w, field_prec=prec, **(setup or {}))
    St = to_dev(S)
    spx.llg_heun_step(h, St, **kw)
    torch.cuda.synchronize()
    return St.cpu().numpy()


HEUN_CASES = [
    ("sc_det_fp64_1", sc_nn_fp64((10, 9, 8)), "fp64", dict(n_steps=1), 1e-12),
    ("sc_det_fp64_5", sc_nn_fp64((10, 9, 8)), "fp64", dict(n_steps=5), 1e-12),
    ("sc_det_fp32_1", sc_nn_fp64((10, 9, 8)), "fp32", dict(n_steps=1), 1e-9),
    ("bcc_stoch_fp32_1", bcc_5shell_stochastic((6, 5, 4)), "fp32", dict(n_steps=1), 1e-9),
    ("bcc_stoch_fp64_3", bcc_5shell_stochastic((6, 5, 4)), "fp64", dict(n_steps=3), 1e-12),
    ("sc_stoch_fp32_1", sc_billion((12, 11, 10)), "fp32", dict(n_steps=1), 1e-9),
    ("bcc_stoch_fp32_multitile", bcc_5shell_stochastic((65, 17, 16)), "fp32", dict(n_steps=2), 1e-9),
    ("sc3_stoch_fp32_multitile", Workload(name="t", L=(100, 20, 16), periodic=(1, 0, 1),
                                          J_shell=(1.0, -0.3, 0.15), K=0.1, B=(0.2, 0.0, 0.4), T_K=300.0,
                                          alpha=0.1, dt_fs=0.5, philox_seed=9), "fp32", dict(n_steps=2), 1e-9),
    ("dmi_zeeman_open_fp64", Workload(name="t", L=(7, 6, 5), periodic=(0, 0, 0), J_shell=(1.0,),
                                      D_shell=(0.3,), B=(0.0, 0.0, 0.5), mu=(2.0,), K=0.1, alpha=0.3,
                                      dt_fs=1.0, T_K=10.0, philox_seed=77), "fp64", dict(n_steps=2), 1e-12),
]


HEUN_SETUPS = [dict(stencil_engine=1), dict(stencil_engine=0, heun_field=1),
               dict(stencil_engine=0, heun_field=3), dict(stencil_engine=0, heun_field=4),
               dict(stencil_engine=0, heun_field=7), dict(stencil_engine=0, heun_field=0, zchunk=3)]


@pytest.mark.parametrize("setup", HEUN_SETUPS, ids=["gather", "zmarch_recompute", "zmarch_stage",
                                                     "zmarch_noisepass", "zmarch_stage_redraw", "auto_z3"])
@pytest.mark.parametrize("name,w,prec,extra,tol", HEUN_CASES, ids=[c[0] for c in HEUN_CASES])
def test_heun_parity(name, w, prec, extra, tol, setup):
    S = w.initial_state() if w.init != "random" else random_sphere(w.N, 51)
    n = extra["n_steps"]
    ref = oracle.heun(oracle_model(w), S, alpha=w.alpha, dt_fs=w.dt_fs, T_K=w.T_K, seed=w.philox_seed,
                      step0=17, n_steps=n)
    got = gpu_heun(w, S, prec, setup=setup, alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K,
                   seed=w.philox_seed, step0=17, n_steps=n)
    err = np.max(np.abs(got - ref))
    assert err <= tol * n, (name, err)
    assert np.max(np.abs(np.sqrt((got * got).sum(0)) - 1.0)) < 1e-14


def test_heun_stored_field_equals_recompute():
    # the stored FP32 field of S^n is bit-identical to recomputing it
    w = bcc_5shell_stochastic((10, 9, 7))
    S = w.initial_state()
    kw = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed, step0=0, n_steps=3)
    a = gpu_heun(w, S, "fp32", setup=dict(heun_field=1), **kw)
    b = gpu_heun(w, S, "fp32", setup=dict(heun_field=2), **kw)
    assert np.array_equal(a, b)
    # the stored stage regroups S + dt/2 f0 + dt/2 f1: equal up to rounding
    c = gpu_heun(w, S, "fp32", setup=dict(heun_field=3), **kw)
    assert np.max(np.abs(a - c)) <= 1e-14
    # the noise pre-pass draws the same numbers
    d = gpu_heun(w, S, "fp32", setup=dict(heun_field=4), **kw)
    assert np.array_equal(c, d)
    # the split mode (stencil pass + elementwise stages) computes the same
    e = gpu_heun(w, S, "fp32", setup=dict(heun_field=5), **kw)
    assert np.array_equal(c, e)
    f = gpu_heun(w, S, "fp32", setup=dict(heun_field=6), **kw)
    assert np.array_equal(c, f)
    # the corrector that draws the noise again gets the same numbers
    g = gpu_heun(w, S, "fp32", setup=dict(heun_field=7), **kw)
    assert np.array_equal(c, g)
    # deterministic case (no noise store)
    kw["temperature_K"] = 0.0
    a = gpu_heun(w, S, "fp32", setup=dict(heun_field=1), **kw)
    c = gpu_heun(w, S, "fp32", setup=dict(heun_field=3), **kw)
    assert np.max(np.abs(a - c)) <= 1e-14
    e = gpu_heun(w, S, "fp32", setup=dict(heun_field=5), **kw)
    assert np.array_equal(c, e)
    f = gpu_heun(w, S, "fp32", setup=dict(heun_field=6), **kw)
    assert np.array_equal(c, f)
    g = gpu_heun(w, S, "fp32", setup=dict(heun_field=7), **kw)
    assert np.array_equal(c, g)


@pytest.mark.parametrize("mode", [1, 2, 3, 4, 5, 6, 7])
def test_autotuner_reads_every_mode_from_its_cache(tmp_path, mode):
    # a cached choice of any Heun mode is taken as is, without tuning again
    from paper_2605_26016_amd import spx
    w = bcc_5shell_stochastic((16, 16, 16))
    cache = tmp_path / "tune.txt"
    cache.write_text(f"shape3_prec1_sub2_16x16x16_per111 8 {mode} 123.5\n")
    info = spx.get_info(gpu_hamiltonian(w, field_prec="fp32", autotune=1, tune_cache_path=str(cache)))
    assert (info.tuned, info.zchunk, info.heun_field, info.tuned_step_us) == (1, 8, mode, 123.5)
    assert cache.read_text().count("\n") == 1


def test_heun_resume_and_determinism():
    w = bcc_5shell_stochastic((6, 6, 4))
    S = w.initial_state()
    kw = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed)
    a = gpu_heun(w, S, "fp32", step0=0, n_steps=6, **kw)
    b = gpu_heun(w, S, "fp32", step0=0, n_steps=6, **kw)
    assert np.array_equal(a, b)
    c = gpu_heun(w, S, "fp32", step0=0, n_steps=3, **kw)
    c = gpu_heun(w, c, "fp32", step0=3, n_steps=3, **kw)
    assert np.array_equal(a, c)


def test_heun_zero_steps_and_analytic_single_spin():
    # single spin in B = 1 T along z: zero steps is a no-op, many steps follow
    # the analytic precession (Methods, single-spin validation)
    import math
    w = Workload(name="t", L=(1, 1, 1), J_shell=(0.0,), B=(0, 0, 1.0), alpha=0.01, dt_fs=10.0)
    S = np.array([[1.0], [0.0], [0.0]])
    assert np.array_equal(gpu_heun(w, S, "fp64", alpha=0.01, dt_fs=10.0, n_steps=0), S)
    got = gpu_heun(w, S, "fp64", alpha=0.01, dt_fs=10.0, n_steps=1000)
    ref = oracle.heun(oracle_model(w), S, alpha=0.01, dt_fs=10.0, n_steps=1000)
    assert np.max(np.abs(got - ref)) < 1e-12
    g = oracle.constants()[2] / (1 + 0.01 ** 2)
    t = 10000.0
    th = 2 * math.atan(math.exp(-0.01 * g * t))
    ana = np.array([math.cos(g * t) * math.sin(th), math.sin(g * t) * math.sin(th), math.cos(th)])
    assert np.max(np.abs(got[:, 0] - ana)) < 1e-5


def test_philox_blocks_bit_exact():
    import torch
    from paper_2605_26016_amd import spx
    rng = np.random.default_rng(3)
    n = 5000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    out = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    spx.philox4x32_10(to_dev(ctr.view(np.int32)), to_dev(key.view(np.int32)), n, out)
    got = out.cpu().numpy().view(np.uint32)
    for k in range(0, n, 7):
        assert np.array_equal(got[k], oracle.philox(ctr[k], key[k])), k


def test_thermal_noise_matches_oracle():
    import torch
    from paper_2605_26016_amd import spx
    N = 70001
    for seed, step, tag in ((1002, 0, 0), (2 ** 40 + 5, 2 ** 33 + 1, 3)):
        eta = torch.zeros((3, N), dtype=torch.float64, device="cuda")
        spx.thermal_noise(seed, step, tag, N, eta)
        got = eta.cpu().numpy()
        ref = oracle.thermal_eta(seed, step, N, tag=tag)
        assert np.max(np.abs(got - ref)) < 1e-13


# ---------------------------------------------------------------- dipolar
def dip_workload(L):
    w = sc_chiral_dipolar(L)
    return w


# x extents 200 and 130 pad to 512: the x rows run as pairs of real rows in
# one complex transform (45 rows in the first case, so one row is unpaired),
# the last case with the fused z pass as well
@pytest.mark.parametrize("L", [(5, 4, 6), (8, 8, 8), (1, 3, 2), (7, 1, 9), (4, 256, 3), (3, 4, 200), (200, 3, 5),
                               (130, 2, 140)])
def test_dipolar_field_vs_direct_sum(L):
    from paper_2605_26016_amd import spx  # noqa: F401
    w = dip_workload(L)
    S = random_sphere(w.N, 61)
    m = oracle_model(w)
    ref = oracle.field(m, S)  # includes the direct O(N^2) dipolar sum
    got = gpu_field(w, S, "fp32")
    assert max_rel(got, ref) <= 1e-5
    # the dipolar part alone, relative to its own scale
    w0 = dip_workload(L)
    w0.dipolar = 0
    got0 = gpu_field(w0, S, "fp32")
    _, parts = oracle.field(m, S, terms=True)
    assert max_rel(got - got0, parts["dip"]) <= 2e-5


@pytest.mark.parametrize("cell", [((0.4, 0.0, 0.0), (0.0, 0.4, 0.0), (0.0, 0.0, 0.5)),
                                  ((0.4, 0.0, 0.0), (0.1, 0.4, 0.0), (0.05, 0.08, 0.4))],
                         ids=["orthorhombic", "triclinic"])
def test_dipolar_fused_z_pass_both_cell_kinds(cell):
    # Lz = 150 pads to 512 in z: the fused z pass; an orthorhombic cell lets
    # it read half the spectrum (even / odd in kz), a triclinic one does not
    import dataclasses
    w = dataclasses.replace(dip_workload((3, 4, 150)), cell=cell)
    S = random_sphere(w.N, 62)
    m = oracle_model(w)
    ref = oracle.field(m, S)
    got = gpu_field(w, S, "fp32")
    assert max_rel(got, ref) <= 1e-5
    w0 = dataclasses.replace(w, dipolar=0)
    _, parts = oracle.field(m, S, terms=True)
    assert max_rel(got - gpu_field(w0, S, "fp32"), parts["dip"]) <= 2e-5


def test_dipolar_field_vs_numpy_fft_32():
    from oracle.dipolar_fft import dipolar_field_fft
    L = (32, 24, 20)
    w = dip_workload(L)
    w.J_shell = (0.0,)
    w.D_shell = None
    w.B = (0.0, 0.0, 0.0)
    S = random_sphere(w.N, 62)
    ref = dipolar_field_fft(L, w.cell, 2.0, S)
    got = gpu_field(w, S, "fp32")
    assert max_rel(got, ref) <= 1e-5


def test_heun_graph_replay_is_bit_identical():
    # captured graphs (2 steps, or 16 steps and direct launches for the rest)
    # with a device step counter == direct launches
    from paper_2605_26016_amd import spx
    import torch
    w = bcc_5shell_stochastic((10, 9, 8))
    S0 = w.initial_state()
    kw = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed)
    for n in (10, 11, 37):
        ha = gpu_hamiltonian(w, field_prec="fp32")
        hb = gpu_hamiltonian(w, field_prec="fp32")
        spx.set_heun_graph(hb, False)
        Sa, Sb = to_dev(S0), to_dev(S0)
        spx.llg_heun_step(ha, Sa, step0=5, n_steps=n, **kw)
        spx.llg_heun_step(ha, Sa, step0=5 + n, n_steps=n, **kw)   # graph reused, counter reset
        spx.llg_heun_step(hb, Sb, step0=5, n_steps=2 * n, **kw)
        torch.cuda.synchronize()
        assert spx.get_info(ha).heun_graph == 1 and spx.get_info(hb).heun_graph == 0
        assert torch.equal(Sa, Sb), n


def test_autotuner_picks_candidate_and_caches(tmp_path):
    from paper_2605_26016_amd import spx
    import torch
    w = bcc_5shell_stochastic((16, 16, 16))
    cache = str(tmp_path / "tune.txt")
    h = gpu_hamiltonian(w, field_prec="fp32", autotune=1, tune_cache_path=cache)
    info = spx.get_info(h)
    assert info.tuned == 1 and info.zchunk in (4, 8, 16) and info.heun_field in (1, 2, 3, 4, 5, 6, 7)
    assert info.tuned_step_us > 0
    # one JSON object per line
    entries = [json.loads(l) for l in open(cache) if l.strip()]
    assert [e["key"] for e in entries] == ["shape3_prec1_sub2_16x16x16_per111"]
    assert (entries[0]["zchunk"], entries[0]["heun_mode"]) == (info.zchunk, info.heun_field)
    h2 = gpu_hamiltonian(w, field_prec="fp32", autotune=1, tune_cache_path=cache)
    i2 = spx.get_info(h2)
    assert (i2.zchunk, i2.heun_field) == (info.zchunk, info.heun_field)
    # the second setup read the cache instead of tuning again
    assert sum(1 for l in open(cache) if l.strip()) == 1
    assert i2.tuned == 1 and i2.tuned_step_us == pytest.approx(info.tuned_step_us, abs=1e-3)
    # the z chunk does not change results (same Heun mode, other launch shape)
    S0 = w.initial_state()
    h3 = gpu_hamiltonian(w, field_prec="fp32", zchunk=3, heun_field=info.heun_field)
    kw = dict(alpha=w.alpha, dt_fs=w.dt_fs, temperature_K=w.T_K, seed=w.philox_seed, step0=0, n_steps=4)
    Sa, Sb = to_dev(S0), to_dev(S0)
    spx.llg_heun_step(h, Sa, **kw)
    spx.llg_heun_step(h3, Sb, **kw)
    torch.cuda.synchronize()
    assert torch.equal(Sa, Sb)
