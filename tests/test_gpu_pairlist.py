"""GPU pair-list Hamiltonian (spx_setup_pairlist) against the FP64 oracle,
and against the library's own lattice engines for a lattice written out as a
pair list.

Tolerances: FP64 field 1e-12 relative (list-order sums on both sides); FP32
field max-rel 1e-5; energy terms 1e-12 relative; stochastic Heun after 4
steps 1e-11 (FP64) and 1e-8 (FP32 field, FP64 state).
"""
import numpy as np
import pytest

import oracle
from tests.helpers import gpu_hamiltonian, max_rel, oracle_model, require_gpu, to_dev
from tests.test_oracle_pairlist import disordered, empty_list, lattice_to_pairlist
from workloads import Workload, bcc_5shell_stochastic, random_sphere

pytestmark = pytest.mark.gpu

MU_B = 5.7883818060e-2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def gpu_pl(pl, prec="fp64"):
    from paper_2605_26016_amd import spx
    J = pl.J.reshape(len(pl.i), 3, 3) if pl.tensor else pl.J
    return spx.setup_pairlist(pl.N, pl.i, pl.j, J, mu=pl.mu, K=pl.K, K_axis=pl.K_axis, B=pl.B, field_prec=prec)


def field(h, S, prec):
    import torch
    from paper_2605_26016_amd import spx
    b = torch.empty((3, S.shape[1]), dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
    spx.eval_field(h, to_dev(S), b)
    return b.double().cpu().numpy()


LATTICES = {"sc3shell_dmi": Workload(name="sc", L=(9, 7, 6), periodic=(1, 0, 1), J_shell=(1.0, -0.3, 0.1),
                                     D_shell=(0.4, 0.0, 0.0), K=0.2, K_axis=(0.0, 0.6, 0.8), B=(1.0, -2.0, 0.5),
                                     field_prec="fp64"),
            "bcc5shell": bcc_5shell_stochastic((5, 4, 6))}


@pytest.mark.parametrize("name", list(LATTICES))
def test_lattice_as_pairlist(name):
    w = LATTICES[name]
    pl = lattice_to_pairlist(w)
    S = random_sphere(w.N, 12)
    ref = oracle.pl_field(pl, S)
    got = field(gpu_pl(pl), S, "fp64")
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the library's own lattice engine on the same model
    lat = field(gpu_hamiltonian(w, field_prec="fp64"), S, "fp64")
    assert np.max(np.abs(got - lat)) <= 1e-12 * np.max(np.abs(ref))
    assert max_rel(field(gpu_pl(pl, "fp32"), S, "fp32"), ref) <= 1e-5


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_disordered_field_and_energy(prec, tol):
    import torch
    from paper_2605_26016_amd import spx
    pl, _ = disordered(N=3001, P=20000, seed=4)
    S = random_sphere(pl.N, 13)
    h = gpu_pl(pl, prec)
    assert max_rel(field(h, S, prec), oracle.pl_field(pl, S)) <= tol
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    T = torch.zeros(5, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S), E, T)
    ref = oracle.pl_energy(pl, S)
    np.testing.assert_allclose(T.cpu().numpy(), ref, rtol=max(tol, 1e-12), atol=1e-9)
    assert abs(float(E.item()) - ref[4]) <= max(tol, 1e-12) * abs(ref[4]) + 1e-9


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-8)])
def test_stochastic_heun_matches_the_oracle(prec, tol):
    from paper_2605_26016_amd import spx
    pl, _ = disordered(N=2500, P=9000, seed=6)
    S0 = random_sphere(pl.N, 14)
    S = to_dev(S0)
    kw = dict(alpha=0.05, dt_fs=0.1, seed=11, step0=2, n_steps=4)
    spx.llg_heun_step(gpu_pl(pl, prec), S, temperature_K=200.0, **kw)
    ref = oracle.pl_heun(pl, S0, T_K=200.0, **kw)
    assert float(np.max(np.abs(S.cpu().numpy() - ref))) <= tol


@pytest.mark.parametrize("kind", ["empty", "isolated_sites"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_empty_list_and_sites_without_couplings(kind, prec, tol):
    # an empty list leaves only the on-site terms; in the second list the
    # couplings name only the first half of the sites, so the rest see
    # on-site fields only
    import torch
    from paper_2605_26016_amd import spx
    if kind == "empty":
        pl = empty_list(N=301)
    else:
        pl0, _ = disordered(N=600, P=2000, seed=5)
        keep = (pl0.i < 300) & (pl0.j < 300)
        pl = oracle.PairList(pl0.N, pl0.i[keep], pl0.j[keep], pl0.J[keep].reshape(-1, 3, 3), mu=pl0.mu, K=pl0.K,
                             K_axis=pl0.K_axis, B=pl0.B)
    S0 = random_sphere(pl.N, 21)
    assert max_rel(field(gpu_pl(pl, prec), S0, prec), oracle.pl_field(pl, S0)) <= tol
    h = gpu_pl(pl, prec)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    T = torch.zeros(5, dtype=torch.float64, device="cuda")
    spx.energy(h, to_dev(S0), E, T)
    np.testing.assert_allclose(T.cpu().numpy(), oracle.pl_energy(pl, S0), rtol=max(tol, 1e-12), atol=1e-9)
    S = to_dev(S0)
    kw = dict(alpha=0.05, dt_fs=0.1, seed=3, step0=0, n_steps=3)
    spx.llg_heun_step(h, S, temperature_K=100.0, **kw)
    ref = oracle.pl_heun(pl, S0, T_K=100.0, **kw)
    assert float(np.max(np.abs(S.cpu().numpy() - ref))) <= (1e-11 if prec == "fp64" else 1e-8)


def test_minimiser_on_a_pairlist_reaches_the_ground_state():
    # a disordered ferromagnet (positive couplings, reciprocal entries) in a
    # strong field along z: the ground state is uniform along z
    from paper_2605_26016_amd import spx
    rng = np.random.default_rng(2)
    N, P = 500, 2000
    i = rng.integers(0, N, P)
    j = (i + rng.integers(1, N, P)) % N
    Jv = rng.uniform(0.1, 1.0, P)
    mu = rng.uniform(1.0, 2.0, N)
    h = spx.setup_pairlist(N, np.concatenate([i, j]), np.concatenate([j, i]), np.concatenate([Jv, Jv]), mu=mu,
                           B=(0.0, 0.0, 50.0))
    S = to_dev(random_sphere(N, 3))
    mn = spx.min_create(h, method="lbfgs", dt=0.02, max_step=0.2, tol_force=1e-9)
    spx.min_step(mn, S, 3000)
    assert spx.min_get_stats(mn)["converged"] == 1
    assert np.max(np.abs(S.cpu().numpy()[2] - 1.0)) < 1e-9


def test_lattice_only_methods_refuse_a_pairlist():
    from paper_2605_26016_amd import spx
    pl, _ = disordered(N=50, P=100, seed=1)
    h = gpu_pl(pl)
    S = to_dev(random_sphere(pl.N, 1))
    with pytest.raises(spx.SpxError):
        spx.mc_sweep(h, S, 10.0, seed=1, method="metropolis")
    Y = to_dev(np.stack([random_sphere(pl.N, k) for k in range(4)]))
    with pytest.raises(spx.SpxError):
        spx.gneb_create([h], [Y])
    assert spx.get_info(h).backend == 3
