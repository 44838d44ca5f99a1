"""The Monte Carlo colouring search of libspx on the host (no GPU): it
agrees with the oracle's colouring on ordinary lattices, refuses at once a
bond that joins a site to itself (eight sublattices, periodic axes of extent
1: the search space would be 64^9), and stops at its work bound, with the
reason, on a five-sublattice bond table that no colouring of at most 64
colours satisfies."""
import time

import numpy as np
import pytest

import oracle
from tests.helpers import oracle_model
from workloads import Workload


def lib_colouring(w, bonds=None, cmax=64):
    from paper_2605_26016_amd import spx
    if bonds is None:
        m = oracle_model(w)
        ab = np.stack([m.b_a, m.b_b], 1)
        dl = np.asarray(m.b_delta).reshape(-1, 3)
    else:
        ab, dl = bonds
    return spx.mc_find_colouring(len(w.frac), w.L, w.periodic, ab, dl, cmax)


@pytest.mark.parametrize("w", [
    Workload(name="sc1", L=(20, 20, 20), J_shell=(1.0,)),
    Workload(name="sc2", L=(200, 200, 200), J_shell=(1.0, 0.3)),
    Workload(name="sc3", L=(23, 17, 11), J_shell=(1.0, 0.3, 0.1)),
    Workload(name="sc4_open", L=(10, 9, 8), periodic=(0, 1, 0), J_shell=(1.0, 0.3, 0.1, 0.05)),
    Workload(name="sc_odd", L=(5, 4, 4), J_shell=(1.0,)),
    Workload(name="bcc", L=(8, 8, 8), frac=((0, 0, 0), (0.5, 0.5, 0.5)), mu=(1.0, 1.0),
             J_shell=(1.33, 0.75, -0.05)),
], ids=lambda w: w.name)
def test_colouring_matches_oracle(w):
    C, coef = lib_colouring(w)
    Co, coefo = oracle.mc_colouring(oracle_model(w))
    assert C == Co and np.array_equal(coef, coefo), (C, coef, Co, coefo)


def test_self_bond_refused_at_once():
    from paper_2605_26016_amd import spx
    n_sub = 8
    w = Workload(name="self", L=(1, 1, 1), frac=tuple((0.1 * a, 0.0, 0.0) for a in range(n_sub)),
                 mu=(1.0,) * n_sub)
    # sublattice 3 bonded to itself one cell over: on periodic axes of extent
    # 1 that is the site itself
    ab = [(3, 3)] + [(a, (a + 1) % n_sub) for a in range(n_sub)]
    dl = [(1, 0, 0)] + [(0, 0, 0)] * n_sub
    t0 = time.perf_counter()
    with pytest.raises(spx.SpxError) as e:
        lib_colouring(w, (np.array(ab), np.array(dl)))
    assert time.perf_counter() - t0 < 1.0
    assert "itself" in str(e.value)


def test_search_bound_reached_with_reason():
    from paper_2605_26016_amd import spx
    # sublattice 1 <- 0 at dx = 0 .. 63 on an open axis: every residue mod
    # C <= 64 is realised, so no colouring exists; five sublattices make the
    # candidates grow as C^6 and the bound ends the search, two end it at cmax
    ab = np.array([(1, 0)] * 64)
    dl = np.array([(d, 0, 0) for d in range(64)])
    w5 = Workload(name="w5", L=(80, 2, 2), periodic=(0, 1, 1), frac=tuple((0.1 * a, 0, 0) for a in range(5)),
                  mu=(1.0,) * 5)
    t0 = time.perf_counter()
    with pytest.raises(spx.SpxError) as e:
        lib_colouring(w5, (ab, dl))
    print(f"bound reached after {time.perf_counter() - t0:.2f} s: {e.value}")
    assert "2^26" in str(e.value)
    w2 = Workload(name="w2", L=(80, 2, 2), periodic=(0, 1, 1), frac=((0, 0, 0), (0.5, 0, 0)), mu=(1.0, 1.0))
    with pytest.raises(spx.SpxError) as e:
        lib_colouring(w2, (ab, dl))
    assert "at most 64 colours" in str(e.value)
