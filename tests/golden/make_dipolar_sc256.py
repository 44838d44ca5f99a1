"""Writes tests/golden/dipolar_sc256_direct.npz: the oracle's direct O(N^2)
open-boundary dipolar field of the chiral-magnet workload's seeded start
(sc 256^3, a = 0.4 nm, mu = 2 mu_B; workloads.sc_chiral_dipolar, seed 3) at
the sampled sites of the full-size parity test: the 8 corners, the 12 edge
midpoints, the 6 face centres, the body centre and 4000 random sites (seed
2605).  Calls only the oracle (about 4 minutes on 8 cores); the stored
SHA-256 of the input state lets the test check that it regenerates the same
start.

    python tests/golden/make_dipolar_sc256.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import sc_chiral_dipolar  # noqa: E402

OUT = os.path.join(HERE, "dipolar_sc256_direct.npz")


def sample_sites(L, n_random=4000, seed=2605):
    Lx, Ly, Lz = L
    xs, ys, zs = (0, Lx // 2, Lx - 1), (0, Ly // 2, Ly - 1), (0, Lz // 2, Lz - 1)
    pts = []
    # corners, edge midpoints, face centres, body centre: the 27 points whose
    # coordinates are each an end or the middle of their axis
    for z in zs:
        for y in ys:
            for x in xs:
                pts.append((x, y, z))
    rng = np.random.default_rng(seed)
    pts += [tuple(int(v) for v in rng.integers(0, (Lx, Ly, Lz))) for _ in range(n_random)]
    return np.array([x + Lx * (y + Ly * z) for x, y, z in pts], dtype=np.int64)


def state_digest(S):
    return hashlib.sha256(np.ascontiguousarray(S, np.float64).tobytes()).hexdigest()


def main():
    w = sc_chiral_dipolar()
    S = w.initial_state()
    lat = oracle.Lattice(w.L, w.cell, w.frac, w.periodic, w.mu)
    sites = sample_sites(w.L)
    b = oracle.dipolar_direct(lat, S, sites)
    np.savez_compressed(OUT, sites=sites, b_dip=b, state_sha256=np.array(state_digest(S)))
    print(f"wrote {OUT}: {len(sites)} sites, max |b_dip| {np.abs(b).max():.4e} meV")


if __name__ == "__main__":
    main()
