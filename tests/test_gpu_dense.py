"""Dense 7^3 window on MFMA (BF16 / FP16 operands, FP32 accumulation) against
the FP64 oracle with the operands rounded the same way (FP64 -> FP32 -> 16-bit,
nearest even; couplings scaled by 1/max|K| before rounding), plus the MFMA
lane-layout probe and the FP32 direct (VALU) evaluation of the same window.

Tolerances: layout probe exact; MFMA vs emulated oracle max|b - b_ref| /
max|b_ref| <= 1e-5 (FP32 accumulation of 1029 products); vs the true FP64
field the error is reported and bounded by the operand rounding (BF16 5e-3,
FP16 1e-3); FP32 direct vs FP64 <= 1e-5.

Cases: 6 and 2 tiles (10 x 32 x 16 output sites each), 30 tiles (more than
one per XCD and not a multiple of 8, the tile-dealing branch), and the
256^3 chiral workload's window checked on z-slabs (the window reaches 3
cells, so the oracle run on a slab plus 3 planes each side, open like the
lattice, is exact on the slab's interior planes): the middle of the lattice
and the planes at its open top face.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import k7_table, max_rel, require_gpu, round_bf16, round_fp16, to_dev
from workloads import random_sphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mfma_lane_layout_probe(prec):
    import torch
    from paper_2605_26016_amd import spx
    rng = np.random.default_rng(7)
    A = rng.integers(-4, 5, size=(32, 16)).astype(np.float32)
    B = rng.integers(-4, 5, size=(16, 32)).astype(np.float32)
    D = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    spx.mfma_probe(prec, to_dev(A), to_dev(B), D)
    assert np.array_equal(D.cpu().numpy(), A @ B)


def dense_case(L, periodic, prec, seed=5, backend=2):
    import torch
    from paper_2605_26016_amd import spx
    ab, dl, J = k7_table()
    cell = np.eye(3) * 0.4
    h = spx.setup_hamiltonian(L, cell=cell, mu=(2.0,), periodic=periodic, bonds=(ab, dl, J), B=(0, 0, 0.5),
                              field_prec=prec, backend=backend)
    lat = oracle.Lattice(L, cell, [0, 0, 0], periodic=periodic, mu=[2.0])
    N = lat.N
    S = random_sphere(N, seed)
    b = torch.zeros((3, N), dtype=torch.float32, device="cuda")
    spx.eval_field(h, to_dev(S), b)
    return b.double().cpu().numpy(), S, lat, (ab, dl, J)


def emulated(prec, rnd, J, S):
    """Couplings and spins rounded as the kernel rounds its operands: exact
    power-of-two scalings (BF16: max|K| in [1,2); FP16: max|K| in
    [2^12, 2^13) and spins x 2^10), 16-bit nearest even, scaled back."""
    ke = int(np.floor(np.log2(np.max(np.abs(J)))))
    ws = 2.0 ** ((0 if prec == "bf16" else 12) - ke)
    ins = 1.0 if prec == "bf16" else 1024.0
    return rnd(J * ws) / ws, rnd(S * ins) / ins


@pytest.mark.parametrize("prec,rnd,bound", [("bf16", round_bf16, 5e-3), ("fp16", round_fp16, 1e-3)])
@pytest.mark.parametrize("L,per", [((23, 37, 11), (0, 0, 0)), ((20, 32, 16), (1, 1, 1)), ((41, 70, 20), (0, 0, 0)),
                                   ((41, 70, 20), (1, 0, 1))],
                         ids=["6tiles_open", "2tiles_periodic", "30tiles_open", "30tiles_mixed"])
def test_dense_mfma_matches_emulated_oracle(prec, rnd, bound, L, per):
    got, S, lat, (ab, dl, J) = dense_case(L, per, prec)
    Je, Se = emulated(prec, rnd, J, S)
    B = (0, 0, 0.5)
    me = oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], dl, Je), B=B)
    mt = oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], dl, J), B=B)
    # emulated operands, FP64 accumulation; the Zeeman term is exact on both sides
    ref_e = oracle.field(me, Se)
    assert max_rel(got, ref_e) <= 1e-5, max_rel(got, ref_e)
    ref_t = oracle.field(mt, S)
    err = max_rel(got, ref_t)
    print(f"{prec} {L} {per}: max-rel error vs FP64 field {err:.2e}")
    assert err <= bound


@pytest.mark.parametrize("L,periodic", [((21, 18, 9), (0, 0, 0)), ((37, 19, 17), (1, 0, 1)), ((5, 4, 3), (1, 1, 1)),
                                        ((33, 8, 8), (0, 1, 0))],
                         ids=["open", "mixed_ragged", "smaller_than_window", "exact_y_z_tiles"])
def test_dense_fp32_direct_matches_fp64(L, periodic):
    # the FP32 direct window (16 x 8 x 8 tiles): ragged tails on every axis,
    # periodic wrap, and a lattice smaller than the window (periodic images
    # of one site reached through several offsets); FP32 operands and
    # accumulation over 343 offsets: 1e-5 of the largest field
    got, S, lat, (ab, dl, J) = dense_case(L, periodic, "fp32")
    ref = oracle.field(oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], dl, J), B=(0, 0, 0.5)), S)
    err = max_rel(got, ref)
    print(f"fp32 direct {L} {periodic}: max-rel error vs FP64 {err:.2e}", flush=True)
    assert err <= 1e-5


def test_dense_fp32_gather_matches_fp64():
    got, S, lat, (ab, dl, J) = dense_case((21, 18, 9), (0, 0, 0), "fp32", backend=1)
    ref = oracle.field(oracle.Model(lat, bonds=(ab[:, 0], ab[:, 1], dl, J), B=(0, 0, 0.5)), S)
    assert max_rel(got, ref) <= 1e-5


@pytest.mark.parametrize("prec,rnd", [("bf16", round_bf16), ("fp16", round_fp16)])
def test_dense_mfma_256_slabs(prec, rnd):
    import torch
    from paper_2605_26016_amd import spx
    from workloads import sc_chiral_dipolar
    w = sc_chiral_dipolar()
    L = w.L
    Lx, Ly, Lz = L
    plane = Lx * Ly
    ab, dl, J = k7_table()
    cell = np.eye(3) * 0.4
    h = spx.setup_hamiltonian(L, cell=cell, mu=(2.0,), periodic=(0, 0, 0), bonds=(ab, dl, J), B=(0, 0, 0.5),
                              field_prec=prec, backend=2)
    S = w.initial_state()
    b = torch.zeros((3, w.N), dtype=torch.float32, device="cuda")
    spx.eval_field(h, to_dev(S), b)
    torch.cuda.synchronize()
    Je, Se = emulated(prec, rnd, J, S)
    for z0, nz in ((124, 8), (250, 6)):
        lo, hi = max(z0 - 3, 0), min(z0 + nz + 3, Lz)
        slat = oracle.Lattice((Lx, Ly, hi - lo), cell, [0, 0, 0], periodic=(0, 0, 0), mu=[2.0])
        ref = oracle.field(oracle.Model(slat, bonds=(ab[:, 0], ab[:, 1], dl, Je), B=(0, 0, 0.5)),
                           Se[:, lo * plane:hi * plane])
        ref = ref[:, (z0 - lo) * plane:(z0 - lo + nz) * plane]
        got = b[:, z0 * plane:(z0 + nz) * plane].double().cpu().numpy()
        err = max_rel(got, ref)
        print(f"{prec} 256^3 planes {z0}..{z0 + nz - 1}: max-rel vs emulated oracle {err:.2e}", flush=True)
        assert err <= 1e-5
