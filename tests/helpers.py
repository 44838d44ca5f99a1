"""Shared test helpers: turn a workload description into oracle objects."""
import numpy as np

import oracle
from workloads import Workload


def oracle_lattice(w: Workload) -> "oracle.Lattice":
    return oracle.Lattice(w.L, w.cell, w.frac, w.periodic, w.mu)


def oracle_model(w: Workload) -> "oracle.Model":
    lat = oracle_lattice(w)
    K = None
    if w.K != 0.0:
        K = np.full((w.n_sub, 1), w.K)
        Kax = np.tile(np.asarray(w.K_axis, np.float64), (w.n_sub, 1))
    else:
        Kax = None
    return oracle.Model(lat, n_shells=w.n_shells, J_shell=w.J_shell, D_shell=w.D_shell, K=K,
                        K_axis=Kax, B=w.B, dipolar=w.dipolar)


def max_rel(a, b):
    """max |a - b| / max |b| over all elements."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_hamiltonian(w: Workload, field_prec=None, **kw):
    """libspx Hamiltonian for a workload (shell-defined couplings)."""
    from paper_2605_26016_amd import spx
    prec = field_prec or w.field_prec
    K = w.K if w.K != 0.0 else None
    return spx.setup_hamiltonian(w.L, cell=w.cell, sub_frac=w.frac, mu=w.mu, periodic=w.periodic,
                                 J_shell=w.J_shell, D_shell=w.D_shell, K=K, K_axis=w.K_axis, B=w.B,
                                 dipolar=w.dipolar, field_prec=prec, **kw)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def require_gpu():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def k7_table(J=1.0, D=0.3, mu=2.0, a=0.4, dip=True):
    """The dense 7^3 window's coupling table (workloads.dense7_couplings)."""
    from workloads import dense7_couplings
    return dense7_couplings(J=J, D=D, mu=mu, a=a, dipolar=dip)


def round_bf16(x):
    """FP64 -> FP32 (nearest even) -> BF16 (nearest even), returned as FP64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_fp16(x):
    """FP64 -> FP32 (nearest even) -> FP16 (nearest even), returned as FP64."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)
