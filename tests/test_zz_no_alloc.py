"""GPU test of spx_energy_noalloc (the energy entry point for callers that
cannot allocate) through the C ABI: two calls in a row on one device, the
second on a smaller lattice, each against spx_energy's energy and terms on the
same state, plus the FP32-field and tensor-coupling tables and the
unsupported cases.  Bars: FP64 fields 1e-12 of the largest term (both are
fixed-order FP64 reductions, in different orders); FP32 fields 1e-6 (the two
accumulate each site's FP32 bilinear sum in different orders, the field's own
bar being 1e-5 of its largest value)."""
import numpy as np
import pytest

from tests.helpers import gpu_hamiltonian, require_gpu, to_dev
from workloads import Workload, bcc_5shell_stochastic, random_sphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def both(h, S):
    import torch
    from paper_2605_26016_amd import spx
    Sd = to_dev(S)
    E0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    t0 = torch.zeros(5, dtype=torch.float64, device="cuda")
    E1 = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    t1 = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    spx.energy(h, Sd, E0, t0)
    spx.energy_noalloc(h, Sd, E1, t1)
    torch.cuda.synchronize()
    return E0.item(), t0.cpu().numpy(), E1.item(), t1.cpu().numpy()


def check(h, S, name, tol=1e-12):
    E0, t0, E1, t1 = both(h, S)
    scale = max(np.max(np.abs(t0)), 1e-300)
    err = max(abs(E1 - E0), float(np.max(np.abs(t1 - t0))))
    print(f"{name}: E {E0:.12e} vs {E1:.12e}, max term diff {err:.2e} (scale {scale:.3e})", flush=True)
    assert err <= tol * scale
    assert t1[3] == 0.0


def test_noalloc_energy_two_calls_second_smaller():
    # large lattice first (4096 strided blocks), then a small one that uses
    # far fewer quadruples of the same scratch
    big = Workload(name="big", L=(160, 150, 140), J_shell=(1.0, -0.2), K=0.1, B=(0.1, 0.0, 0.4))
    small = Workload(name="small", L=(9, 7, 5), periodic=(1, 0, 1), J_shell=(1.0,), D_shell=(0.3,),
                     B=(0.0, 0.0, 0.5), mu=(2.0,))
    check(gpu_hamiltonian(big, field_prec="fp64"), random_sphere(big.N, 81), "big fp64")
    check(gpu_hamiltonian(small, field_prec="fp64"), random_sphere(small.N, 82), "small fp64 (dmi tensor)")


def test_noalloc_energy_fp32_bcc_and_repeat():
    w = bcc_5shell_stochastic((40, 36, 33))
    h = gpu_hamiltonian(w, field_prec="fp32")
    S = w.initial_state()
    check(h, S, "bcc fp32", 1e-6)
    w2 = bcc_5shell_stochastic((6, 5, 4))
    check(gpu_hamiltonian(w2, field_prec="fp32"), w2.initial_state(), "bcc fp32 small", 1e-6)
    # repeated call on the first handle after the smaller one
    check(h, S, "bcc fp32 again", 1e-6)


def test_noalloc_energy_unsupported():
    from paper_2605_26016_amd import spx
    import torch
    wd = Workload(name="d", L=(6, 6, 6), periodic=(0, 0, 0), dipolar=1, mu=(2.0,),
                  cell=((0.4, 0, 0), (0, 0.4, 0), (0, 0, 0.4)))
    h = gpu_hamiltonian(wd, field_prec="fp32")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(spx.SpxError):
        spx.energy_noalloc(h, to_dev(wd.initial_state()), E)
