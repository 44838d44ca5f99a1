"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/spx.h declares, and rejects bad arguments with the
documented status codes before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


@pytest.fixture(scope="module")
def lib():
    from paper_2605_26016_amd import spx
    path = spx.LIB_PATH
    if not os.path.exists(path):
        from paper_2605_26016_amd import build
        build.build()
    return spx.load()


def declared_symbols():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "spx_setup_hamiltonian" in syms and "spx_llg_heun_step" in syms
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_abi_version(lib):
    from paper_2605_26016_amd import spx
    assert spx.abi_version() == 1


def _status(fn, *args):
    return fn(*args)


def test_null_arguments_rejected(lib):
    from paper_2605_26016_amd import spx
    h = C.c_void_p()
    assert lib.spx_setup_hamiltonian(None, None, None, None, C.byref(h)) == 1
    assert "NULL" in spx.last_error()
    assert lib.spx_setup_hamiltonian(None, None, None, None, None) == 1


def test_bad_descriptors_rejected(lib):
    from paper_2605_26016_amd import spx
    for kw, code in (({"dims": (0, 4, 4)}, 1), ({"mu": (-1.0,)}, 1), ({"periodic": (2, 1, 1)}, 1),
                     ({"field_prec": 7}, 1), ({"backend": 5}, 1),
                     ({"dipolar": 1, "periodic": (1, 1, 1)}, 2),
                     ({"dipolar": 1, "sub_frac": ((0, 0, 0), (0.5, 0.5, 0.5)), "mu": (1, 1),
                       "periodic": (0, 0, 0)}, 2),
                     ({"sub_frac": np.zeros((9, 3)), "mu": np.ones(9)}, 1)):
        args = dict(dims=(4, 4, 4), J_shell=[1.0], stream=0)
        args.update(kw)
        with pytest.raises(spx.SpxError) as ei:
            spx.setup_hamiltonian(**args)
        assert ei.value.status == code, (kw, ei.value)


def test_bad_handles_rejected(lib):
    from paper_2605_26016_amd import spx
    bogus = C.c_void_p(0x1234)
    assert lib.spx_eval_field(bogus, None, None, None) == 6
    assert lib.spx_energy(None, None, None, None, None) == 6
    assert lib.spx_destroy_hamiltonian(bogus) == 6
    info = spx.HamInfo()
    assert lib.spx_get_info(bogus, C.byref(info)) == 6


def test_no_device_reports_hip_error_or_succeeds(lib):
    # In a GPU-less container setup fails with SPX_ERR_HIP, never a crash.
    import torch
    from paper_2605_26016_amd import spx
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(spx.SpxError) as ei:
        spx.setup_hamiltonian((4, 4, 4), J_shell=[1.0], stream=0)
    assert ei.value.status == 4


def test_noise_and_philox_argument_checks(lib):
    assert lib.spx_thermal_noise(1, 2, 0, -5, None, None) == 1
    assert lib.spx_thermal_noise(1, 2, 0, 10, None, None) == 1
    assert lib.spx_philox4x32_10(None, None, 3, None, None) == 1
    assert lib.spx_thermal_noise(1, 2, 0, 0, None, None) == 0


def test_binding_fails_loudly_without_the_library(tmp_path):
    # the Python package copied without libspx.so: every entry point must
    # raise, never fall back to another implementation
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2605_26016_amd")
    dst = tmp_path / "paper_2605_26016_amd"
    dst.mkdir()
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), dst / f)
    code = ("import numpy as np\n"
            "from paper_2605_26016_amd import spx\n"
            "for call in (lambda: spx.load(), lambda: spx.setup_hamiltonian((4, 4, 4), J_shell=(1.0,)),\n"
            "             lambda: spx.abi_version()):\n"
            "    try:\n"
            "        call()\n"
            "    except RuntimeError as e:\n"
            "        assert 'missing' in str(e), e\n"
            "    else:\n"
            "        raise SystemExit('no error without the library')\n"
            "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=120,
                       env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
