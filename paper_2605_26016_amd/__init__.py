"""MI355X-native spin-field / LLG-Heun / GNEB library for the hot path of
"SpinX" (arXiv 2605.26016).

The compute lives in libspx.so (HIP kernels for gfx950 behind the C ABI of
include/spx.h); `spx` is its thin ctypes binding.  Build with
`python -m paper_2605_26016_amd.build`.
"""
from . import spx  # noqa: F401
from .spx import (SpxError, abi_version, energy, eval_field, get_bonds, get_info,  # noqa: F401
                  last_error, llg_heun_step, philox4x32_10, setup_hamiltonian, thermal_noise)
