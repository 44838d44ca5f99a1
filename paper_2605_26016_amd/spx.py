"""ctypes binding of libspx.so (include/spx.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libspx.so.  Device buffers are torch tensors on the GPU (or raw
integer device pointers); streams default to torch's current stream.  Every
function raises SpxError on a non-OK status, and importing the binding raises
if the library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspx.so")

SPX_FP64, SPX_FP32, SPX_BF16_MFMA, SPX_FP16_MFMA = 0, 1, 2, 3
PREC = {"fp64": SPX_FP64, "fp32": SPX_FP32, "bf16": SPX_BF16_MFMA, "fp16": SPX_FP16_MFMA}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY", 4: "HIP", 5: "FFT",
          6: "BAD_HANDLE"}


class SpxError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: SPX_ERR_{STATUS.get(status, status)}: {msg}")
        self.status = status


class LatticeDesc(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("dims", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("cell", C.c_double * 9), ("sub_frac", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double))]


class ModelDesc(C.Structure):
    _fields_ = [("n_shells", C.c_int32), ("J_shell", C.POINTER(C.c_double)),
                ("D_shell", C.POINTER(C.c_double)), ("n_bonds", C.c_int32),
                ("bond_ab", C.POINTER(C.c_int32)), ("bond_delta", C.POINTER(C.c_int32)),
                ("bond_J", C.POINTER(C.c_double)), ("n_aniso", C.c_int32),
                ("K", C.POINTER(C.c_double)), ("K_axis", C.POINTER(C.c_double)),
                ("B_ext", C.c_double * 3), ("dipolar", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("field_prec", C.c_int32), ("backend", C.c_int32), ("autotune", C.c_int32),
                ("tune_cache_path", C.c_char_p), ("stencil_engine", C.c_int32), ("zchunk", C.c_int32),
                ("heun_field", C.c_int32), ("tile_rows", C.c_int32)]


class LlgParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("dt_fs", C.c_double), ("temperature_K", C.c_double),
                ("gamma", C.c_double), ("seed", C.c_uint64), ("step0", C.c_uint64),
                ("tag", C.c_uint32), ("n_steps", C.c_int32)]


class GnebParams(C.Structure):
    _fields_ = [("spring_k", C.c_double), ("vp_dt", C.c_double), ("vp_mass", C.c_double),
                ("ci_mode", C.c_int32), ("ci_on_below", C.c_double), ("tol_force", C.c_double)]


class McParams(C.Structure):
    _fields_ = [("temperature_K", C.c_double), ("seed", C.c_uint64), ("sweep0", C.c_uint64),
                ("n_sweeps", C.c_int32), ("method", C.c_int32), ("layout", C.c_int32)]


class MinParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("retraction", C.c_int32), ("dt", C.c_double), ("mass", C.c_double),
                ("history", C.c_int32), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("max_step", C.c_double), ("tol_force", C.c_double)]


class PairListDesc(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_pairs", C.c_int64), ("target", C.c_void_p), ("source", C.c_void_p),
                ("J", C.c_void_p), ("tensor", C.c_int32), ("mu", C.c_void_p), ("K", C.c_void_p),
                ("K_axis", C.c_void_p), ("B_ext", C.c_double * 3)]


class HamInfo(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_bonds", C.c_int32), ("field_prec", C.c_int32),
                ("backend", C.c_int32), ("radius", C.c_int32 * 3), ("dipolar", C.c_int32),
                ("workspace_bytes", C.c_int64), ("stencil_engine", C.c_int32), ("shape", C.c_int32),
                ("zchunk", C.c_int32), ("heun_field", C.c_int32), ("tuned", C.c_int32),
                ("tuned_step_us", C.c_double), ("heun_graph", C.c_int32), ("tile_rows", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libspx.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -m paper_2605_26016_amd.build)")
    L = C.CDLL(path)
    vp, i32, i64, u64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32, C.c_double
    sigs = {
        "spx_setup_hamiltonian": [C.POINTER(LatticeDesc), C.POINTER(ModelDesc), C.POINTER(Options), vp,
                                  C.POINTER(vp)],
        "spx_destroy_hamiltonian": [vp],
        "spx_eval_field": [vp, vp, vp, vp],
        "spx_energy": [vp, vp, vp, vp, vp],
        "spx_energy_noalloc": [vp, vp, vp, vp, vp],
        "spx_llg_heun_step": [vp, vp, C.POINTER(LlgParams), vp],
        "spx_thermal_noise": [u64, u64, u32, i64, vp, vp],
        "spx_philox4x32_10": [vp, vp, i64, vp, vp],
        "spx_get_info": [vp, C.POINTER(HamInfo)],
        "spx_get_bonds": [vp, vp, vp, vp],
        "spx_set_kernel_timing": [vp, i32],
        "spx_set_heun_graph": [vp, i32],
        "spx_gneb_create": [C.POINTER(vp), i32, C.POINTER(vp), C.POINTER(C.c_int32), C.POINTER(GnebParams),
                            vp, C.POINTER(vp)],
        "spx_gneb_destroy": [vp],
        "spx_gneb_init_path": [vp, i32, vp, vp, vp],
        "spx_net_create": [vp, C.POINTER(vp)],
        "spx_net_destroy": [vp],
        "spx_net_set_dilation": [vp, C.POINTER(C.c_int32)],
        "spx_net_set_precision": [vp, i32],
        "spx_mfma16_probe": [vp, vp, vp, vp],
        "spx_net_forward": [vp, vp, C.POINTER(C.c_int32), i32, vp, vp, vp, vp, vp, vp],
        "spx_net_backward": [vp, vp, C.POINTER(C.c_int32), i32, vp, vp, vp, vp, vp, vp, vp, vp],
        "spx_net_adam_step": [vp, vp, vp, vp, i64, i64, dbl, dbl, dbl, dbl, vp],
        "spx_gneb_step": [vp, i32, vp],
        "spx_gneb_get_stats": [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp],
        "spx_gneb_set_graph": [vp, i32],
        "spx_mc_sweep": [vp, vp, C.POINTER(McParams), vp, vp],
        "spx_setup_pairlist": [C.POINTER(PairListDesc), C.POINTER(Options), vp, C.POINTER(vp)],
        "spx_min_create": [vp, C.POINTER(MinParams), vp, C.POINTER(vp)],
        "spx_min_step": [vp, vp, i32, vp],
        "spx_min_get_stats": [vp, vp, vp, vp, vp],
        "spx_min_reset": [vp, vp],
        "spx_min_destroy": [vp],
        "spx_mc_colouring": [vp, C.POINTER(C.c_int32), vp],
        "spx_magnetization": [vp, vp, vp, vp],
        "spx_gneb_set_spacing": [vp, i32, vp, vp],
        "spx_gneb_redistribute": [vp, vp],
        "spx_gneb_set_params": [vp, C.POINTER(GnebParams), vp],
        "spx_mfma_probe": [i32, vp, vp, vp, vp],
        "spx_stream_probe": [i32, vp, vp, i64, vp],
        "spx_mc_find_colouring": [i32, vp, vp, i32, vp, vp, i32, vp, vp],
        "spx_get_kernel_times": [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.spx_last_error.restype = C.c_char_p
    L.spx_last_error.argtypes = []
    L.spx_abi_version.restype = C.c_int32
    L.spx_abi_version.argtypes = []
    L.spx_net_nparams.restype = C.c_int64
    L.spx_net_nparams.argtypes = []
    _lib = L
    _register_extensions(L)
    return L


_ext_registrars = []


def _register_extensions(L):
    for fn in _ext_registrars:
        fn(L)


def _check(status: int, where: str):
    if status != 0:
        raise SpxError(status, where, last_error())


def last_error() -> str:
    return load().spx_last_error().decode()


def abi_version() -> int:
    return int(load().spx_abi_version())


# ---------------------------------------------------------------- marshalling
def _ptr(x) -> Optional[int]:
    """Device pointer of a torch tensor (checked contiguous), an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        if x.device.type != "cuda":
            raise ValueError("device buffers must live on the GPU")
        return x.data_ptr()
    raise TypeError(f"cannot take a device pointer of {type(x)}")


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Hamiltonian:
    """Owner of an spx_ham handle (destroyed with the object)."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep
        self._info = None

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load().spx_destroy_hamiltonian(self.handle)
            except Exception:
                pass
            self.handle = None

    def destroy(self):
        if self.handle:
            _check(load().spx_destroy_hamiltonian(self.handle), "spx_destroy_hamiltonian")
            self.handle = None

    @property
    def info(self) -> HamInfo:
        if self._info is None:
            self._info = get_info(self)
        return self._info

    @property
    def N(self) -> int:
        return int(self.info.n_sites)


def setup_hamiltonian(dims: Sequence[int], cell=None, sub_frac=((0.0, 0.0, 0.0),), mu=(1.0,),
                      periodic=(1, 1, 1), J_shell=None, D_shell=None, bonds=None, K=None,
                      K_axis=None, B=(0.0, 0.0, 0.0), dipolar=0, field_prec="fp64", backend=0,
                      autotune=0, tune_cache_path=None, stencil_engine=0, zchunk=0, heun_field=0,
                      tile_rows=0, stream=None) -> Hamiltonian:
    """Wraps spx_setup_hamiltonian.  K: [n_sub][n_aniso] meV (or scalar applied
    to every sublattice with one axis), K_axis: matching unit vectors.
    bonds = (ab [n][2], delta [n][3], J [n][9]) overrides the shells."""
    L = load()
    frac = np.ascontiguousarray(np.asarray(sub_frac, np.float64).reshape(-1))
    n_sub = len(frac) // 3
    mu_a = np.ascontiguousarray(np.asarray(mu, np.float64).reshape(-1))
    cell_a = np.asarray(np.eye(3) if cell is None else cell, np.float64).reshape(9)
    lat = LatticeDesc()
    lat.n_sub = n_sub
    lat.dims[:] = [int(v) for v in dims]
    lat.periodic[:] = [int(v) for v in periodic]
    lat.cell[:] = list(cell_a)
    lat.sub_frac = _dptr(frac)
    lat.mu = _dptr(mu_a)
    keep = [frac, mu_a]
    m = ModelDesc()
    if J_shell is not None:
        Js = np.ascontiguousarray(np.asarray(J_shell, np.float64).reshape(-1))
        keep.append(Js)
        m.n_shells = len(Js)
        m.J_shell = _dptr(Js)
        if D_shell is not None:
            Ds = np.ascontiguousarray(np.asarray(D_shell, np.float64).reshape(-1))
            if len(Ds) != len(Js):
                raise ValueError("D_shell must match J_shell")
            keep.append(Ds)
            m.D_shell = _dptr(Ds)
    if bonds is not None:
        ab, dl, Jb = bonds
        ab = np.ascontiguousarray(np.asarray(ab, np.int32).reshape(-1))
        dl = np.ascontiguousarray(np.asarray(dl, np.int32).reshape(-1))
        Jb = np.ascontiguousarray(np.asarray(Jb, np.float64).reshape(-1))
        keep += [ab, dl, Jb]
        m.n_bonds = len(ab) // 2
        m.bond_ab, m.bond_delta, m.bond_J = _iptr(ab), _iptr(dl), _dptr(Jb)
    if K is not None:
        Ka = np.asarray(K, np.float64)
        if Ka.ndim == 0:
            Ka = np.full((n_sub, 1), float(Ka))
        Ka = np.ascontiguousarray(Ka.reshape(n_sub, -1))
        ax = np.asarray((0.0, 0.0, 1.0) if K_axis is None else K_axis, np.float64)
        if ax.size == 3:
            ax = np.tile(ax, (n_sub, Ka.shape[1], 1))
        ax = np.ascontiguousarray(ax.reshape(-1))
        keep += [Ka, ax]
        m.n_aniso = Ka.shape[1]
        m.K, m.K_axis = _dptr(Ka.reshape(-1)), _dptr(ax)
    m.B_ext[:] = [float(v) for v in B]
    m.dipolar = int(dipolar)
    o = Options()
    o.field_prec = PREC[field_prec] if isinstance(field_prec, str) else int(field_prec)
    o.backend = int(backend)
    o.autotune = int(autotune)
    o.tune_cache_path = None if tune_cache_path is None else tune_cache_path.encode()
    o.stencil_engine = int(stencil_engine)
    o.zchunk = int(zchunk)
    o.heun_field = int(heun_field)
    o.tile_rows = int(tile_rows)
    h = C.c_void_p()
    _check(L.spx_setup_hamiltonian(C.byref(lat), C.byref(m), C.byref(o), _stream(stream), C.byref(h)),
           "spx_setup_hamiltonian")
    return Hamiltonian(h.value, keep)


def setup_pairlist(n_sites, target, source, J, mu=None, K=None, K_axis=None, B=(0.0, 0.0, 0.0),
                   field_prec="fp64", stream=None) -> Hamiltonian:
    """Pair-list Hamiltonian: entry p couples target[p] <- source[p] with J[p]
    (scalar per entry, or [n][3][3] blocks); per-site moments mu, uniaxial
    anisotropy K with unit axes K_axis (host arrays, copied)."""
    L = load()
    t = np.ascontiguousarray(target, dtype=np.int64)
    so = np.ascontiguousarray(source, dtype=np.int64)
    Ja = np.asarray(J, dtype=np.float64)
    tensor = 1 if Ja.ndim == 3 else 0
    Ja = np.ascontiguousarray(Ja.reshape(len(t), 9) if tensor else Ja.reshape(-1))
    keep = [t, so, Ja]
    d = PairListDesc()
    d.n_sites, d.n_pairs = int(n_sites), len(t)
    d.target, d.source, d.J = t.ctypes.data, so.ctypes.data, Ja.ctypes.data
    d.tensor = tensor
    for name, arr in (("mu", mu), ("K", K), ("K_axis", K_axis)):
        if arr is None:
            setattr(d, name, None)
        else:
            a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
            keep.append(a)
            setattr(d, name, a.ctypes.data)
    d.B_ext[:] = [float(v) for v in B]
    o = Options()
    o.field_prec = PREC[field_prec] if isinstance(field_prec, str) else int(field_prec)
    h = C.c_void_p()
    _check(L.spx_setup_pairlist(C.byref(d), C.byref(o), _stream(stream), C.byref(h)), "spx_setup_pairlist")
    return Hamiltonian(h.value, keep)


def _h(h):
    return h.handle if isinstance(h, Hamiltonian) else h


def eval_field(h, S, b, stream=None):
    _check(load().spx_eval_field(_h(h), _ptr(S), _ptr(b), _stream(stream)), "spx_eval_field")


def energy(h, S, E, terms=None, stream=None):
    _check(load().spx_energy(_h(h), _ptr(S), _ptr(E), _ptr(terms), _stream(stream)), "spx_energy")


def energy_noalloc(h, S, E, terms=None, stream=None):
    """spx_energy_noalloc: the same energy with no allocation in the call."""
    _check(load().spx_energy_noalloc(_h(h), _ptr(S), _ptr(E), _ptr(terms), _stream(stream)),
           "spx_energy_noalloc")


def llg_heun_step(h, S, alpha, dt_fs, temperature_K=0.0, gamma=0.0, seed=0, step0=0, tag=0,
                  n_steps=1, stream=None):
    p = LlgParams(float(alpha), float(dt_fs), float(temperature_K), float(gamma), int(seed),
                  int(step0), int(tag), int(n_steps))
    _check(load().spx_llg_heun_step(_h(h), _ptr(S), C.byref(p), _stream(stream)), "spx_llg_heun_step")


def thermal_noise(seed, step, tag, N, eta, stream=None):
    _check(load().spx_thermal_noise(int(seed), int(step), int(tag), int(N), _ptr(eta), _stream(stream)),
           "spx_thermal_noise")


def philox4x32_10(ctr, key, n, out, stream=None):
    _check(load().spx_philox4x32_10(_ptr(ctr), _ptr(key), int(n), _ptr(out), _stream(stream)),
           "spx_philox4x32_10")


def get_info(h) -> HamInfo:
    info = HamInfo()
    _check(load().spx_get_info(_h(h), C.byref(info)), "spx_get_info")
    return info


def get_bonds(h):
    info = get_info(h)
    n = info.n_bonds
    ab = np.zeros(2 * max(n, 1), np.int32)
    dl = np.zeros(3 * max(n, 1), np.int32)
    J = np.zeros(9 * max(n, 1), np.float64)
    _check(load().spx_get_bonds(_h(h), ab.ctypes.data, dl.ctypes.data, J.ctypes.data), "spx_get_bonds")
    return ab[:2 * n].reshape(n, 2), dl[:3 * n].reshape(n, 3), J[:9 * n].reshape(n, 3, 3)


KERNEL_KINDS = {"heun_predict": 0, "heun_correct": 1, "field": 2, "noise": 3}


def set_kernel_timing(h, enable=True):
    _check(load().spx_set_kernel_timing(_h(h), int(bool(enable))), "spx_set_kernel_timing")


def get_kernel_times(h, kind):
    """(launch count, summed duration in ms) of one kernel kind since the last query."""
    k = KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
    n = C.c_int64()
    t = C.c_double()
    _check(load().spx_get_kernel_times(_h(h), k, C.byref(n), C.byref(t)), "spx_get_kernel_times")
    return int(n.value), float(t.value)


# ---------------------------------------------------------------- GNEB
class Gneb:
    """Owner of an spx_gneb handle; keeps the Hamiltonians and image buffers alive."""

    def __init__(self, handle, hams, images, n_img):
        self.handle = handle
        self.hams = list(hams)
        self.images = list(images)
        self.n_img = list(n_img)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load().spx_gneb_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def gneb_create(hams, images, spring_k=1.0, vp_dt=0.1, vp_mass=1.0, ci_mode=1, ci_on_below=1e-2,
                tol_force=0.0, stream=None) -> Gneb:
    """images: list of device tensors [n_img][3][N_k] (updated in place)."""
    n = len(hams)
    H = (C.c_void_p * n)(*[_h(h) for h in hams])
    Y = (C.c_void_p * n)(*[_ptr(y) for y in images])
    n_img = [int(y.shape[0]) for y in images]
    NI = (C.c_int32 * n)(*n_img)
    p = GnebParams(float(spring_k), float(vp_dt), float(vp_mass), int(ci_mode), float(ci_on_below),
                   float(tol_force))
    g = C.c_void_p()
    _check(load().spx_gneb_create(H, n, Y, NI, C.byref(p), _stream(stream), C.byref(g)), "spx_gneb_create")
    return Gneb(g.value, hams, images, n_img)


def gneb_init_path(g, method=0, net=None, params=None, stream=None):
    """method 0: geodesic; method 1: geodesic corrected by the network `net`
    with FP32 parameter tensor `params`."""
    _check(load().spx_gneb_init_path(g.handle, int(method), None if net is None else net.handle, _ptr(params),
                                     _stream(stream)), "spx_gneb_init_path")


def gneb_step(g, n_iter=1, stream=None):
    _check(load().spx_gneb_step(g.handle, int(n_iter), _stream(stream)), "spx_gneb_step")


def gneb_set_spacing(g, inst, alpha, stream=None):
    """Target arc-length fractions of instance `inst` (alpha[0] = 0, alpha[-1] = 1)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    _check(load().spx_gneb_set_spacing(g.handle, int(inst), a.ctypes.data_as(C.c_void_p), _stream(stream)),
           "spx_gneb_set_spacing")


def gneb_redistribute(g, stream=None):
    """Geodesic reparameterisation of every instance to its target spacing."""
    _check(load().spx_gneb_redistribute(g.handle, _stream(stream)), "spx_gneb_redistribute")


def gneb_set_params(g, spring_k=1.0, vp_dt=0.1, vp_mass=1.0, ci_mode=1, ci_on_below=1e-2, tol_force=0.0,
                    stream=None):
    """New parameters for every instance (the paths are kept; velocities,
    counters and flags are cleared)."""
    p = GnebParams(float(spring_k), float(vp_dt), float(vp_mass), int(ci_mode), float(ci_on_below),
                   float(tol_force))
    _check(load().spx_gneb_set_params(g.handle, C.byref(p), _stream(stream)), "spx_gneb_set_params")


def gneb_set_graph(g, enable=True):
    _check(load().spx_gneb_set_graph(g.handle, int(bool(enable))), "spx_gneb_set_graph")


MIN_METHODS = {"vp": 0, "bb": 1, "lbfgs": 2, "adam": 3}
RETRACTIONS = {"exp": 0, "norm": 1}


class Minimizer:
    """Owner of an spx_min handle (keeps its Hamiltonian alive)."""

    def __init__(self, handle, ham):
        self.handle = handle
        self.ham = ham

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load().spx_min_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def min_create(h, method="vp", retraction="exp", dt=0.1, mass=1.0, history=5, beta1=0.9, beta2=0.999,
               eps=1e-8, max_step=0.0, tol_force=0.0, stream=None) -> Minimizer:
    p = MinParams(MIN_METHODS[method] if isinstance(method, str) else int(method),
                  RETRACTIONS[retraction] if isinstance(retraction, str) else int(retraction), float(dt),
                  float(mass), int(history), float(beta1), float(beta2), float(eps), float(max_step),
                  float(tol_force))
    m = C.c_void_p()
    _check(load().spx_min_create(_h(h), C.byref(p), _stream(stream), C.byref(m)), "spx_min_create")
    return Minimizer(m.value, h)


def min_step(m, S, n_iter=1, stream=None):
    _check(load().spx_min_step(m.handle, _ptr(S), int(n_iter), _stream(stream)), "spx_min_step")


def min_get_stats(m, stream=None):
    mf = C.c_double()
    it, conv = C.c_int32(), C.c_int32()
    _check(load().spx_min_get_stats(m.handle, C.byref(mf), C.byref(it), C.byref(conv), _stream(stream)),
           "spx_min_get_stats")
    return {"max_force": mf.value, "iterations": it.value, "converged": conv.value}


def min_reset(m, stream=None):
    _check(load().spx_min_reset(m.handle, _stream(stream)), "spx_min_reset")


MC_METHODS = {"heat_bath": 0, "metropolis": 1}


def mc_sweep(h, S, temperature_K, seed, sweep0=0, n_sweeps=1, method="heat_bath", accepted=None, stream=None,
             in_place=False):
    """n_sweeps heat-bath or Metropolis sweeps of the device state S in place;
    `accepted` (device uint64 tensor of 1, optional) receives the accepted moves;
    in_place keeps the sweeps in the natural layout (no colour-major copy)."""
    m = MC_METHODS[method] if isinstance(method, str) else int(method)
    p = McParams(float(temperature_K), int(seed), int(sweep0), int(n_sweeps), m, 1 if in_place else 0)
    _check(load().spx_mc_sweep(_h(h), _ptr(S), C.byref(p), _ptr(accepted), _stream(stream)), "spx_mc_sweep")


def mc_colouring(h):
    """(C, coef) with coef = (ky, kz, o_0 .. o_{n_sub-1})."""
    nc = C.c_int32()
    coef = np.zeros(2 + 8, np.int32)
    _check(load().spx_mc_colouring(_h(h), C.byref(nc), coef.ctypes.data_as(C.c_void_p)), "spx_mc_colouring")
    return nc.value, coef


def magnetization(h, S, m, stream=None):
    """m (device double tensor of 3) = sum_i S_i."""
    _check(load().spx_magnetization(_h(h), _ptr(S), _ptr(m), _stream(stream)), "spx_magnetization")


def gneb_destroy(g):
    """Release the library's buffers of g now (otherwise when g is collected)."""
    if getattr(g, "handle", None):
        _check(load().spx_gneb_destroy(g.handle), "spx_gneb_destroy")
        g.handle = None


def gneb_get_stats(g, inst=0, stream=None):
    n = g.n_img[inst]
    E = np.zeros(n)
    d = np.zeros(max(n - 1, 1))
    mf = C.c_double()
    ci, con, iters, conv = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().spx_gneb_get_stats(g.handle, int(inst), E.ctypes.data, d.ctypes.data, C.byref(mf),
                                     C.byref(ci), C.byref(con), C.byref(iters), C.byref(conv),
                                     _stream(stream)), "spx_gneb_get_stats")
    return {"E": E, "dist": d[:n - 1], "max_force": mf.value, "ci_index": ci.value, "ci_on": con.value,
            "iterations": iters.value, "converged": conv.value}


def mfma_probe(prec, A, B, D, stream=None):
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(load().spx_mfma_probe(p, _ptr(A), _ptr(B), _ptr(D), _stream(stream)), "spx_mfma_probe")


# ---------------------------------------------------------------- learned corrector
class Net:
    """Owner of an spx_net workspace handle; dilation: per-layer dilation of
    the four 3^3 convolutions (spx_net_set_dilation)."""

    def __init__(self, dilation=(1, 1, 1, 1)):
        h = C.c_void_p()
        _check(load().spx_net_create(None, C.byref(h)), "spx_net_create")
        self.handle = h.value
        self.dilation = tuple(int(v) for v in dilation)
        if self.dilation != (1, 1, 1, 1):
            net_set_dilation(self, self.dilation)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load().spx_net_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def net_set_dilation(net, dil):
    d = (C.c_int32 * 4)(*[int(v) for v in dil])
    _check(load().spx_net_set_dilation(net.handle, d), "spx_net_set_dilation")
    net.dilation = tuple(int(v) for v in dil)


def net_set_precision(net, prec):
    """Forward arithmetic of the net: "fp32" or "bf16" (BF16 MFMA)."""
    p = {"fp32": PREC["fp32"], "bf16": PREC["bf16"]}[prec] if isinstance(prec, str) else int(prec)
    _check(load().spx_net_set_precision(net.handle, p), "spx_net_set_precision")


def mfma16_probe(A, B, D, stream=None):
    _check(load().spx_mfma16_probe(_ptr(A), _ptr(B), _ptr(D), _stream(stream)), "spx_mfma16_probe")


def net_nparams() -> int:
    return int(load().spx_net_nparams())


def _dims(dims):
    return (C.c_int32 * 3)(*[int(v) for v in dims])


def net_forward(net, params, dims, batch, Sg, SA, SB, t, Shat, stream=None):
    _check(load().spx_net_forward(net.handle, _ptr(params), _dims(dims), int(batch), _ptr(Sg), _ptr(SA), _ptr(SB),
                                  _ptr(t), _ptr(Shat), _stream(stream)), "spx_net_forward")


def net_backward(net, params, dims, batch, Sg, SA, SB, t, Sstar, grad, loss=None, stream=None):
    _check(load().spx_net_backward(net.handle, _ptr(params), _dims(dims), int(batch), _ptr(Sg), _ptr(SA), _ptr(SB),
                                   _ptr(t), _ptr(Sstar), _ptr(grad), _ptr(loss), _stream(stream)),
           "spx_net_backward")


def net_adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    n = int(params.numel())
    _check(load().spx_net_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, int(step), float(lr), float(b1),
                                    float(b2), float(eps), _stream(stream)), "spx_net_adam_step")


def set_heun_graph(h, enable=True):
    _check(load().spx_set_heun_graph(_h(h), int(bool(enable))), "spx_set_heun_graph")


def stream_probe(kind, src, dst, n_bytes, stream=None):
    """spx_stream_probe: kind 0 copy src -> dst, 1 read src, 2 write dst."""
    _check(load().spx_stream_probe(int(kind), _ptr(src), _ptr(dst), int(n_bytes), _stream(stream)),
           "spx_stream_probe")


def mc_find_colouring(n_sub, dims, periodic, bond_ab, bond_delta, cmax=64):
    """spx_mc_find_colouring (host only): (C, coef) of the Monte Carlo
    colouring, or SpxError when there is none within the search's limits."""
    L = load()
    d = np.ascontiguousarray(np.asarray(dims, np.int32))
    pr = np.ascontiguousarray(np.asarray(periodic, np.int32))
    ab = np.ascontiguousarray(np.asarray(bond_ab, np.int32).reshape(-1))
    dl = np.ascontiguousarray(np.asarray(bond_delta, np.int32).reshape(-1))
    n = C.c_int32(0)
    coef = np.zeros(2 + int(n_sub), np.int32)
    _check(L.spx_mc_find_colouring(int(n_sub), _iptr(d), _iptr(pr), len(ab) // 2, _iptr(ab), _iptr(dl), int(cmax),
                                   C.byref(n), _iptr(coef)), "spx_mc_find_colouring")
    return int(n.value), coef
