"""Plain FP64 CPU oracle for the SpinX hot path (arXiv 2605.26016).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library under ``paper_2605_26016_amd/``: the C source
``spx_oracle.c`` and the NumPy reference ``dipolar_fft.py`` are written from the
paper's equations alone (Methods: Hamiltonian, effective field, sublattice
convolution, LLG/Heun, stochastic LLG, minimum-energy paths).

Every array is float64 NumPy; spin and field arrays are SoA planes of shape
``(3, N)`` with the site index ``x + Lx*(y + Ly*(z + Lz*a))``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spx_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libspx_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        L.or_const.restype = C.c_double
        L.or_const.argtypes = [C.c_int]
        L.or_shell_distances.restype = C.c_int
        L.or_shell_distances.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp]
        L.or_build_bonds.restype = C.c_int
        L.or_build_bonds.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, C.c_void_p, C.c_int,
                                     _ip, _ip, _ip, _dp, _ip]
        model = [C.c_int, _ip, _ip, _dp, _dp, C.c_int, _ip, _ip, _ip, _dp, C.c_int, _dp, _dp,
                 _dp, _dp, C.c_int]
        L.or_field.restype = None
        L.or_field.argtypes = model + [_dp] + [C.c_void_p] * 5
        L.or_energy.restype = None
        L.or_energy.argtypes = model + [_dp, _dp]
        L.or_bruteforce.restype = None
        L.or_bruteforce.argtypes = [C.c_int, _ip, _ip, _dp, _dp, C.c_int, _dp, C.c_void_p, _dp,
                                    _dp, C.c_void_p]
        L.or_dipolar_direct.restype = None
        L.or_dipolar_direct.argtypes = [C.c_int, _ip, _dp, _dp, _dp, _dp, C.c_int, _lp, _dp]
        L.or_philox4x32_10.restype = None
        L.or_philox4x32_10.argtypes = [_up, _up, _up]
        L.or_thermal_eta.restype = None
        L.or_thermal_eta.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_long, _dp]
        L.or_heun.restype = None
        L.or_heun.argtypes = model + [C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_uint64,
                                      C.c_uint32, C.c_uint64, C.c_int, _dp]
        L.or_image_distance.restype = C.c_double
        L.or_image_distance.argtypes = [C.c_long, _dp, _dp]
        L.or_geodesic_path.restype = None
        L.or_geodesic_path.argtypes = [C.c_long, _dp, _dp, C.c_int, _dp]
        L.or_gneb_iterate.restype = None
        L.or_gneb_iterate.argtypes = [C.c_int, _ip, _ip, _dp, _dp, C.c_int, _ip, _ip, _ip, _dp,
                                      C.c_int, _dp, _dp, _dp, _dp, C.c_int, _dp, _dp, C.c_double,
                                      C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.POINTER(C.c_int), C.c_void_p, _dp, _dp, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int)]
        L.or_mc_colouring.restype = C.c_int
        L.or_mc_colouring.argtypes = [C.c_int, _ip, _ip, _dp, _dp, C.c_int, _ip, _ip, _ip, _dp, C.c_int, _ip]
        L.or_mc_sweeps.restype = C.c_long
        L.or_mc_sweeps.argtypes = model + [_dp, C.c_double, C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_int,
                                           _ip]
        L.or_min_iterate.restype = None
        L.or_min_iterate.argtypes = model + [_dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                             C.c_double, C.c_double, C.c_double, C.c_double, _dp, _lp,
                                             C.POINTER(C.c_double)]
        pl = [C.c_long, C.c_long, _lp, _lp, _dp, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, _dp]
        L.or_pl_field.restype = None
        L.or_pl_field.argtypes = pl + [_dp, _dp]
        L.or_pl_energy.restype = None
        L.or_pl_energy.argtypes = pl + [_dp, _dp]
        L.or_pl_heun.restype = None
        L.or_pl_heun.argtypes = pl + [C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_uint64, C.c_uint32,
                                      C.c_int, _dp]
        L.or_reparametrize.restype = None
        L.or_reparametrize.argtypes = [C.c_long, C.c_int, _dp, C.c_void_p, _dp]
        L.or_net_nparams.restype = C.c_long
        L.or_net_nparams.argtypes = [_ip]
        L.or_net_forward.restype = None
        L.or_net_forward.argtypes = [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp, _dp, _dp, C.c_void_p]
        L.or_net_predict_loss.restype = C.c_double
        L.or_net_predict_loss.argtypes = [C.c_long, _dp, _dp, C.c_void_p, C.c_void_p]
        L.or_net_forward_q.restype = None
        L.or_net_forward_q.argtypes = [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp, _dp, _dp, C.c_void_p, C.c_int]
        L.or_net_backward.restype = C.c_double
        L.or_net_backward.argtypes = [C.c_int, C.c_int, C.c_int, _ip, _ip, _dp, _dp, _dp, _dp, _dp]
        L.or_adam.restype = None
        L.or_adam.argtypes = [C.c_long, _dp, _dp, _dp, _dp, C.c_long, C.c_double, C.c_double,
                              C.c_double, C.c_double]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- constants
MU_B = None
K_B = None
GAMMA = None
DIP_PREF = None


def constants():
    """(mu_B meV/T, k_B meV/K, gamma rad/(fs T), mu0/4pi mu_B^2 meV nm^3)."""
    L = lib()
    return tuple(L.or_const(k) for k in range(4))


# ---------------------------------------------------------------- model objects
class Lattice:
    """Bravais lattice with n_sub sublattices, L cells per axis."""

    def __init__(self, L, cell, frac, periodic=(1, 1, 1), mu=None):
        self.L = _i32(L)
        self.cell = _f64(np.asarray(cell, dtype=np.float64).reshape(9))
        self.frac = _f64(np.asarray(frac, dtype=np.float64).reshape(-1))
        self.n_sub = len(self.frac) // 3
        self.periodic = _i32(periodic)
        self.mu = _f64(mu if mu is not None else np.ones(self.n_sub))

    @property
    def N(self):
        return int(self.n_sub * np.prod(self.L))


class Model:
    """Directed bonds + on-site terms (host arrays)."""

    def __init__(self, lat: Lattice, n_shells=0, J_shell=(), D_shell=None, bonds=None,
                 K=None, K_axis=None, B=(0.0, 0.0, 0.0), dipolar=0, max_bonds=4096):
        self.lat = lat
        if bonds is None:
            a = np.zeros(max_bonds, np.int32)
            b = np.zeros(max_bonds, np.int32)
            d = np.zeros(3 * max_bonds, np.int32)
            J = np.zeros(9 * max_bonds, np.float64)
            sh = np.zeros(max_bonds, np.int32)
            Jp = _f64(J_shell).reshape(-1)
            Dp = None if D_shell is None else _f64(D_shell).reshape(-1)
            # the bond builder reads one J and one D per shell
            if len(Jp) < n_shells or (Dp is not None and len(Dp) < n_shells):
                raise ValueError("J_shell and D_shell need one entry per shell")
            nb = lib().or_build_bonds(lat.n_sub, lat.cell, lat.frac, int(n_shells), Jp,
                                      _ptr(Dp), max_bonds, a, b, d, J, sh)
            if nb < 0:
                raise RuntimeError("oracle bond enumeration failed")
            self.b_a, self.b_b = a[:nb].copy(), b[:nb].copy()
            self.b_delta = d[:3 * nb].copy()
            self.b_J = J[:9 * nb].copy()
            self.b_shell = sh[:nb].copy()
        else:
            ba, bb, bd, bJ = bonds
            self.b_a, self.b_b = _i32(ba), _i32(bb)
            self.b_delta = _i32(np.asarray(bd).reshape(-1))
            self.b_J = _f64(np.asarray(bJ).reshape(-1))
            self.b_shell = np.full(len(self.b_a), -1, np.int32)
        self.n_shells = n_shells
        self.J_shell = _f64(J_shell) if n_shells else _f64([0.0])
        self.D_shell = None if D_shell is None else _f64(D_shell)
        if K is None:
            self.n_aniso = 0
            self.K = _f64([0.0])
            self.K_axis = _f64([0.0, 0.0, 1.0])
        else:
            K = np.asarray(K, np.float64).reshape(lat.n_sub, -1)
            self.n_aniso = K.shape[1]
            self.K = _f64(K.reshape(-1))
            self.K_axis = _f64(np.asarray(K_axis, np.float64).reshape(-1))
        self.B = _f64(B)
        self.dipolar = int(dipolar)

    @property
    def n_bonds(self):
        return len(self.b_a)

    def _args(self):
        lt = self.lat
        return (lt.n_sub, lt.L, lt.periodic, lt.cell, lt.frac, self.n_bonds, self.b_a, self.b_b,
                self.b_delta, self.b_J, self.n_aniso, self.K, self.K_axis, self.B, lt.mu,
                self.dipolar)


def shell_distances(lat: Lattice, n_max: int):
    out = np.zeros(n_max, np.float64)
    ns = lib().or_shell_distances(lat.n_sub, lat.cell, lat.frac, n_max, out)
    return out[:ns]


def field(model: Model, S, terms=False):
    """Total reduced field b (meV), shape (3, N); with terms=True also a dict
    of the bilinear, Zeeman, anisotropy and dipolar parts."""
    S = _f64(S)
    N = model.lat.N
    bt = np.zeros((3, N))
    parts = {k: np.zeros((3, N)) for k in ("bil", "zeeman", "aniso", "dip")} if terms else None
    lib().or_field(*model._args(), S, _ptr(bt),
                   *(_ptr(parts[k]) if terms else None for k in ("bil", "zeeman", "aniso", "dip")))
    return (bt, parts) if terms else bt


def energy(model: Model, S):
    """Energy terms [bilinear, Zeeman, anisotropy, dipolar, total] (meV)."""
    out = np.zeros(5)
    lib().or_energy(*model._args(), _f64(S), out)
    return out


def bruteforce(model: Model, S):
    """(b_bil, E_pair) from an O(N^2) sum over all pairs and periodic images,
    with couplings looked up by distance (no bond table)."""
    lt = model.lat
    N = lt.N
    b = np.zeros((3, N))
    E = np.zeros(1)
    lib().or_bruteforce(lt.n_sub, lt.L, lt.periodic, lt.cell, lt.frac, model.n_shells,
                        model.J_shell, _ptr(model.D_shell), _f64(S), b, _ptr(E))
    return b, float(E[0])


def dipolar_direct(lat: Lattice, S, targets):
    """Direct open-boundary dipolar field (meV) at the listed site indices."""
    t = np.ascontiguousarray(targets, dtype=np.int64)
    out = np.zeros((len(t), 3))
    lib().or_dipolar_direct(lat.n_sub, lat.L, lat.cell, lat.frac, lat.mu, _f64(S), len(t), t, out)
    return out.T.copy()


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.ascontiguousarray(ctr, np.uint32), np.ascontiguousarray(key, np.uint32), out)
    return out


def thermal_eta(seed, step, N, tag=0):
    eta = np.zeros((3, N))
    lib().or_thermal_eta(seed, step, tag, N, eta)
    return eta


def heun(model: Model, S, alpha, dt_fs, T_K=0.0, seed=0, step0=0, n_steps=1, tag=0, site0=0):
    """n_steps normalised Heun steps (FP64) from S; returns the new state.
    site0 offsets the noise counters (a block of a larger lattice)."""
    S = _f64(S).copy()
    lib().or_heun(*model._args(), float(alpha), float(dt_fs), float(T_K), int(seed), int(step0),
                  int(tag), int(site0), int(n_steps), S)
    return S


def image_distance(A, B):
    A, B = _f64(A), _f64(B)
    return lib().or_image_distance(A.shape[-1], A, B)


def geodesic_path(SA, SB, n_img):
    SA, SB = _f64(SA), _f64(SB)
    N = SA.shape[-1]
    out = np.zeros((n_img, 3, N))
    lib().or_geodesic_path(N, SA, SB, n_img, out)
    return out


def mc_colouring(model: Model, cmax: int = 64):
    """(C, coef) of the Monte Carlo colouring (x + ky y + kz z + o_a) mod C:
    coef = (ky, kz, o_0 .. o_{n_sub-1}); C = 0 if none with C <= cmax."""
    lt = model.lat
    coef = np.zeros(2 + lt.n_sub, np.int32)
    Cn = lib().or_mc_colouring(lt.n_sub, lt.L, lt.periodic, lt.cell, lt.frac, model.n_bonds, model.b_a,
                               model.b_b, model.b_delta, model.b_J, int(cmax), coef)
    return Cn, coef


def mc_sweeps(model: Model, S, T_K, seed, sweep0=0, n_sweeps=1, method=0, colouring=None):
    """n_sweeps heat-bath (method 0) or Metropolis (method 1) sweeps of S in
    place; returns the number of accepted moves (-1: unsupported case)."""
    if colouring is None:
        colouring = mc_colouring(model)
    Cn, coef = colouring
    coef = _i32(coef)
    return lib().or_mc_sweeps(*model._args(), S, float(T_K), int(seed), int(sweep0), int(n_sweeps), int(method),
                              int(Cn), coef)


MIN_METHODS = {"vp": 0, "bb": 1, "lbfgs": 2, "adam": 3}
RETRACTIONS = {"exp": 0, "norm": 1}


class MinState:
    """State of a static minimiser run (velocities, moments, previous step and
    force, L-BFGS history); zero at the start."""

    def __init__(self, N, method="vp", retraction="exp", dt=0.1, mass=1.0, hist=5, beta1=0.9, beta2=0.999,
                 eps=1e-8, max_step=0.0):
        self.method = MIN_METHODS[method] if isinstance(method, str) else int(method)
        self.retraction = RETRACTIONS[retraction] if isinstance(retraction, str) else int(retraction)
        self.dt, self.mass, self.hist = float(dt), float(mass), int(hist)
        self.beta1, self.beta2, self.eps, self.max_step = float(beta1), float(beta2), float(eps), float(max_step)
        self.work = np.zeros((4 + 2 * self.hist) * 3 * N + self.hist)
        self.ist = np.zeros(3, dtype=np.int64)


def min_iterate(model: Model, S, st: MinState):
    """One minimiser iteration of S in place; returns max |F| before the update."""
    mf = C.c_double(0.0)
    lib().or_min_iterate(*model._args(), S, st.method, st.retraction, st.dt, st.mass, st.hist, st.beta1,
                         st.beta2, st.eps, st.max_step, st.work, st.ist, C.byref(mf))
    return mf.value


class PairList:
    """Explicit couplings (pair-list backend): targets i, sources j, J per entry
    (scalar, or [n][3][3] when tensor), per-site moments mu (None: 1),
    per-site uniaxial anisotropy K with unit axes (None: none), field B (T)."""

    def __init__(self, n_sites, i, j, J, mu=None, K=None, K_axis=None, B=(0.0, 0.0, 0.0)):
        self.N = int(n_sites)
        self.i = np.ascontiguousarray(i, dtype=np.int64)
        self.j = np.ascontiguousarray(j, dtype=np.int64)
        J = np.asarray(J, dtype=np.float64)
        self.tensor = 1 if J.ndim == 3 else 0
        self.J = np.ascontiguousarray(J.reshape(len(self.i), 9) if self.tensor else J)
        self.mu = None if mu is None else _f64(mu)
        self.K = None if K is None else _f64(K)
        self.K_axis = None if K_axis is None else _f64(K_axis)
        self.B = _f64(B)

    def _args(self):
        return (self.N, len(self.i), self.i, self.j, self.J, self.tensor, _ptr(self.mu), _ptr(self.K),
                _ptr(self.K_axis), self.B)


def pl_field(pl: PairList, S):
    S = _f64(S)
    b = np.zeros_like(S)
    lib().or_pl_field(*pl._args(), S, b)
    return b


def pl_energy(pl: PairList, S):
    S = _f64(S)
    t = np.zeros(5)
    lib().or_pl_energy(*pl._args(), S, t)
    return t


def pl_heun(pl: PairList, S, alpha, dt_fs, T_K=0.0, seed=0, step0=0, tag=0, n_steps=1):
    S = _f64(S).copy()
    lib().or_pl_heun(*pl._args(), float(alpha), float(dt_fs), float(T_K), int(seed), int(step0), int(tag),
                     int(n_steps), S)
    return S


def reparametrize(Y, alpha=None):
    """The path Y [n_img][3][N] moved along the geodesic reaction coordinate to
    the arc-length fractions alpha (None: equal spacing); end images kept."""
    Y = _f64(Y)
    out = np.zeros_like(Y)
    a = None if alpha is None else _f64(alpha)
    lib().or_reparametrize(Y.shape[-1], Y.shape[0], Y, _ptr(a), out)
    return out


class GnebState:
    """Images, velocities and the climbing-image switch of one GNEB path
    (ci_mode 4: string method with target arc-length fractions alpha)."""

    def __init__(self, images, k_spring=1.0, dt=0.1, mass=1.0, ci_mode=1, ci_on_below=1e-2, alpha=None):
        self.Y = _f64(images).copy()
        self.V = np.zeros_like(self.Y)
        self.k, self.dt, self.mass = k_spring, dt, mass
        self.ci_mode, self.ci_on_below = ci_mode, ci_on_below
        self.ci_on = C.c_int(0)
        self.alpha = None if alpha is None else _f64(alpha)


def gneb_iterate(model: Model, st: GnebState):
    """One GNEB + VP iteration in place; returns (E, dist, max_force, ci_index)."""
    lt = model.lat
    n_img = st.Y.shape[0]
    E = np.zeros(n_img)
    dist = np.zeros(max(n_img - 1, 1))
    mf = C.c_double(0.0)
    ci = C.c_int(-1)
    args = model._args()[:-1]
    lib().or_gneb_iterate(*args, n_img, st.Y, st.V, st.k, st.dt, st.mass, st.ci_mode,
                          st.ci_on_below, C.byref(st.ci_on), _ptr(st.alpha), E, dist, C.byref(mf),
                          C.byref(ci))
    return E, dist[:n_img - 1], mf.value, ci.value


# ---------------------------------------------------------------- learned net
NET_CHANNELS = (10, 16, 16, 16, 3)


def net_nparams(ch=NET_CHANNELS):
    return lib().or_net_nparams(_i32(ch))


def net_forward(L, params, x, ch=NET_CHANNELS, want_act=False, dil=(1, 1, 1, 1), bf16=False):
    """Raw net output [c4][P] (and the pre-activations of every layer with
    want_act) for input x [c0][P] on an L grid; dil: per-layer dilation;
    bf16: every layer's weights and inputs rounded to float and then to
    bfloat16 (nearest even) before an FP64 convolution."""
    Lx, Ly, Lz = (int(v) for v in L)
    P = Lx * Ly * Lz
    out = np.zeros((ch[4], P))
    act = np.zeros((sum(ch[1:]), P)) if want_act else None
    lib().or_net_forward_q(Lx, Ly, Lz, _i32(ch), _i32(dil), _f64(params), _f64(x), out, _ptr(act), int(bool(bf16)))
    return (out, act) if want_act else out


def net_predict_loss(raw, Sg, Sstar=None):
    raw, Sg = _f64(raw), _f64(Sg)
    P = Sg.shape[-1]
    shat = np.zeros((3, P))
    Ss = None if Sstar is None else _f64(Sstar)
    loss = lib().or_net_predict_loss(P, raw, Sg, _ptr(Ss), _ptr(shat))
    return shat, loss


def net_backward(L, params, x, Sg, Sstar, ch=NET_CHANNELS, dil=(1, 1, 1, 1)):
    Lx, Ly, Lz = (int(v) for v in L)
    g = np.zeros(net_nparams(ch))
    loss = lib().or_net_backward(Lx, Ly, Lz, _i32(ch), _i32(dil), _f64(params), _f64(x), _f64(Sg),
                                 _f64(Sstar), g)
    return loss, g


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    lib().or_adam(len(w), w, _f64(g), m, v, int(t), lr, b1, b2, eps)
