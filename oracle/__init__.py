"""Python driver for the FP64 CPU oracle (``afm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, single-threaded FP64 statement of the
dynamic-AFM force inversion of Busch, Zou and Ganapathysubramanian (arXiv 1109.0334); it checks the
GPU library and is never called by it.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It imports nothing from the GPU package.

Functions take a model ``dict`` (keys of :data:`MODEL_FIELDS`, SI units) and full parameter
vectors ``p`` whose entry 0 is the separation z_c (law layouts in :data:`LAW_PARAMS`).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "afm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

MAX_MODES = 8
MAX_PARAMS = 12
LAW = {"dmt": 0, "lj": 1, "kv": 2, "hooke": 3, "sd": 4, "none": 5}
LAW_PARAMS = {
    "dmt": ("zc", "H", "Estar", "a0", "R"),
    "lj": ("zc", "eps", "r0", "n", "m"),
    "kv": ("zc", "H", "Estar", "a0", "R", "eta"),
    "hooke": ("zc", "ks"),
    "sd": ("zc", "ks", "zeta_s"),
    "none": ("zc",),
}
ST_NONFINITE, ST_DIVERGED = 1, 2
IC = {"free_steady": 0, "rest": 1}


class _Model(C.Structure):
    _fields_ = [
        ("n_modes", C.c_int32), ("law", C.c_int32), ("steps_per_cycle", C.c_int32),
        ("n_cycles", C.c_int32), ("lockin_cycles", C.c_int32), ("ic", C.c_int32),
        ("k", C.c_double), ("f0", C.c_double), ("drive_freq", C.c_double),
        ("free_amplitude", C.c_double), ("div_limit", C.c_double),
        ("q", C.c_double * MAX_MODES), ("ratio", C.c_double * MAX_MODES),
        ("gain", C.c_double * MAX_MODES), ("drive_mode", C.c_int32),
    ]


MODEL_FIELDS = ("n_modes", "law", "steps_per_cycle", "n_cycles", "lockin_cycles", "ic", "k", "f0",
                "drive_freq", "free_amplitude", "div_limit", "q", "ratio", "gain", "drive_mode")
DRIVE = {"table": 0, "params": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", _SRC,
                        "-lm", "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, ip, mp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(_Model)
        u32p = C.POINTER(C.c_uint32)
        L.orc_trajectory.argtypes = [mp, dp, C.c_int32, dp, C.c_int64, dp, dp, dp]
        L.orc_trajectory.restype = C.c_int
        L.orc_forward.argtypes = [mp, dp, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_forward.restype = C.c_int
        L.orc_forward_points.argtypes = [mp, dp, C.c_int32, C.c_int32, dp, dp, dp, dp]
        L.orc_forward_steady.argtypes = [mp, dp, C.c_int32, C.c_double, dp, dp, dp, dp, dp, ip]
        L.orc_forward_steady.restype = C.c_int
        L.orc_forward_points.restype = C.c_int
        L.orc_lockin.argtypes = [dp, C.c_int64, C.c_int32, C.c_int64, dp, dp]
        L.orc_misfit.argtypes = [dp, dp, C.c_int64]
        L.orc_misfit.restype = C.c_double
        L.orc_base_amplitude.argtypes = [mp]
        L.orc_base_amplitude.restype = C.c_double
        L.orc_initial_state.argtypes = [mp, dp]
        L.orc_force.argtypes = [C.c_int, dp, C.c_double, C.c_double]
        L.orc_force.restype = C.c_double
        L.orc_steady_amplitude.argtypes = [mp, dp, C.c_int32, C.c_double, ip]
        L.orc_steady_amplitude.restype = C.c_double
        L.orc_zc_from_setpoint.argtypes = [mp, dp, C.c_double, C.c_int32, C.c_double, C.c_double]
        L.orc_zc_from_setpoint.restype = C.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_draw.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               u32p]
        L.orc_pso_init.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_uint64, dp, dp, dp, dp,
                                   dp, dp, ip]
        L.orc_pso_update.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, C.c_int32,
                                     C.c_uint64, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, dp, dp, dp, dp, dp, dp, ip]
        L.orc_z_to_theta.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_z_to_theta.restype = C.c_double
        L.orc_dtheta_dz.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_dtheta_dz.restype = C.c_double
        L.orc_misfit_grad.argtypes = [mp, dp, C.c_int32, dp, dp, dp]
        L.orc_misfit_grad.restype = C.c_int
        L.orc_pso_invert.argtypes = [mp, dp, C.c_int32, ip, dp, dp, ip, dp, C.c_int32, C.c_int32,
                                     C.c_uint64, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, dp, dp, ip, dp]
        L.orc_lbfgs.argtypes = [mp, dp, C.c_int32, ip, dp, dp, ip, dp, dp, C.c_int32]
        L.orc_lbfgs.restype = C.c_double
        L.orc_eb_shape.argtypes = [C.c_double, C.c_double]
        L.orc_eb_shape.restype = C.c_double
        L.orc_eb_root.argtypes = [C.c_int32]
        L.orc_eb_root.restype = C.c_double
        L.orc_eb_modes.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp]
        L.orc_law_param_count.argtypes = [C.c_int]
        L.orc_law_param_count.restype = C.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------------------------
# marshalling helpers


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def make_model(m: dict) -> _Model:
    s = _Model()
    law = m["law"]
    s.law = LAW[law] if isinstance(law, str) else int(law)
    ic = m.get("ic", 0)
    s.ic = IC[ic] if isinstance(ic, str) else int(ic)
    s.n_modes = int(m.get("n_modes", 1))
    for f in ("steps_per_cycle", "n_cycles", "lockin_cycles"):
        setattr(s, f, int(m[f]))
    for f in ("k", "f0", "free_amplitude"):
        setattr(s, f, float(m[f]))
    s.drive_freq = float(m.get("drive_freq", m["f0"]))
    s.div_limit = float(m.get("div_limit", 100.0))
    nm = s.n_modes
    q = list(m.get("q", [400.0] * nm))
    ratio = list(m.get("ratio", [1.0] * nm))
    gain = list(m.get("gain", [1.0] * nm))
    for i in range(nm):
        s.q[i], s.ratio[i], s.gain[i] = q[i], ratio[i], gain[i]
    drive = m.get("drive", "table")
    s.drive_mode = DRIVE[drive] if isinstance(drive, str) else int(drive)
    return s


def _pv(p):
    """Parameter vector padded to MAX_PARAMS entries (law parameters first; with the "params"
    drive the base motion a, f, g at 8, 9, 10)."""
    v = np.zeros(MAX_PARAMS)
    p = np.asarray(p, dtype=np.float64).ravel()
    v[: len(p)] = p
    return v


def window_len(m: dict) -> int:
    return int(m["lockin_cycles"]) * int(m["steps_per_cycle"])


def law_id(m: dict) -> int:
    return LAW[m["law"]] if isinstance(m["law"], str) else int(m["law"])


def nparams(m: dict) -> int:
    return lib().orc_law_param_count(law_id(m))


# --------------------------------------------------------------------------------------------
# forward problem


def trajectory(m: dict, p, n_cycles=None, y0=None, n_out=None, want_rate=False):
    """Tip deflection u_n (and rate) for the last ``n_out`` states; returns (status, u, ud, y_end)."""
    L, mo = lib(), make_model(m)
    nc = int(m["n_cycles"] if n_cycles is None else n_cycles)
    n_out = window_len(m) if n_out is None else int(n_out)
    p = _pv(p)
    u = np.empty(n_out)
    ud = np.empty(n_out) if want_rate else None
    yend = np.empty(2 * mo.n_modes)
    y0a = None if y0 is None else _f64(y0)
    st = L.orc_trajectory(C.byref(mo), _dp(p), nc, _dp(y0a), n_out, _dp(u), _dp(ud), _dp(yend))
    return st, u, ud, yend


def forward(m: dict, p, target=None, n_cycles=None, want_trace=False):
    """One forward solve: dict(status, A, phi, J, trace)."""
    L, mo = lib(), make_model(m)
    nc = int(m["n_cycles"] if n_cycles is None else n_cycles)
    p = _pv(p)
    U = None if target is None else _f64(target)
    A, phi, J = C.c_double(), C.c_double(), C.c_double()
    tr = np.empty(window_len(m)) if want_trace else None
    st = L.orc_forward(C.byref(mo), _dp(p), nc, _dp(U), C.byref(A), C.byref(phi), C.byref(J),
                       _dp(tr))
    return {"status": st, "A": A.value, "phi": phi.value, "J": J.value, "trace": tr}


def forward_steady(m: dict, p, rtol, target=None, n_cycles=None, want_trace=False):
    """Forward solve with the adaptive steady-state exit: dict(status, A, phi, J, trace,
    periods); n_cycles (default the model's) is the cap on the periods integrated."""
    L, mo = lib(), make_model(m)
    nc = int(m["n_cycles"] if n_cycles is None else n_cycles)
    U = None if target is None else _f64(target)
    A, phi, J = C.c_double(), C.c_double(), C.c_double()
    per = np.zeros(1, np.int32)
    tr = np.empty(window_len(m)) if want_trace else None
    st = L.orc_forward_steady(C.byref(mo), _dp(_pv(p)), nc, float(rtol), _dp(U), C.byref(A),
                              C.byref(phi), C.byref(J), _dp(tr), _ip(per))
    return {"status": st, "A": A.value, "phi": phi.value, "J": J.value, "trace": tr,
            "periods": int(per[0])}


def forward_points(m: dict, p, weights, n_cycles=None, want_trace=False):
    """Deflection at points along the beam: weights [n_pts][n_modes] (Phi_i(x_k) / Phi_i(L));
    returns dict(status, A [n_pts], phi [n_pts], trace [n_pts][W] or None)."""
    L, mo = lib(), make_model(m)
    nc = int(m["n_cycles"] if n_cycles is None else n_cycles)
    w = np.ascontiguousarray(np.atleast_2d(np.asarray(weights, dtype=np.float64)))
    assert w.shape[1] == mo.n_modes
    k = w.shape[0]
    A, phi = np.empty(k), np.empty(k)
    tr = np.empty((k, window_len(m))) if want_trace else None
    st = L.orc_forward_points(C.byref(mo), _dp(_pv(p)), nc, k, _dp(w), _dp(A), _dp(phi), _dp(tr))
    return {"status": st, "A": A, "phi": phi, "trace": tr}


def forward_batch(m: dict, P, targets=None, target_id=None, n_cycles=None):
    """Forward solves for every row of P ([n][nparams]); returns arrays A, phi, J, status."""
    P = np.atleast_2d(_f64(P))
    n = P.shape[0]
    A, phi, J, st = np.empty(n), np.empty(n), np.empty(n), np.empty(n, np.int32)
    for i in range(n):
        U = None
        if targets is not None:
            t = 0 if target_id is None else int(target_id[i])
            U = np.atleast_2d(targets)[t]
        nc = None if n_cycles is None else int(np.atleast_1d(n_cycles)[i])
        r = forward(m, P[i], U, n_cycles=nc)
        A[i], phi[i], J[i], st[i] = r["A"], r["phi"], r["J"], r["status"]
    return A, phi, J, st


def lockin(u, N: int, p0: int = 1):
    u = _f64(u)
    A, phi = C.c_double(), C.c_double()
    lib().orc_lockin(_dp(u), len(u), int(N), int(p0), C.byref(A), C.byref(phi))
    return A.value, phi.value


def misfit(U, u) -> float:
    U, u = _f64(U), _f64(u)
    return lib().orc_misfit(_dp(U), _dp(u), len(U))


def base_amplitude(m: dict) -> float:
    mo = make_model(m)
    return lib().orc_base_amplitude(C.byref(mo))


def initial_state(m: dict):
    mo = make_model(m)
    y = np.empty(2 * mo.n_modes)
    lib().orc_initial_state(C.byref(mo), _dp(y))
    return y


def force(m: dict, p, d: float, dd: float = 0.0) -> float:
    p = _pv(p)
    return lib().orc_force(law_id(m), _dp(p), float(d), float(dd))


def steady_amplitude(m: dict, p, max_cycles=4000, rtol=1e-10):
    p = _pv(p)
    used = C.c_int32()
    mo = make_model(m)
    A = lib().orc_steady_amplitude(C.byref(mo), _dp(p), int(max_cycles), float(rtol),
                                   C.byref(used))
    return A, used.value


def zc_from_setpoint(m: dict, p, setpoint: float, max_cycles=4000, rtol=1e-10, tol=1e-9):
    p = _pv(p)
    mo = make_model(m)
    return lib().orc_zc_from_setpoint(C.byref(mo), _dp(p), float(setpoint), int(max_cycles),
                                      float(rtol), float(tol))


def misfit_grad(m: dict, p, target, n_cycles=None):
    """(status, J, dJ/dp) with the gradient over every entry of the full parameter vector."""
    L, mo = lib(), make_model(m)
    nc = int(m["n_cycles"] if n_cycles is None else n_cycles)
    n = len(np.atleast_1d(p))
    p, U = _pv(p), _f64(target)
    J = C.c_double()
    g = np.empty(MAX_PARAMS)
    st = L.orc_misfit_grad(C.byref(mo), _dp(p), nc, _dp(U), C.byref(J), _dp(g))
    return st, J.value, g[:n].copy()


# --------------------------------------------------------------------------------------------
# random numbers and PSO


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


def u53(a: int, b: int) -> float:
    return lib().orc_u53(a, b)


def draw(seed, swarm, it, particle, dim, purpose):
    o = (C.c_uint32 * 4)()
    lib().orc_draw(int(seed), int(swarm), int(it), int(particle), int(dim), int(purpose), o)
    return tuple(o)


PSO_DEFAULTS = {"w": 0.7298, "c1": 1.49618, "c2": 1.49618, "vmax": 1.0}


class Swarm:
    """Swarm state in the library's structure-of-arrays layout ([D][S*P], [S*P], [D][S], [S])."""

    def __init__(self, D, P, S, seed):
        self.D, self.P, self.S, self.seed = D, P, S, int(seed)
        n = S * P
        self.z, self.v, self.pbest_z = np.empty((D, n)), np.empty((D, n)), np.empty((D, n))
        self.pbest_J, self.gbest_z = np.empty(n), np.empty((D, S))
        self.gbest_J, self.gen_to_cutoff = np.empty(S), np.empty(S, np.int32)
        lib().orc_pso_init(D, P, S, self.seed, _dp(self.z), _dp(self.v), _dp(self.pbest_z),
                           _dp(self.pbest_J), _dp(self.gbest_z), _dp(self.gbest_J),
                           _ip(self.gen_to_cutoff))

    def update(self, J, it, is_last, cutoff=0.0, **pso):
        c = dict(PSO_DEFAULTS, **pso)
        J = _f64(J)
        lib().orc_pso_update(self.D, self.P, self.S, _dp(J), int(it), int(bool(is_last)),
                             self.seed, float(cutoff), c["w"], c["c1"], c["c2"], c["vmax"],
                             _dp(self.z), _dp(self.v), _dp(self.pbest_z), _dp(self.pbest_J),
                             _dp(self.gbest_z), _dp(self.gbest_J), _ip(self.gen_to_cutoff))


def z_to_theta(z, lo, hi, log_scale) -> float:
    return lib().orc_z_to_theta(float(z), float(lo), float(hi), int(bool(log_scale)))


def dtheta_dz(z, lo, hi, log_scale) -> float:
    return lib().orc_dtheta_dz(float(z), float(lo), float(hi), int(bool(log_scale)))


def _free_spec(free):
    idx = np.asarray([f[0] for f in free], np.int32)
    lo = _f64([f[1] for f in free])
    hi = _f64([f[2] for f in free])
    lg = np.asarray([int(bool(f[3])) for f in free], np.int32)
    return idx, lo, hi, lg


def pso_invert(m: dict, p_fixed, free, target, P, T, seed, cutoff=0.0, **pso):
    """Single-swarm PSO inversion; free = [(index, lo, hi, log_scale), ...]."""
    c = dict(PSO_DEFAULTS, **pso)
    mo = make_model(m)
    idx, lo, hi, lg = _free_spec(free)
    D = len(idx)
    bz, bJ, gen = np.empty(D), C.c_double(), C.c_int32()
    hist = np.empty(T)
    pf, U = _pv(p_fixed), _f64(target)
    lib().orc_pso_invert(C.byref(mo), _dp(pf), D, _ip(idx), _dp(lo), _dp(hi), _ip(lg), _dp(U),
                         int(P), int(T), int(seed), float(cutoff), c["w"], c["c1"], c["c2"],
                         c["vmax"], _dp(bz), C.byref(bJ), C.byref(gen), _dp(hist))
    return {"z": bz, "J": bJ.value, "gen_to_cutoff": gen.value, "hist": hist}


def lbfgs(m: dict, p_fixed, free, target, z0, steps):
    mo = make_model(m)
    idx, lo, hi, lg = _free_spec(free)
    z = _f64(z0).copy()
    pf, U = _pv(p_fixed), _f64(target)
    J = lib().orc_lbfgs(C.byref(mo), _dp(pf), len(idx), _ip(idx), _dp(lo), _dp(hi), _ip(lg),
                        _dp(U), _dp(z), int(steps))
    return z, J


# --------------------------------------------------------------------------------------------
# Euler-Bernoulli modes


def eb_root(i: int) -> float:
    return lib().orc_eb_root(int(i))


def eb_shape(bL: float, xi: float) -> float:
    return lib().orc_eb_shape(float(bL), float(xi))


def eb_modes(n: int, npts: int = 501):
    bL, ratio, mass, gain = (np.empty(n) for _ in range(4))
    lib().orc_eb_modes(int(n), int(npts), _dp(bL), _dp(ratio), _dp(mass), _dp(gain))
    return {"betaL": bL, "ratio": ratio, "mass": mass, "gain": gain}
