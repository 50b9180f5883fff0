"""MI355X tip-sample force inversion (dynamic AFM), Python binding of libafm.so.

The binding only marshals arguments: torch tensors provide device memory and the current HIP
stream, every computation runs in the library's HIP kernels.  Names follow the C ABI in
``include/afm.h``:

* :meth:`Plan.forward_batch` -- FP of Sec. 2.2: lock-in amplitude/phase (and window trace) of a
  batch of parameter points;
* :meth:`Plan.misfit` -- the cost J of Eq. 5 on the lock-in window against measured traces;
* :meth:`Plan.swarm_init`, :meth:`Plan.pso_step` -- the particle swarm of Sec. 3.4 (Eq. 8);
* :meth:`Plan.invert` -- whole inversions (IP of Sec. 2.3) replayed as one HIP graph.

There is no CPU fallback: if the library is missing or cannot be loaded, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafm.so")

MAX_MODES = 8
MAX_PARAMS = 12
PREC = {"mixed": 0, "fp64": 1}
LAW = {"dmt": 0, "lj": 1, "kv": 2, "hooke": 3, "sd": 4, "none": 5}
LAW_PARAMS = {
    "dmt": ("zc", "H", "Estar", "a0", "R"),
    "lj": ("zc", "eps", "r0", "n", "m"),
    "kv": ("zc", "H", "Estar", "a0", "R", "eta"),
    "hooke": ("zc", "ks"),
    "sd": ("zc", "ks", "zeta_s"),
    "none": ("zc",),
}
IC = {"free_steady": 0, "rest": 1}
DRIVE = {"table": 0, "params": 1}
P_BASE_A, P_BASE_F, P_BASE_G = 8, 9, 10  # base-motion slots of a "params" drive
POLISH = {"plan": 0, "mixed": 1, "fp64": 2}
GRAD_FORM = {"auto": 0, "sweep": 1, "segments": 2}
ST_NONFINITE, ST_DIVERGED, ST_BAD_INPUT = 1, 2, 4
EXPORTS = ("afm_plan_create", "afm_plan_destroy", "afm_set_launch_shape", "afm_forward_batch",
           "afm_misfit",
           "afm_grad_batch", "afm_polish", "afm_swarm_init", "afm_pso_step", "afm_invert",
           "afm_forward_steady", "afm_forward_points", "afm_beam_modes", "afm_beam_shapes", "afm_last_error",
           "afm_version", "afm_grad_batch_noalloc", "afm_separations",
           "afm_misfit_swarms", "afm_set_grad_form")


class AfmError(RuntimeError):
    pass


class _Problem(C.Structure):
    _fields_ = [
        ("n_modes", C.c_int32), ("law", C.c_int32), ("steps_per_cycle", C.c_int32),
        ("n_cycles", C.c_int32), ("lockin_cycles", C.c_int32), ("ic", C.c_int32),
        ("k", C.c_double), ("f0", C.c_double), ("drive_freq", C.c_double),
        ("free_amplitude", C.c_double), ("div_limit", C.c_double),
        ("q", C.c_double * MAX_MODES), ("ratio", C.c_double * MAX_MODES),
        ("gain", C.c_double * MAX_MODES),
        ("params", C.c_double * MAX_PARAMS), ("n_free", C.c_int32),
        ("free_index", C.c_int32 * MAX_PARAMS), ("lo", C.c_double * MAX_PARAMS),
        ("hi", C.c_double * MAX_PARAMS), ("log_scale", C.c_int32 * MAX_PARAMS),
        ("pso_w", C.c_double), ("pso_c1", C.c_double), ("pso_c2", C.c_double),
        ("pso_vmax", C.c_double), ("polish_precision", C.c_int32), ("drive_mode", C.c_int32),
        ("steady_rtol", C.c_double),
    ]


class _Swarm(C.Structure):
    _fields_ = [
        ("n_dim", C.c_int32), ("particles", C.c_int32), ("swarms", C.c_int32),
        ("z", C.c_void_p), ("v", C.c_void_p), ("pbest_z", C.c_void_p), ("pbest_J", C.c_void_p),
        ("gbest_z", C.c_void_p), ("gbest_J", C.c_void_p), ("gen_to_cutoff", C.c_void_p),
        ("theta", C.c_void_p),
    ]


_lib = None


def lib() -> C.CDLL:
    """Load libafm.so (built in-tree by ``paper_1109_0334_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise AfmError(f"{LIB_PATH} is missing: build it with python -m paper_1109_0334_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    L.afm_plan_create.argtypes = [C.POINTER(_Problem), i32, C.POINTER(vp)]
    L.afm_plan_destroy.argtypes = [vp]
    L.afm_set_launch_shape.argtypes = [vp, i32, i32]
    L.afm_set_grad_form.argtypes = [vp, i32]
    L.afm_forward_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.afm_misfit.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp, vp, vp]
    L.afm_grad_batch.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp, vp, i32, vp, vp]
    L.afm_grad_batch_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp, vp, i32, vp, vp]
    L.afm_swarm_init.argtypes = [vp, C.POINTER(_Swarm), u64, vp]
    L.afm_pso_step.argtypes = [vp, C.POINTER(_Swarm), vp, u64, i32, i32, dbl, vp]
    L.afm_polish.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, i32, vp, vp]
    L.afm_invert.argtypes = [vp, i32, vp, vp, vp, i32, i32, u64, dbl, i32, i32, vp, vp, vp, vp]
    L.afm_separations.argtypes = [vp, i32, vp, vp, i32, i32, dbl, i32, vp, vp]
    L.afm_beam_modes.argtypes = [i32, i32, dbl, dbl, dbl, dbl, vp, vp, vp]
    L.afm_beam_shapes.argtypes = [i32, i32, vp, vp]
    L.afm_forward_points.argtypes = [vp, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp]
    L.afm_forward_steady.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.afm_misfit_swarms.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.afm_last_error.restype = C.c_char_p
    L.afm_version.restype = C.c_char_p
    for f in ("afm_plan_create", "afm_plan_destroy", "afm_forward_batch", "afm_misfit",
              "afm_grad_batch", "afm_grad_batch_noalloc", "afm_polish", "afm_swarm_init", "afm_pso_step", "afm_invert",
              "afm_beam_modes", "afm_beam_shapes", "afm_forward_points", "afm_forward_steady",
              "afm_separations", "afm_misfit_swarms"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(code: int, what: str):
    if code != 0:
        msg = lib().afm_last_error().decode()
        raise AfmError(f"{what} failed (status {code}): {msg}")


def beam_modes(n_modes: int, n_points: int = 501, E=0.0, I=0.0, mu=0.0, L=0.0) -> dict:
    """Clamped-free Euler-Bernoulli modes (afm_beam_modes, host only): frequency ratios, base-drive
    gains of the tip-normalised modes and, from the beam's properties, the first frequency."""
    ratio, gain, f1 = (C.c_double * n_modes)(), (C.c_double * n_modes)(), C.c_double()
    _check(lib().afm_beam_modes(int(n_modes), int(n_points), float(E), float(I), float(mu),
                                float(L), ratio, gain, C.byref(f1)), "afm_beam_modes")
    return {"ratio": list(ratio), "gain": list(gain), "f1": f1.value}


def beam_shapes(n_modes: int, x) -> np.ndarray:
    """Tip-normalised clamped-free mode shapes at x (units of L): [len(x)][n_modes] weights for
    Plan.forward_points (afm_beam_shapes, host only)."""
    x = np.ascontiguousarray(np.atleast_1d(np.asarray(x, dtype=np.float64)))
    w = np.empty((x.size, int(n_modes)))
    _check(lib().afm_beam_shapes(int(n_modes), x.size, x.ctypes.data, w.ctypes.data),
           "afm_beam_shapes")
    return w


def make_problem(model: dict, params, free=(), pso=None, polish="plan") -> _Problem:
    """afm_problem from a model dict (SI; keys as in ``workloads``; ``drive`` "table" or
    "params"), the full parameter vector (the law's, and with a "params" drive the base motion's
    a, f, g at slots 8, 9, 10) and the free-parameter spec [(index, lo, hi, log_scale), ...]."""
    p = _Problem()
    law = model["law"]
    p.law = LAW[law] if isinstance(law, str) else int(law)
    ic = model.get("ic", "free_steady")
    p.ic = IC[ic] if isinstance(ic, str) else int(ic)
    drive = model.get("drive", "table")
    p.drive_mode = DRIVE[drive] if isinstance(drive, str) else int(drive)
    p.steady_rtol = float(model.get("steady_rtol", 0.0))
    p.n_modes = int(model.get("n_modes", 1))
    p.steps_per_cycle = int(model["steps_per_cycle"])
    p.n_cycles = int(model["n_cycles"])
    p.lockin_cycles = int(model["lockin_cycles"])
    p.k, p.f0 = float(model["k"]), float(model["f0"])
    p.drive_freq = float(model.get("drive_freq", model["f0"]))
    p.free_amplitude = float(model["free_amplitude"])
    p.div_limit = float(model.get("div_limit", 100.0))
    nm = p.n_modes
    for i, (q, r, g) in enumerate(zip(model.get("q", [400.0] * nm), model.get("ratio", [1.0] * nm),
                                      model.get("gain", [1.0] * nm))):
        if i < nm:
            p.q[i], p.ratio[i], p.gain[i] = float(q), float(r), float(g)
    for j, v in enumerate(np.asarray(params, dtype=np.float64)):
        p.params[j] = float(v)
    p.n_free = len(free)
    for j, (idx, lo, hi, lg) in enumerate(free):
        p.free_index[j], p.lo[j], p.hi[j], p.log_scale[j] = int(idx), float(lo), float(hi), int(bool(lg))
    pso = pso or {}
    p.pso_w, p.pso_c1 = float(pso.get("w", 0.0)), float(pso.get("c1", 0.0))
    p.pso_c2, p.pso_vmax = float(pso.get("c2", 0.0)), float(pso.get("vmax", 0.0))
    p.polish_precision = POLISH[polish]
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(x, device):
    import torch

    return torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x,
                           dtype=torch.float64, device=device).contiguous()


def _dev_i32(x, device):
    import torch

    if x is None:
        return None
    return torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x,
                           dtype=torch.int32, device=device).contiguous()


class Swarm:
    """Swarm state as device tensors in the library's structure-of-arrays layout."""

    def __init__(self, D, P, S, device):
        import torch

        n = S * P
        f = dict(dtype=torch.float64, device=device)
        self.D, self.P, self.S = D, P, S
        self.z, self.v, self.pbest_z = (torch.empty(D, n, **f) for _ in range(3))
        self.theta = torch.empty(D, n, **f)
        self.pbest_J = torch.empty(n, **f)
        self.gbest_z = torch.empty(D, S, **f)
        self.gbest_J = torch.empty(S, **f)
        self.gen_to_cutoff = torch.empty(S, dtype=torch.int32, device=device)

    def cstruct(self) -> _Swarm:
        s = _Swarm()
        s.n_dim, s.particles, s.swarms = self.D, self.P, self.S
        for f in ("z", "v", "pbest_z", "pbest_J", "gbest_z", "gbest_J", "gen_to_cutoff", "theta"):
            setattr(s, f, getattr(self, f).data_ptr())
        return s


class Plan:
    """An afm_plan: problem constants and tables resident on the current GPU."""

    def __init__(self, model: dict, params, free=(), precision="mixed", pso=None, device="cuda",
                 polish="plan"):
        import torch

        self.device = torch.device(device)
        self.model = dict(model)
        self.free = list(free)
        self.n_free = len(self.free)
        self.W = int(model["lockin_cycles"]) * int(model["steps_per_cycle"])
        self._prob = make_problem(model, params, self.free, pso, polish)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().afm_plan_create(C.byref(self._prob), PREC[precision], C.byref(h)),
                   "afm_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().afm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch_shape(self, block=0, tpl=1):
        """Pin the plain forward kernel's launch shape (block lanes, trajectories per lane);
        block=0 returns to autotuning."""
        _check(lib().afm_set_launch_shape(self._h, int(block), int(tpl)), "afm_set_launch_shape")

    def set_grad_form(self, form="auto"):
        """Pin the gradient form ("sweep" or "segments") or return to tuning ("auto")."""
        _check(lib().afm_set_grad_form(self._h, GRAD_FORM[form]), "afm_set_grad_form")

    def forward_batch(self, theta, n_cycles=None, trace=False):
        """theta [n_free][n] (SI) -> dict(amp [n] m, phase [n] rad, status [n], trace [n][W])."""
        import torch

        theta = _dev_f64(theta, self.device).reshape(self.n_free, -1) if self.n_free else \
            torch.empty(0, 1, dtype=torch.float64, device=self.device)
        n = theta.shape[1]
        amp = torch.empty(n, dtype=torch.float64, device=self.device)
        phase = torch.empty_like(amp)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        tr = torch.empty(n, self.W, dtype=torch.float64, device=self.device) if trace else None
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_forward_batch(self._h, n, _ptr(theta), _ptr(nc), _ptr(amp), _ptr(phase),
                                       _ptr(tr), _ptr(status), _stream()), "afm_forward_batch")
        return {"amp": amp, "phase": phase, "status": status, "trace": tr}

    def forward_steady(self, theta, n_cycles=None, trace=False):
        """forward_batch plus the periods each trajectory integrated (afm_forward_steady)."""
        import torch

        theta = _dev_f64(theta, self.device).reshape(self.n_free, -1) if self.n_free else \
            torch.empty(0, 1, dtype=torch.float64, device=self.device)
        n = theta.shape[1]
        amp = torch.empty(n, dtype=torch.float64, device=self.device)
        phase = torch.empty_like(amp)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        periods = torch.empty(n, dtype=torch.int32, device=self.device)
        tr = torch.empty(n, self.W, dtype=torch.float64, device=self.device) if trace else None
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_forward_steady(self._h, n, _ptr(theta), _ptr(nc), _ptr(amp), _ptr(phase),
                                        _ptr(tr), _ptr(status), _ptr(periods), _stream()),
               "afm_forward_steady")
        return {"amp": amp, "phase": phase, "status": status, "periods": periods, "trace": tr}

    def forward_points(self, theta, weights, n_cycles=None, trace=False):
        """Deflection at points along the beam: weights [n_points][n_modes] (host) ->
        dict(amp, phase [n_points][n], status [n], trace [n_points][n][W])."""
        import torch

        theta = _dev_f64(theta, self.device).reshape(self.n_free, -1) if self.n_free else \
            torch.empty(0, 1, dtype=torch.float64, device=self.device)
        n = theta.shape[1]
        w = np.ascontiguousarray(np.atleast_2d(np.asarray(weights, dtype=np.float64)))
        k = w.shape[0]
        amp = torch.empty(k, n, dtype=torch.float64, device=self.device)
        phase = torch.empty_like(amp)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        tr = torch.empty(k, n, self.W, dtype=torch.float64, device=self.device) if trace else None
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_forward_points(self._h, n, _ptr(theta), _ptr(nc), k, w.ctypes.data,
                                        _ptr(amp), _ptr(phase), _ptr(tr), _ptr(status),
                                        _stream()), "afm_forward_points")
        return {"amp": amp, "phase": phase, "status": status, "trace": tr}

    def misfit(self, theta, targets, target_id=None, n_cycles=None):
        """theta [n_free][n], targets [n_targets][W] (m) -> (J [n], status [n])."""
        theta = _dev_f64(theta, self.device).reshape(self.n_free, -1)
        n = theta.shape[1]
        targets = _dev_f64(targets, self.device).reshape(-1, self.W)
        import torch

        J = torch.empty(n, dtype=torch.float64, device=self.device)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        tid = _dev_i32(target_id, self.device)
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_misfit(self._h, n, _ptr(theta), _ptr(nc), _ptr(tid), _ptr(targets),
                                targets.shape[0], _ptr(J), _ptr(status), _stream()), "afm_misfit")
        return J, status

    def misfit_swarms(self, theta, targets, particles, n_cycles=None, swarm_params=None):
        """afm_misfit_swarms: S swarms of `particles` points (theta [n_free][S*P]) against
        target rows [S][W], per-swarm period counts [S] and parameter vectors [MAX_PARAMS][S]
        -> (J [S*P], status [S*P]).  Keep n_cycles the same tensor across calls to reuse the
        work-queue order."""
        import torch

        targets = _dev_f64(targets, self.device).reshape(-1, self.W)
        S = targets.shape[0]
        theta = _dev_f64(theta, self.device).reshape(self.n_free, S * int(particles))
        J = torch.empty(S * int(particles), dtype=torch.float64, device=self.device)
        status = torch.empty(S * int(particles), dtype=torch.int32, device=self.device)
        nc = n_cycles if (n_cycles is None or isinstance(n_cycles, torch.Tensor)) else \
            _dev_i32(n_cycles, self.device)
        sp = None if swarm_params is None else \
            _dev_f64(swarm_params, self.device).reshape(MAX_PARAMS, S)
        self._keep_ms = (targets, nc, sp)
        _check(lib().afm_misfit_swarms(self._h, S, int(particles), _ptr(theta), _ptr(nc), _ptr(sp),
                                       _ptr(targets), _ptr(J), _ptr(status), _stream()),
               "afm_misfit_swarms")
        return J, status

    def grad_batch(self, theta, targets, target_id=None, n_cycles=None, ckpt_stride=0):
        """Discrete-adjoint gradient: (J [n], dJ [n_free][n] per SI unit, status [n])."""
        import torch

        theta = _dev_f64(theta, self.device).reshape(self.n_free, -1)
        n = theta.shape[1]
        targets = _dev_f64(targets, self.device).reshape(-1, self.W)
        J = torch.empty(n, dtype=torch.float64, device=self.device)
        dJ = torch.empty(self.n_free, n, dtype=torch.float64, device=self.device)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        tid = _dev_i32(target_id, self.device)
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_grad_batch(self._h, n, _ptr(theta), _ptr(nc), _ptr(tid), _ptr(targets),
                                    targets.shape[0], _ptr(J), _ptr(dJ), int(ckpt_stride),
                                    _ptr(status), _stream()), "afm_grad_batch")
        return J, dJ, status

    def grad_batch_noalloc(self, theta, targets, J, dJ, status, target_id=None, n_cycles=None,
                           ckpt_stride=0):
        """afm_grad_batch_noalloc: grad_batch into caller-provided device tensors J [n],
        dJ [n_free][n] (float64) and status [n] (int32), with the checkpoints in the library's
        fixed scratch array (nothing is allocated on the device by the call)."""
        n = J.shape[0]
        tid = _dev_i32(target_id, self.device)
        nc = _dev_i32(n_cycles, self.device)
        _check(lib().afm_grad_batch_noalloc(self._h, n, _ptr(theta), _ptr(nc), _ptr(tid),
                                            _ptr(targets), targets.shape[0], _ptr(J), _ptr(dJ),
                                            int(ckpt_stride), _ptr(status), _stream()),
               "afm_grad_batch_noalloc")

    def separations(self, setpoint, params=None, periods=3000, lockin=2, step=0.25e-9, rounds=6):
        """afm_separations: z_c [S] (m) at which each pixel's steady amplitude equals
        setpoint[s] * A0; params: optional [MAX_PARAMS][S] full parameter vectors per pixel."""
        import torch

        sp = _dev_f64(setpoint, self.device).reshape(-1)
        S = sp.shape[0]
        pp = None if params is None else _dev_f64(params, self.device).reshape(MAX_PARAMS, S)
        zc = torch.empty(S, dtype=torch.float64, device=self.device)
        _check(lib().afm_separations(self._h, S, _ptr(pp), _ptr(sp), int(periods), int(lockin),
                                     float(step), int(rounds), _ptr(zc), _stream()),
               "afm_separations")
        return zc

    def swarm_init(self, particles, swarms=1, seed=0) -> Swarm:
        sw = Swarm(self.n_free, particles, swarms, self.device)
        sw._c = sw.cstruct()
        _check(lib().afm_swarm_init(self._h, C.byref(sw._c), int(seed) & (2**64 - 1), _stream()),
               "afm_swarm_init")
        return sw

    def pso_step(self, sw: Swarm, J, seed, it, is_last, cutoff=0.0):
        J = _dev_f64(J, self.device)
        _check(lib().afm_pso_step(self._h, C.byref(sw._c), _ptr(J), int(seed) & (2**64 - 1),
                                  int(it), int(bool(is_last)), float(cutoff), _stream()),
               "afm_pso_step")

    def polish(self, z, targets, target_id=None, n_cycles=None, steps=10, params=None):
        """L-BFGS polish of normalised positions z [n_free][n] (in place) -> J [n]."""
        import torch

        targets = _dev_f64(targets, self.device).reshape(-1, self.W)
        n = z.shape[1]
        J = torch.empty(n, dtype=torch.float64, device=self.device)
        tid = _dev_i32(target_id, self.device)
        nc = _dev_i32(n_cycles, self.device)
        pp = None if params is None else _dev_f64(params, self.device).reshape(MAX_PARAMS, n)
        _check(lib().afm_polish(self._h, n, _ptr(z), _ptr(pp), _ptr(nc), _ptr(tid), _ptr(targets),
                                targets.shape[0], int(steps), _ptr(J), _stream()), "afm_polish")
        return J

    def invert(self, targets, particles, iters, seed=0, cutoff=0.0, n_cycles=None, out=None,
               lbfgs_steps=0, lbfgs_topk=0, swarm_params=None):
        """S inversions (one swarm per target row) -> dict(best_theta [D][S], best_J, gen).

        swarm_params: optional [MAX_PARAMS][S] full parameter vectors per target."""
        import torch

        targets = _dev_f64(targets, self.device).reshape(-1, self.W)
        S = targets.shape[0]
        if out is None:
            out = {"best_theta": torch.empty(self.n_free, S, dtype=torch.float64, device=self.device),
                   "best_J": torch.empty(S, dtype=torch.float64, device=self.device),
                   "gen_to_cutoff": torch.empty(S, dtype=torch.int32, device=self.device)}
        nc = _dev_i32(n_cycles, self.device)
        sp = None if swarm_params is None else \
            _dev_f64(swarm_params, self.device).reshape(MAX_PARAMS, S)
        self._keep = (targets, nc, sp)  # the captured graph refers to these buffers
        _check(lib().afm_invert(self._h, S, _ptr(targets), _ptr(nc), _ptr(sp), int(particles),
                                int(iters),
                                int(seed) & (2**64 - 1), float(cutoff), int(lbfgs_steps),
                                int(lbfgs_topk), _ptr(out["best_theta"]),
                                _ptr(out["best_J"]), _ptr(out["gen_to_cutoff"]), _stream()),
               "afm_invert")
        return out


def _misfit_fn():
    import torch

    class MisfitFn(torch.autograd.Function):
        """J(theta) of afm_misfit with the discrete-adjoint gradient of afm_grad_batch.

        apply(theta [n_free][n], plan, targets [, target_id, n_cycles]) -> J [n]."""

        @staticmethod
        def forward(ctx, theta, plan, targets, target_id=None, n_cycles=None):
            J, _ = plan.misfit(theta, targets, target_id, n_cycles)
            ctx.save_for_backward(theta)
            ctx.plan, ctx.targets, ctx.tid, ctx.nc = plan, targets, target_id, n_cycles
            return J

        @staticmethod
        def backward(ctx, gJ):
            (theta,) = ctx.saved_tensors
            _, dJ, _ = ctx.plan.grad_batch(theta.detach(), ctx.targets, ctx.tid, ctx.nc)
            return gJ.to(dJ.dtype)[None, :] * dJ, None, None, None, None

    return MisfitFn


_MISFIT_FN = None


def misfit_fn():
    """The torch.autograd.Function class over afm_misfit / afm_grad_batch."""
    global _MISFIT_FN
    if _MISFIT_FN is None:
        _MISFIT_FN = _misfit_fn()
    return _MISFIT_FN


def version() -> str:
    return lib().afm_version().decode()
