"""FP64 CPU oracle (test infrastructure only).

Plain double-precision reference of the direct-summation Hermite hot path,
written from the paper (Portegies Zwart, Belleman & Geldof, Section 2 and the
Appendix A listing).  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the HIP library never does and
shares no code with it.

The arithmetic lives in ``nbody_oracle.c`` (built into ``liboracle.so`` with
``-ffp-contract=off``); this module only marshals numpy arrays, plus the two
linear adjoints of the shared-step Hermite chain, written out in numpy.

Arrays are float64 numpy arrays of shape (3, n) for vectors (x, y, z rows,
i.e. component-major structure-of-arrays) and (n,) for scalars.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

E_RANGE = -3
E_NONFINITE = -4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O3, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c99", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC,
               "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        I = ctypes.c_int
        lib.oracle_force.argtypes = [I64, P, I64, P, P, P, D, P, P, P]
        lib.oracle_force.restype = None
        lib.oracle_force_sum32.argtypes = [I64, P, I64, P, P, P, D, I, P, P, P]
        lib.oracle_force_sum32.restype = I
        lib.oracle_predict.argtypes = [I64, D, P, P, P, P, P, P, P]
        lib.oracle_predict.restype = None
        lib.oracle_schedule.argtypes = [I64, P, P, P, P]
        lib.oracle_schedule.restype = I64
        lib.oracle_initial_dt.argtypes = [I64, D, P, P, D, D, D, P]
        lib.oracle_initial_dt.restype = I
        lib.oracle_correct.argtypes = [I64, I64, P, P, P, P, P, D, D, D, I,
                                       P, P, P, P, P, P]
        lib.oracle_correct.restype = I
        lib.oracle_energy.argtypes = [I64, P, P, P, D, P]
        lib.oracle_energy.restype = None
        lib.oracle_init.argtypes = [I64, D, P, D, D, D, D, P, P, P, P, P, P]
        lib.oracle_init.restype = I
        lib.oracle_blockstep.argtypes = [I64, P, D, D, D, D, D, P, P, P, P, P,
                                         P, P, P]
        lib.oracle_blockstep.restype = I64
        lib.oracle_integrate.argtypes = [I64, P, D, D, D, D, D, I64, P, P, P,
                                         P, P, P, P]
        lib.oracle_integrate.restype = I
        lib.oracle_shared_run.argtypes = [I64, I64, D, P, D, P, P, P, P]
        lib.oracle_shared_run.restype = None
        lib.oracle_force_adjoint.argtypes = [I64, P, P, P, D, P, P, P, P, P, P]
        lib.oracle_force_adjoint.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = I
        lib.oracle_set_num_threads.argtypes = [I]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _L().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _L().oracle_set_num_threads(int(n))


def force(pos, vel, mass, eps2, active=None):
    """Acceleration, jerk and potential of the active particles.

    Returns (acc (3, n_i), jerk (3, n_i), pot (n_i,)).
    """
    pos, vel, mass = _f64(pos), _f64(vel), _f64(mass)
    n_j = mass.shape[0]
    if active is None:
        n_i, act = n_j, None
    else:
        act = np.ascontiguousarray(active, dtype=np.int32)
        n_i = act.shape[0]
    acc = np.empty((3, n_i))
    jerk = np.empty((3, n_i))
    pot = np.empty(n_i)
    _L().oracle_force(n_i, None if act is None else _p(act), n_j, _p(pos),
                      _p(vel), _p(mass), float(eps2), _p(acc), _p(jerk), _p(pot))
    return acc, jerk, pot


def force_sum32(pos, vel, mass, eps2, active=None, order="sorted"):
    """The pair sums of force(), each term rounded to float32 and added in
    float32 in ascending j (order="index") or smallest force first
    (order="sorted", the summation order Section 6 proposes).

    Returns (acc (3, n_i), jerk (3, n_i), pot (n_i,)) as float64 arrays
    holding the float32 sums.
    """
    pos, vel, mass = _f64(pos), _f64(vel), _f64(mass)
    n_j = mass.shape[0]
    if active is None:
        n_i, act = n_j, None
    else:
        act = np.ascontiguousarray(active, dtype=np.int32)
        n_i = act.shape[0]
    acc = np.empty((3, n_i))
    jerk = np.empty((3, n_i))
    pot = np.empty(n_i)
    code = {"index": 0, "sorted": 1}[order]
    rc = _L().oracle_force_sum32(n_i, None if act is None else _p(act), n_j, _p(pos), _p(vel),
                                 _p(mass), float(eps2), code, _p(acc), _p(jerk), _p(pot))
    if rc != 0:
        raise MemoryError("oracle_force_sum32: out of memory")
    return acc, jerk, pot


def predict(t_target, t, x, v, a, k):
    t, x, v, a, k = map(_f64, (t, x, v, a, k))
    n = t.shape[0]
    xp = np.empty((3, n))
    vp = np.empty((3, n))
    _L().oracle_predict(n, float(t_target), _p(t), _p(x), _p(v), _p(a), _p(k),
                        _p(xp), _p(vp))
    return xp, vp


def schedule(t, dt):
    t, dt = _f64(t), _f64(dt)
    n = t.shape[0]
    act = np.empty(max(n, 1), dtype=np.int32)
    tn = np.empty(1)
    m = _L().oracle_schedule(n, _p(t), _p(dt), _p(tn), _p(act))
    return float(tn[0]), act[:m].copy()


def initial_dt(t0, a, k, eta_s, dt_max, dt_min):
    a, k = _f64(a), _f64(k)
    n = a.shape[1]
    dt = np.empty(n)
    rc = _L().oracle_initial_dt(n, float(t0), _p(a), _p(k), float(eta_s),
                                float(dt_max), float(dt_min), _p(dt))
    return dt, rc


def correct(active, xp, vp, acc_new, jerk_new, eta, dt_max, dt_min, t, dt, x,
            v, a, k, fixed_dt=False):
    """Correct the active particles in place (t, dt, x, v, a, k); returns rc."""
    xp, vp, acc_new, jerk_new = map(_f64, (xp, vp, acc_new, jerk_new))
    for arr in (t, dt, x, v, a, k):
        assert arr.dtype == np.float64 and arr.flags.c_contiguous
    n = t.shape[0]
    if active is None:
        act, n_i = None, n
    else:
        act = np.ascontiguousarray(active, dtype=np.int32)
        n_i = act.shape[0]
    return _L().oracle_correct(n, n_i, None if act is None else _p(act),
                               _p(xp), _p(vp), _p(acc_new), _p(jerk_new),
                               float(eta), float(dt_max), float(dt_min),
                               int(bool(fixed_dt)), _p(t), _p(dt), _p(x),
                               _p(v), _p(a), _p(k))


def energy(pos, vel, mass, eps2):
    """(K, W): kinetic and softened potential energy."""
    pos, vel, mass = _f64(pos), _f64(vel), _f64(mass)
    out = np.empty(2)
    _L().oracle_energy(mass.shape[0], _p(pos), _p(vel), _p(mass), float(eps2),
                       _p(out))
    return float(out[0]), float(out[1])


@dataclass
class State:
    """Block-step integrator state of n particles (all float64)."""
    t: np.ndarray
    dt: np.ndarray
    x: np.ndarray
    v: np.ndarray
    a: np.ndarray
    k: np.ndarray
    m: np.ndarray
    eps2: float
    eta: float = 0.02
    eta_s: float = 0.01
    dt_max: float = 0.125
    dt_min: float = 2.0 ** -40

    @property
    def n(self) -> int:
        return self.m.shape[0]

    def copy(self) -> "State":
        return State(self.t.copy(), self.dt.copy(), self.x.copy(), self.v.copy(),
                     self.a.copy(), self.k.copy(), self.m.copy(), self.eps2,
                     self.eta, self.eta_s, self.dt_max, self.dt_min)


def init_state(pos, vel, mass, eps2, eta=0.02, eta_s=0.01, dt_max=0.125,
               dt_min=2.0 ** -40, t0=0.0) -> State:
    n = len(mass)
    s = State(np.empty(n), np.empty(n), _f64(pos).copy(), _f64(vel).copy(),
              np.empty((3, n)), np.empty((3, n)), _f64(mass).copy(),
              float(eps2), eta, eta_s, dt_max, dt_min)
    rc = _L().oracle_init(n, float(t0), _p(s.m), s.eps2, eta_s, dt_max, dt_min,
                          _p(s.t), _p(s.dt), _p(s.x), _p(s.v), _p(s.a), _p(s.k))
    if rc != 0:
        raise RuntimeError("oracle_init failed: %d" % rc)
    return s


def blockstep(s: State, t_end=np.inf):
    """One block step in place.  Returns (n_i, t_next, active)."""
    act = np.empty(s.n, dtype=np.int32)
    tn = np.empty(1)
    r = _L().oracle_blockstep(s.n, _p(s.m), s.eps2, s.eta, s.dt_max, s.dt_min,
                              float(t_end), _p(s.t), _p(s.dt), _p(s.x),
                              _p(s.v), _p(s.a), _p(s.k), _p(tn), _p(act))
    if r < 0:
        raise RuntimeError("oracle_blockstep failed: %d" % r)
    return int(r), float(tn[0]), act[:r].copy()


def integrate(s: State, t_end, max_steps=1 << 40):
    """Block steps until the next block would pass t_end.

    Returns (steps, sum of block sizes).
    """
    stats = np.zeros(2, dtype=np.int64)
    rc = _L().oracle_integrate(s.n, _p(s.m), s.eps2, s.eta, s.dt_max, s.dt_min,
                               float(t_end), int(max_steps), _p(s.t), _p(s.dt),
                               _p(s.x), _p(s.v), _p(s.a), _p(s.k), _p(stats))
    if rc != 0:
        raise RuntimeError("oracle_integrate failed: %d" % rc)
    return int(stats[0]), int(stats[1])


def shared_run(pos, vel, mass, eps2, h, n_steps):
    """Shared-step Hermite run; returns (x, v, a, k) after n_steps of h."""
    x, v, m = _f64(pos).copy(), _f64(vel).copy(), _f64(mass)
    n = m.shape[0]
    a = np.empty((3, n))
    k = np.empty((3, n))
    _L().oracle_shared_run(n, int(n_steps), float(h), _p(m), float(eps2),
                           _p(x), _p(v), _p(a), _p(k))
    return x, v, a, k


def force_adjoint(pos, vel, mass, eps2, abar, kbar, pbar):
    """(xbar, vbar, mbar) of L = sum abar.a + kbar.k + pbar phi (full set)."""
    pos, vel, mass, abar, kbar, pbar = map(_f64, (pos, vel, mass, abar, kbar,
                                                  pbar))
    n = mass.shape[0]
    xb = np.empty((3, n))
    vb = np.empty((3, n))
    mb = np.empty(n)
    _L().oracle_force_adjoint(n, _p(pos), _p(vel), _p(mass), float(eps2),
                              _p(abar), _p(kbar), _p(pbar), _p(xb), _p(vb),
                              _p(mb))
    return xb, vb, mb


# ---------------------------------------------------------------------------
# Shared-step Hermite chain and its adjoint (numpy; force pieces in C).
#
# One step with common step h, from (x, v, a, k):
#   predictor (Section 2):  xp = x + (v + (h/2)(a + (h/3)k))h,
#                           vp = v + (a + (h/2)k)h
#   force:                  a1, k1 = F(xp, vp)
#   corrector (Section 2):  with A3 = 2(a-a1) + (k+k1)h and
#                           A2 = -3(a-a1) - (2k+k1)h,
#                           x1 = xp + (A2/12 + A3/20)h^2,
#                           v1 = vp + (A2/3 + A3/4)h.
# Expanding A2, A3 makes the corrector linear in (a, k, a1, k1):
#   x1 = xp - (3/20)h^2 (a - a1) - h^3 (7k/60 + k1/30)
#   v1 = vp - (h/2)(a - a1)      - h^2 (5k/12 + k1/12)
# whose transpose is written out below.
# ---------------------------------------------------------------------------

def shared_chain_forward(pos, vel, mass, eps2, h, n_steps):
    """Forward run storing every step's start state (for the adjoint)."""
    x, v = _f64(pos).copy(), _f64(vel).copy()
    a, k, _ = force(x, v, mass, eps2)
    tape = []
    t = np.zeros(x.shape[1])
    for _ in range(n_steps):
        tape.append((x, v, a, k))
        xp, vp = predict(h, t, x, v, a, k)
        a1, k1, _ = force(xp, vp, mass, eps2)
        x1 = xp.copy()
        v1 = vp.copy()
        tt = t.copy()
        dt = np.full_like(t, h)
        aa, kk = a.copy(), k.copy()
        correct(None, xp, vp, a1, k1, 0.0, h, h, tt, dt, x1, v1, aa, kk,
                fixed_dt=True)
        x, v, a, k = x1, v1, aa, kk
    return (x, v, a, k), tape


def shared_chain_adjoint(pos, vel, mass, eps2, h, n_steps, xbar_T, vbar_T):
    """dL/dx0, dL/dv0, dL/dm for L depending on the final (x, v) only."""
    (_, _, _, _), tape = shared_chain_forward(pos, vel, mass, eps2, h, n_steps)
    mass = _f64(mass)
    xb = _f64(xbar_T).copy()
    vb = _f64(vbar_T).copy()
    ab = np.zeros_like(xb)   # cotangent of the a carried into the next step
    kb = np.zeros_like(xb)
    mb = np.zeros_like(mass)
    t = np.zeros(xb.shape[1])
    for (x, v, a, k) in reversed(tape):
        xp, vp = predict(h, t, x, v, a, k)
        # corrector transpose
        xpb = xb.copy()
        vpb = vb.copy()
        # (ab, kb carry the cotangent of this step's outputs a <- a1, k <- k1)
        a0b = -0.15 * h * h * xb - 0.5 * h * vb
        a1b = ab + 0.15 * h * h * xb + 0.5 * h * vb
        k0b = -(7.0 / 60.0) * h ** 3 * xb - (5.0 / 12.0) * h * h * vb
        k1b = kb - (1.0 / 30.0) * h ** 3 * xb - (1.0 / 12.0) * h * h * vb
        # force transpose at the predicted state
        gx, gv, gm = force_adjoint(xp, vp, mass, eps2, a1b, k1b,
                                   np.zeros(xb.shape[1]))
        xpb += gx
        vpb += gv
        mb += gm
        # predictor transpose
        xb = xpb
        vb = h * xpb + vpb
        ab = a0b + 0.5 * h * h * xpb + h * vpb
        kb = k0b + (h ** 3 / 6.0) * xpb + 0.5 * h * h * vpb
    # initial force a0, k0 = F(x0, v0)
    x0, v0 = _f64(pos), _f64(vel)
    gx, gv, gm = force_adjoint(x0, v0, mass, eps2, ab, kb, np.zeros(xb.shape[1]))
    return xb + gx, vb + gv, mb + gm
