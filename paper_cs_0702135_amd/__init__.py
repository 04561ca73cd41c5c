"""MI355X (gfx950) direct-summation Hermite library: Python binding.

Thin marshalling layer over libnbody.so (include/nbody.h): every step of the
computation runs in the library's HIP kernels; PyTorch only provides device
memory and the stream.  Tensors are float64 on a CUDA (HIP) device, vectors
of shape (3, n) (component-major structure-of-arrays), scalars of shape (n,),
index lists int32.

Paper: Portegies Zwart, Belleman & Geldof, "High Performance Direct
Gravitational N-body Simulations on Graphics Processing Units" -- Section 2
(force, Hermite predictor-corrector, block time steps) and the Appendix A
listing (softened acceleration, jerk and potential).
"""
from __future__ import annotations

import atexit
import ctypes
import math
import threading

import torch

from . import _lib as L

__all__ = [
    "NBodyError", "Context", "context", "force", "force_sorted", "force_noalloc", "predict",
    "schedule",
    "schedule_async", "predict_dev", "force_dev", "correct_dev",
    "correct", "initial_dt", "energy", "System", "ACC_FP32", "ACC_DS",
    "ForceShape", "tune_set", "tune_clear", "tune_get", "profile",
    "force_adjoint", "predict_adjoint", "correct_adjoint", "ensemble_run",
    "ensemble_set", "ensemble_get", "ensemble_info", "ensemble_timing", "ensemble_plan",
]

ACC_FP32 = L.NBODY_ACC_FP32
ACC_DS = L.NBODY_ACC_DS
_MODES = {"fp32": ACC_FP32, "ds": ACC_DS}


class NBodyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libnbody error %d: %s" % (code, msg))
        self.code = code


class Context:
    """One library context per device; re-bound to torch's current stream."""

    def __init__(self, device: int):
        self.lib = L.load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.nbody_create(ctypes.byref(h), device, None)
        if rc != 0:
            raise NBodyError(rc, "nbody_create failed on device %d" % device)
        self.h = h

    def bind(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.nbody_set_stream(self.h, ctypes.c_void_p(s))
        return self.h

    def check(self, rc):
        if rc != 0:
            msg = self.lib.nbody_last_error(self.h)
            raise NBodyError(rc, msg.decode() if msg else "")

    def sync_status(self):
        self.check(self.lib.nbody_sync_status(self.bind()))

    def close(self):
        """Synchronise the context's stream and free its device memory."""
        h = getattr(self, "h", None)
        if h:
            self.h = None
            self.lib.nbody_destroy(h)

    def __del__(self):
        # contexts still open at interpreter exit were closed by
        # _close_all (atexit) while the HIP runtime was fully alive
        try:
            self.close()
        except Exception:
            pass


_ctx = {}
_ctx_lock = threading.Lock()
_atexit_registered = False


def _close_all():
    """Destroy every context (registered with atexit at the first context:
    it runs before torch's and the HIP runtime's own teardown, so no library
    call is made during interpreter or runtime finalisation)."""
    with _ctx_lock:
        ctxs = list(_ctx.values())
        _ctx.clear()
    for c in ctxs:
        try:
            c.close()
        except Exception:
            pass


def context(device=None) -> Context:
    if not torch.cuda.is_available():
        raise RuntimeError("libnbody needs a ROCm GPU (torch.cuda.is_available() is False)")
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    if dev is None:
        dev = torch.cuda.current_device()
    global _atexit_registered
    with _ctx_lock:
        if dev not in _ctx:
            if not _atexit_registered:
                atexit.register(_close_all)
                _atexit_registered = True
            _ctx[dev] = Context(dev)
        return _ctx[dev]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _vec(t, n, name):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (3, n):
        raise ValueError("%s must be a contiguous float64 CUDA tensor of shape (3, %d)" % (name, n))
    return t


def _sca(t, n, name):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (n,):
        raise ValueError("%s must be a contiguous float64 CUDA tensor of shape (%d,)" % (name, n))
    return t


def _mode(mode):
    if isinstance(mode, int):
        return mode
    try:
        return _MODES[mode]
    except KeyError:
        raise ValueError("mode must be 'fp32' or 'ds'") from None


def force(pos, vel, mass, eps2, active_idx=None, mode="fp32", out=None):
    """Acceleration, jerk and potential on the active particles.

    Returns (acc (3, n_i), jerk (3, n_i), pot (n_i,)) float64 tensors.
    """
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    if active_idx is not None:
        if active_idx.dtype != torch.int32 or not active_idx.is_cuda or active_idx.dim() != 1:
            raise ValueError("active_idx must be a 1-d int32 CUDA tensor")
        active_idx = active_idx.contiguous()
        n_i = active_idx.shape[0]
    else:
        n_i = n
    if out is None:
        acc = torch.empty((3, n_i), dtype=torch.float64, device=pos.device)
        jerk = torch.empty_like(acc)
        pot = torch.empty((n_i,), dtype=torch.float64, device=pos.device)
    else:
        acc, jerk, pot = out
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_force(ctx.bind(), _ptr(active_idx), n_i, _ptr(pos), _ptr(vel),
                                  _ptr(mass), n, float(eps2), _ptr(acc), _ptr(jerk),
                                  _ptr(pot), _mode(mode)))
    return acc, jerk, pot


def force_sorted(pos, vel, mass, eps2, active_idx=None):
    """Smallest-first float32 pair sums (nbody_force_sorted, Section 6):
    (acc (3, n_i), jerk (3, n_i), pot (n_i,)); n must not exceed 8192."""
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    if active_idx is not None:
        if active_idx.dtype != torch.int32 or not active_idx.is_cuda or active_idx.dim() != 1:
            raise ValueError("active_idx must be a 1-d int32 CUDA tensor")
        active_idx = active_idx.contiguous()
        n_i = active_idx.shape[0]
    else:
        n_i = n
    acc = torch.empty((3, n_i), dtype=torch.float64, device=pos.device)
    jerk = torch.empty_like(acc)
    pot = torch.empty((n_i,), dtype=torch.float64, device=pos.device)
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_force_sorted(ctx.bind(), _ptr(active_idx), n_i, _ptr(pos), _ptr(vel),
                                         _ptr(mass), n, float(eps2), _ptr(acc), _ptr(jerk),
                                         _ptr(pot)))
    return acc, jerk, pot


def force_noalloc(pos, vel, mass, eps2, active_idx=None, mode="fp32", out=None):
    """As force(), through nbody_force_noalloc: the library allocates no
    device memory for the call (its scratch is a static per-device array).
    Pass preallocated (acc, jerk, pot) as `out` to allocate nothing at all;
    n must not exceed NBODY_NOALLOC_MAX_NJ."""
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    if active_idx is not None:
        if active_idx.dtype != torch.int32 or not active_idx.is_cuda or active_idx.dim() != 1 \
                or not active_idx.is_contiguous():
            raise ValueError("active_idx must be a contiguous 1-d int32 CUDA tensor")
        n_i = active_idx.shape[0]
    else:
        n_i = n
    if out is None:
        acc = torch.empty((3, n_i), dtype=torch.float64, device=pos.device)
        jerk = torch.empty_like(acc)
        pot = torch.empty((n_i,), dtype=torch.float64, device=pos.device)
    else:
        acc, jerk, pot = out
        _vec(acc, n_i, "acc"), _vec(jerk, n_i, "jerk"), _sca(pot, n_i, "pot")
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_force_noalloc(ctx.bind(), _ptr(active_idx), n_i, _ptr(pos),
                                          _ptr(vel), _ptr(mass), n, float(eps2), _ptr(acc),
                                          _ptr(jerk), _ptr(pot), _mode(mode)))
    return acc, jerk, pot


def predict(t_target, t, x, v, a, k):
    n = t.shape[0]
    for q, nm in ((x, "x"), (v, "v"), (a, "a"), (k, "k")):
        _vec(q, n, nm)
    _sca(t, n, "t")
    xp = torch.empty_like(x)
    vp = torch.empty_like(v)
    ctx = context(x.device)
    ctx.check(ctx.lib.nbody_predict(ctx.bind(), n, float(t_target), _ptr(t), _ptr(x), _ptr(v),
                                    _ptr(a), _ptr(k), _ptr(xp), _ptr(vp)))
    return xp, vp


def schedule(t, dt):
    """Returns (active_idx int32 (n_i,), t_next float) -- synchronises."""
    n = t.shape[0]
    _sca(t, n, "t"), _sca(dt, n, "dt")
    act = torch.empty((n,), dtype=torch.int32, device=t.device)
    n_i = torch.empty((1,), dtype=torch.int64, device=t.device)
    tn = torch.empty((1,), dtype=torch.float64, device=t.device)
    ctx = context(t.device)
    ctx.check(ctx.lib.nbody_schedule(ctx.bind(), n, _ptr(t), _ptr(dt), _ptr(act), _ptr(n_i),
                                     _ptr(tn)))
    k = int(n_i.item())
    return act[:k], float(tn.item())


def schedule_async(t, dt):
    """nbody_schedule without the host read: returns (active_idx int32 (n,),
    n_i int64 (1,), t_next float64 (1,)) device tensors."""
    n = t.shape[0]
    _sca(t, n, "t"), _sca(dt, n, "dt")
    act = torch.empty((n,), dtype=torch.int32, device=t.device)
    n_i = torch.empty((1,), dtype=torch.int64, device=t.device)
    tn = torch.empty((1,), dtype=torch.float64, device=t.device)
    ctx = context(t.device)
    ctx.check(ctx.lib.nbody_schedule(ctx.bind(), n, _ptr(t), _ptr(dt), _ptr(act), _ptr(n_i),
                                     _ptr(tn)))
    return act, n_i, tn


def predict_dev(t_target, t, x, v, a, k):
    """nbody_predict_dev: t_target is a float64 (1,) device tensor."""
    n = t.shape[0]
    for q, nm in ((x, "x"), (v, "v"), (a, "a"), (k, "k")):
        _vec(q, n, nm)
    _sca(t, n, "t")
    xp, vp = torch.empty_like(x), torch.empty_like(v)
    ctx = context(x.device)
    ctx.check(ctx.lib.nbody_predict_dev(ctx.bind(), n, _ptr(t_target), _ptr(t), _ptr(x), _ptr(v),
                                        _ptr(a), _ptr(k), _ptr(xp), _ptr(vp)))
    return xp, vp


def force_dev(pos, vel, mass, eps2, active_idx, n_i, n_i_cap, mode="fp32"):
    """nbody_force_dev: the block size n_i is an int64 (1,) device tensor;
    returns (acc (3, n_i_cap), jerk (3, n_i_cap), pot (n_i_cap,)), of which
    the first n_i slots are set."""
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    acc = torch.empty((3, n_i_cap), dtype=torch.float64, device=pos.device)
    jerk = torch.empty_like(acc)
    pot = torch.empty((n_i_cap,), dtype=torch.float64, device=pos.device)
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_force_dev(ctx.bind(), _ptr(active_idx), _ptr(n_i), int(n_i_cap),
                                      _ptr(pos), _ptr(vel), _ptr(mass), n, float(eps2),
                                      _ptr(acc), _ptr(jerk), _ptr(pot), _mode(mode)))
    return acc, jerk, pot


def correct_dev(active_idx, n_i, n_i_cap, xp, vp, acc_new, jerk_new, eta, dt_max, dt_min, t,
                dt, x, v, a, k, fixed_dt=False):
    """nbody_correct_dev: the block size n_i is an int64 (1,) device tensor."""
    n = t.shape[0]
    for q, nm in ((xp, "xp"), (vp, "vp"), (x, "x"), (v, "v"), (a, "a"), (k, "k")):
        _vec(q, n, nm)
    _vec(acc_new, n_i_cap, "acc_new"), _vec(jerk_new, n_i_cap, "jerk_new")
    ctx = context(x.device)
    ctx.check(ctx.lib.nbody_correct_dev(ctx.bind(), n, _ptr(n_i), int(n_i_cap), _ptr(active_idx),
                                        _ptr(xp), _ptr(vp), _ptr(acc_new), _ptr(jerk_new),
                                        float(eta), float(dt_max), float(dt_min),
                                        int(bool(fixed_dt)), _ptr(t), _ptr(dt), _ptr(x), _ptr(v),
                                        _ptr(a), _ptr(k)))


def correct(active_idx, xp, vp, acc_new, jerk_new, eta, dt_max, dt_min, t, dt, x, v, a, k,
            fixed_dt=False):
    """Corrector and new steps on the active particles, in place."""
    n = t.shape[0]
    n_i = n if active_idx is None else active_idx.shape[0]
    for q, nm in ((xp, "xp"), (vp, "vp"), (x, "x"), (v, "v"), (a, "a"), (k, "k")):
        _vec(q, n, nm)
    _vec(acc_new, n_i, "acc_new"), _vec(jerk_new, n_i, "jerk_new")
    ctx = context(x.device)
    ctx.check(ctx.lib.nbody_correct(ctx.bind(), n, n_i, _ptr(active_idx), _ptr(xp), _ptr(vp),
                                    _ptr(acc_new), _ptr(jerk_new), float(eta), float(dt_max),
                                    float(dt_min), int(bool(fixed_dt)), _ptr(t), _ptr(dt),
                                    _ptr(x), _ptr(v), _ptr(a), _ptr(k)))


def initial_dt(t0, a, k, eta_s, dt_max, dt_min):
    n = a.shape[1]
    _vec(a, n, "a"), _vec(k, n, "k")
    dt = torch.empty((n,), dtype=torch.float64, device=a.device)
    ctx = context(a.device)
    ctx.check(ctx.lib.nbody_initial_dt(ctx.bind(), n, float(t0), _ptr(a), _ptr(k),
                                       float(eta_s), float(dt_max), float(dt_min), _ptr(dt)))
    return dt


def energy(pos, vel, mass, eps2):
    """(K, W) as host floats -- synchronises."""
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    out = torch.empty((2,), dtype=torch.float64, device=pos.device)
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_energy(ctx.bind(), n, _ptr(pos), _ptr(vel), _ptr(mass), float(eps2),
                                   _ptr(out)))
    K, W = out.tolist()
    return K, W


def force_adjoint(pos, vel, mass, eps2, acc_bar, jerk_bar, pot_bar=None, mode="fp32", out=None):
    """(pos_bar, vel_bar, mass_bar) of L = sum acc_bar.acc + jerk_bar.jerk + pot_bar.pot
    for the full set of particles (nbody_force_adjoint).  With `out` given,
    the gradients are added into those three tensors."""
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    _vec(acc_bar, n, "acc_bar"), _vec(jerk_bar, n, "jerk_bar")
    if pot_bar is not None:
        _sca(pot_bar, n, "pot_bar")
    flags = _mode(mode)
    if out is None:
        xb = torch.empty_like(pos)
        vb = torch.empty_like(vel)
        mb = torch.empty_like(mass)
    else:
        xb, vb, mb = out
        _vec(xb, n, "pos_bar"), _vec(vb, n, "vel_bar"), _sca(mb, n, "mass_bar")
        flags |= L.NBODY_ADJ_ACCUMULATE
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_force_adjoint(ctx.bind(), n, _ptr(pos), _ptr(vel), _ptr(mass),
                                          float(eps2), _ptr(acc_bar), _ptr(jerk_bar),
                                          _ptr(pot_bar), _ptr(xb), _ptr(vb), _ptr(mb), flags))
    return xb, vb, mb


def predict_adjoint(h, xp_bar, vp_bar, x_bar, v_bar, a_bar, k_bar):
    """Accumulate the predictor's transpose for a shared step h (in place)."""
    n = xp_bar.shape[1]
    for q, nm in ((xp_bar, "xp_bar"), (vp_bar, "vp_bar"), (x_bar, "x_bar"), (v_bar, "v_bar"),
                  (a_bar, "a_bar"), (k_bar, "k_bar")):
        _vec(q, n, nm)
    ctx = context(xp_bar.device)
    ctx.check(ctx.lib.nbody_predict_adjoint(ctx.bind(), n, float(h), _ptr(xp_bar), _ptr(vp_bar),
                                            _ptr(x_bar), _ptr(v_bar), _ptr(a_bar), _ptr(k_bar)))


def correct_adjoint(h, x1_bar, v1_bar, xp_bar, vp_bar, a0_bar, k0_bar, a1_bar, k1_bar):
    """Accumulate the corrector's transpose for a shared step h (in place)."""
    n = x1_bar.shape[1]
    for q, nm in ((x1_bar, "x1_bar"), (v1_bar, "v1_bar"), (xp_bar, "xp_bar"),
                  (vp_bar, "vp_bar"), (a0_bar, "a0_bar"), (k0_bar, "k0_bar"),
                  (a1_bar, "a1_bar"), (k1_bar, "k1_bar")):
        _vec(q, n, nm)
    ctx = context(x1_bar.device)
    ctx.check(ctx.lib.nbody_correct_adjoint(ctx.bind(), n, float(h), _ptr(x1_bar), _ptr(v1_bar),
                                            _ptr(xp_bar), _ptr(vp_bar), _ptr(a0_bar),
                                            _ptr(k0_bar), _ptr(a1_bar), _ptr(k1_bar)))


def ensemble_run(pos, vel, mass, offsets, eps2, t_end, eta=0.02, eta_s=0.01, dt_max=0.0625,
                 dt_min=2.0 ** -40, mode="fp32"):
    """Integrate independent clusters (particles [offsets[c], offsets[c+1]) of
    the concatenated (3, n) arrays, softening eps2[c]) from t = 0 to t_end in
    one persistent launch (nbody_ensemble_run).

    Returns a dict with the final t, dt, x, v, a, k tensors and host lists of
    block steps and interactions per cluster.
    """
    import numpy as _np
    n = mass.shape[0]
    _vec(pos, n, "pos"), _vec(vel, n, "vel"), _sca(mass, n, "mass")
    off = _np.ascontiguousarray(offsets, dtype=_np.int64)
    e2 = _np.ascontiguousarray(eps2, dtype=_np.float64)
    nc = off.shape[0] - 1
    if nc < 1 or e2.shape[0] != nc or off[-1] != n:
        raise ValueError("offsets must have n_clusters + 1 entries ending at n, eps2 n_clusters")
    st = {"x": pos.clone(), "v": vel.clone(),
          "t": torch.empty((n,), dtype=torch.float64, device=pos.device),
          "dt": torch.empty((n,), dtype=torch.float64, device=pos.device),
          "a": torch.empty_like(pos), "k": torch.empty_like(pos)}
    e = L.NBodyEnsemble(nc, off.ctypes.data_as(ctypes.c_void_p), e2.ctypes.data_as(ctypes.c_void_p),
                        st["t"].data_ptr(), st["dt"].data_ptr(), st["x"].data_ptr(),
                        st["v"].data_ptr(), st["a"].data_ptr(), st["k"].data_ptr(),
                        mass.data_ptr(), float(eta), float(eta_s), float(dt_max), float(dt_min),
                        _mode(mode))
    steps = (ctypes.c_int64 * nc)()
    inter = (ctypes.c_int64 * nc)()
    ctx = context(pos.device)
    ctx.check(ctx.lib.nbody_ensemble_run(ctx.bind(), ctypes.byref(e), float(t_end), steps, inter))
    st["steps"] = list(steps)
    st["interactions"] = list(inter)
    return st


def ensemble_set(groups_per_cu=None, max_team=None, step_us=None, barrier_us=None,
                 barrier_group_us=None, group_rate=None, steps_coef=None, steps_exp=None,
                 waves=None, j_tile=None, i_per_lane=None, tile_us=None, block_coef=None,
                 block_exp=None, device=None):
    """Change the ensemble launch shape / team-planning model (None keeps)."""
    ctx = context(device)
    c = L.NBodyEnsembleConfig()
    ctx.check(ctx.lib.nbody_ensemble_get(ctx.h, ctypes.byref(c)))
    for k, v in (("groups_per_cu", groups_per_cu), ("max_team", max_team), ("step_us", step_us),
                 ("barrier_us", barrier_us), ("barrier_group_us", barrier_group_us),
                 ("group_rate", group_rate),
                 ("steps_coef", steps_coef), ("steps_exp", steps_exp), ("waves", waves),
                 ("j_tile", j_tile), ("i_per_lane", i_per_lane), ("tile_us", tile_us),
                 ("block_coef", block_coef), ("block_exp", block_exp)):
        if v is not None:
            setattr(c, k, v)
    ctx.check(ctx.lib.nbody_ensemble_set(ctx.h, ctypes.byref(c)))


def ensemble_get(device=None):
    ctx = context(device)
    c = L.NBodyEnsembleConfig()
    ctx.check(ctx.lib.nbody_ensemble_get(ctx.h, ctypes.byref(c)))
    return {k: getattr(c, k) for k, _ in L.NBodyEnsembleConfig._fields_}


def ensemble_timing(n_clusters, device=None):
    """(seconds, groups) per cluster of the last ensemble launch."""
    ctx = context(device)
    sec = (ctypes.c_double * n_clusters)()
    grp = (ctypes.c_int32 * n_clusters)()
    ctx.check(ctx.lib.nbody_ensemble_timing(ctx.h, int(n_clusters), sec, grp))
    return list(sec), list(grp)


def ensemble_info(device=None):
    """(grid, teams) of the last ensemble launch."""
    ctx = context(device)
    g, t = ctypes.c_int32(), ctypes.c_int32()
    ctx.check(ctx.lib.nbody_ensemble_info(ctx.h, ctypes.byref(g), ctypes.byref(t)))
    return g.value, t.value


def ensemble_plan(sizes, groups, t_end, config):
    """Team plan of the ensemble for cluster `sizes` on a grid of `groups`
    workgroups under the planning model `config` (a dict with the fields of
    nbody_ensemble_config), computed on the host (nbody_ensemble_plan).

    Returns (team_of (n_clusters,), team_size (n_teams,), model_seconds
    (n_clusters,)) as numpy arrays.
    """
    import numpy as _np
    sz = _np.ascontiguousarray(sizes, dtype=_np.int64)
    nc = sz.shape[0]
    cfg = L.NBodyEnsembleConfig(int(config["groups_per_cu"]), int(config["max_team"]),
                                float(config["step_us"]), float(config["barrier_us"]),
                                float(config["barrier_group_us"]), float(config["group_rate"]),
                                float(config["steps_coef"]), float(config["steps_exp"]),
                                int(config.get("waves", 4)), int(config.get("j_tile", 256)),
                                int(config.get("i_per_lane", 2)),
                                float(config.get("tile_us", 0.0)),
                                float(config.get("block_coef", 0.20)),
                                float(config.get("block_exp", 0.81)))
    team_of = _np.empty(nc, dtype=_np.int32)
    team_size = _np.empty(nc, dtype=_np.int32)
    secs = _np.empty(nc, dtype=_np.float64)
    nt = ctypes.c_int32()
    lib = L.load()
    rc = lib.nbody_ensemble_plan(sz.ctypes.data_as(ctypes.c_void_p), nc, int(groups),
                                 ctypes.byref(cfg), float(t_end),
                                 team_of.ctypes.data_as(ctypes.c_void_p),
                                 team_size.ctypes.data_as(ctypes.c_void_p),
                                 secs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nt))
    if rc != 0:
        raise NBodyError(rc, "nbody_ensemble_plan: bad arguments")
    return team_of, team_size[:nt.value].copy(), secs


class ForceShape(tuple):
    """Launch shape of the pair kernels (see nbody_force_config)."""
    __slots__ = ()
    _names = ("rep", "i_per_lane", "waves", "tile", "min_j_wave", "target_groups", "layout")

    def __new__(cls, rep=0, i_per_lane=2, waves=1, tile=128, min_j_wave=64, target_groups=32768,
                layout=0):
        return tuple.__new__(cls, (int(rep), int(i_per_lane), int(waves), int(tile),
                                   int(min_j_wave), int(target_groups), int(layout)))

    def asdict(self):
        return dict(zip(self._names, self))

    def __repr__(self):
        return "ForceShape(%s)" % ", ".join("%s=%d" % kv for kv in zip(self._names, self))


def tune_set(n_i_lo, n_i_hi, shape, device=None):
    """Use `shape` for active blocks of n_i in [n_i_lo, n_i_hi); n_i_lo = -1
    sets the block-step driver's shape, n_i_lo = -2 its small-block shape
    (layout 1) for blocks of up to n_i_hi particles."""
    ctx = context(device)
    c = L.NBodyForceConfig(*shape)
    ctx.check(ctx.lib.nbody_tune_set(ctx.h, int(n_i_lo), int(n_i_hi), ctypes.byref(c)))


def tune_clear(device=None):
    ctx = context(device)
    ctx.check(ctx.lib.nbody_tune_clear(ctx.h))


def tune_get(n_i, device=None) -> ForceShape:
    ctx = context(device)
    c = L.NBodyForceConfig()
    ctx.check(ctx.lib.nbody_tune_get(ctx.h, int(n_i), ctypes.byref(c)))
    return ForceShape(c.rep, c.i_per_lane, c.waves, c.tile, c.min_j_wave, c.target_groups,
                      c.layout)


def profile(enable=-1, device=None):
    """Pair-kernel event timing: returns (force_ms, reduce_ms, launches)."""
    ctx = context(device)
    f, r, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    ctx.check(ctx.lib.nbody_profile(ctx.bind(), int(enable), ctypes.byref(f), ctypes.byref(r),
                                    ctypes.byref(k)))
    return f.value, r.value, k.value


VALU_KINDS = ("v_fmac_f32", "v_mul_f32", "v_add_f64", "v_cvt_f32_f64", "v_rsq_f32")


def valu_rates(waves_per_simd=8, device=None):
    """Issue rates of the VALU instruction kinds of the pair kernel's loop
    (nbody_valu_rates): {kind: wave-instructions per second of the device}."""
    ctx = context(device)
    rates = (ctypes.c_double * L.NBODY_VALU_KINDS)()
    ctx.check(ctx.lib.nbody_valu_rates(ctx.bind(), int(waves_per_simd), rates))
    return dict(zip(VALU_KINDS, rates))


class System:
    """Device-resident block-step integrator state (nbody_system)."""

    def __init__(self, pos, vel, mass, eps2, eta=0.02, eta_s=0.01, dt_max=0.125,
                 dt_min=2.0 ** -40, mode="fp32", t0=0.0, init=True, fixed_dt=False):
        dev = pos.device
        n = mass.shape[0]
        self.n = n
        self.x = _vec(pos, n, "pos").clone()
        self.v = _vec(vel, n, "vel").clone()
        self.m = _sca(mass, n, "mass").clone()
        self.t = torch.zeros((n,), dtype=torch.float64, device=dev)
        self.dt = torch.zeros((n,), dtype=torch.float64, device=dev)
        self.a = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.k = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.eps2, self.eta, self.eta_s = float(eps2), float(eta), float(eta_s)
        self.dt_max, self.dt_min = float(dt_max), float(dt_min)
        self.flags = _mode(mode) | (L.NBODY_FIXED_DT if fixed_dt else 0)
        self.steps = 0
        self.interactions = 0
        if init:
            self.init(t0)

    def _struct(self):
        return L.NBodySystem(self.n, self.t.data_ptr(), self.dt.data_ptr(), self.x.data_ptr(),
                             self.v.data_ptr(), self.a.data_ptr(), self.k.data_ptr(),
                             self.m.data_ptr(), self.eps2, self.eta, self.eta_s, self.dt_max,
                             self.dt_min, self.flags)

    def init(self, t0=0.0):
        ctx = context(self.x.device)
        s = self._struct()
        ctx.check(ctx.lib.nbody_init(ctx.bind(), ctypes.byref(s), float(t0)))
        ctx.sync_status()

    def run(self, t_end, max_steps=1 << 40):
        """Block steps until the next block would pass t_end; returns steps."""
        ctx = context(self.x.device)
        s = self._struct()
        steps = ctypes.c_int64(0)
        inter = ctypes.c_int64(0)
        ctx.check(ctx.lib.nbody_blockstep(ctx.bind(), ctypes.byref(s), int(max_steps),
                                          float(t_end), ctypes.byref(steps),
                                          ctypes.byref(inter)))
        self.steps += steps.value
        self.interactions += inter.value
        return steps.value

    def step(self, n_steps=1):
        return self.run(math.inf, max_steps=n_steps)

    def energy(self):
        K, W = energy(self.x, self.v, self.m, self.eps2)
        return K + W
