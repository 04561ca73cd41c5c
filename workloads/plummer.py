"""Seeded synthetic inputs: Plummer spheres and the workload configurations.

This module only draws random numbers and rescales them.  It holds none of
the force, integrator or energy arithmetic, so both the FP64 oracle and the
HIP path can take their inputs from here without sharing any of the method.

Plummer sampling follows the method of Aarseth, Henon & Wielen (1974), the
one the paper cites for its initial conditions (Section 4, "Results"):

* radius from the inverted cumulative mass, r = (X^(-2/3) - 1)^(-1/2), with
  X redrawn when X > 0.999 (truncation of the infinite model);
* speed q = v / v_esc by von Neumann rejection on g(q) = q^2 (1 - q^2)^(7/2)
  under the bound 0.1, with v_esc = sqrt(2) (1 + r^2)^(-1/4);
* isotropic directions for both;
* equal masses m = 1/N, centre-of-mass frame, then the standard conversion
  from Henon units to N-body units (G = M = 1, E = -1/4): positions times
  3 pi / 16, velocities times sqrt(16 / (3 pi)).

The realisation is not re-virialised particle by particle: that would need
the softened potential energy, which belongs to the method, so the sample is
in virial equilibrium only statistically (E = -1/4 up to O(N^-1/2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "plummer",
    "cluster_sizes",
    "Config",
    "CONFIGS",
    "random_active_set",
    "ensemble_members",
]


def _isotropic(rng: np.random.Generator, mag: np.ndarray) -> np.ndarray:
    n = mag.shape[0]
    cos_t = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    out = np.empty((3, n))
    out[0] = mag * sin_t * np.cos(phi)
    out[1] = mag * sin_t * np.sin(phi)
    out[2] = mag * cos_t
    return out


def plummer(n: int, seed: int):
    """Return (pos, vel, mass) of an n-body Plummer sphere in N-body units.

    Layout is structure-of-arrays, component-major: ``pos`` and ``vel`` have
    shape (3, n) (x row, y row, z row) and ``mass`` shape (n,), all float64.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    # radii
    x1 = rng.random(n)
    bad = x1 > 0.999
    while bad.any():
        x1[bad] = rng.random(int(bad.sum()))
        bad = x1 > 0.999
    r = 1.0 / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, r)
    # speeds in units of the local escape speed
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x4 = rng.random(todo.size)
        x5 = rng.random(todo.size)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q[todo[ok]] = x4[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = _isotropic(rng, q * vesc)
    mass = np.full(n, 1.0 / n)
    # centre-of-mass frame (equal masses: plain means)
    pos -= pos.mean(axis=1, keepdims=True)
    vel -= vel.mean(axis=1, keepdims=True)
    # Henon -> N-body units
    pos *= 3.0 * math.pi / 16.0
    vel *= math.sqrt(16.0 / (3.0 * math.pi))
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


def cluster_sizes(n_clusters: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Cluster sizes drawn log-uniform in [lo, hi] and rounded to integers."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), n_clusters)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)


def random_active_set(n: int, n_i: int, seed: int) -> np.ndarray:
    """A seeded, sorted (ascending) subset of n_i distinct indices in [0, n)."""
    if not 0 <= n_i <= n:
        raise ValueError("need 0 <= n_i <= n")
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, size=n_i, replace=False)
    idx.sort()
    return idx.astype(np.int32)


@dataclass(frozen=True)
class Config:
    """One workload: sizes, softening, integrator parameters and seeds."""
    name: str
    n: int
    eps: float
    seed: int
    eta: float = 0.02
    eta_s: float = 0.01
    dt_max: float = 0.125
    t_end: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def eps2(self) -> float:
        return self.eps * self.eps


# The five workloads the hot path is exercised and measured on.
CONFIGS = {
    # Plummer N=1024, eps=1/256, Hermite-4 block steps, eta=0.02, to t=1/4.
    "plummer1k": Config("plummer1k", 1024, 1.0 / 256, 1001, t_end=0.25),
    # Plummer N=65536, eps=1/1024, block steps to t=1/8; full-N force throughput.
    "plummer64k": Config("plummer64k", 65536, 1.0 / 1024, 1002, t_end=0.125),
    # Plummer N=2^20, eps=1/4096; force-only sweep over n_i.
    "plummer1m": Config("plummer1m", 1 << 20, 1.0 / 4096, 1003,
                        extra={"n_i": (1024, 16384, 262144, 1 << 20),
                               "n_i_small": (1, 16, 64),
                               "n_sample": 4096}),
    # Beyond 2^20: N = 9,000,000 (the paper's capacity claim for its GPU),
    # force-only on seeded active subsets; N = 2^22, a few block steps.
    "plummer9m": Config("plummer9m", 9_000_000, 1.0 / 4096, 1007,
                        extra={"n_i": (1024, 65536), "n_sample": 1024}),
    "plummer4m": Config("plummer4m", 1 << 22, 1.0 / 4096, 1008,
                        extra={"steps": 3, "n_sample": 1024}),
    # 256 clusters, N log-uniform in [256, 8192], eps = N^(-1/3)/16, to t=1/16.
    "ensemble256": Config("ensemble256", 0, 0.0, 1004, dt_max=1.0 / 16,
                          t_end=1.0 / 16,
                          extra={"n_clusters": 256, "n_lo": 256, "n_hi": 8192}),
    # Section 4 results-table protocol: Plummer N = 256 ... 524288 (one
    # realisation per N), eps = 1/256, dt_max = 1/8, run t: 0 -> 1/2, timed
    # over t: 1/4 -> 1/2.
    "table_protocol": Config("table_protocol", 0, 1.0 / 256, 1006, t_end=0.5,
                             extra={"n_list": tuple(256 << k for k in range(12)),
                                    "timed_from": 0.25}),
    # Differentiable run: N=16384, eps=1/512, 64 shared steps of 1/512.
    "grad16k": Config("grad16k", 16384, 1.0 / 512, 1005,
                      extra={"dt": 1.0 / 512, "steps": 64, "ckpt": 8,
                             "target_seed": 2005, "fd_seed": 3005,
                             "n_coords": 32, "target_sigma": 1e-3,
                             "fd_h": 1e-6}),
}


def table_protocol_seed(n: int, cfg: Config = CONFIGS["table_protocol"]) -> int:
    """Seed of the one realisation used for N particles in the table protocol."""
    return cfg.seed * 1000 + int(n).bit_length() - 1


def ensemble_members(cfg: Config = CONFIGS["ensemble256"]):
    """Sizes, softenings and seeds of the ensemble's clusters."""
    sizes = cluster_sizes(cfg.extra["n_clusters"], cfg.extra["n_lo"],
                          cfg.extra["n_hi"], cfg.seed)
    eps = sizes.astype(np.float64) ** (-1.0 / 3.0) / 16.0
    seeds = cfg.seed * 1000 + np.arange(sizes.size)
    return sizes, eps, seeds
