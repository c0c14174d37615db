"""Seeded synthetic particle sets shaped like the paper's workloads.

This module only draws random inputs.  It holds none of the method's
arithmetic and is shared, unchanged, by the CPU oracle tests, the GPU parity
tests and the benchmark, so that both sides always see identical inputs.

Source moments use the physical convention (see ``include/fmm.h``):
  order 0: q[N]             (charges)
  order 1: mu[N, 3]         (dipole vectors)
  order 2: Q[N, 6]          (xx, xy, xz, yy, yz, zz of a symmetric 3x3 tensor)
  mixed:   MIXED + mask     (bit k: order k present), rows [q | mu | Q] of the
                            present orders, concatenated in ascending order

The workloads follow the paper's test sets: random charges in a box and a
cubic spin lattice (Section 4), extended to dipoles, a Plummer sphere and
quadrupoles of the sizes the benchmark names.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 200512351
MIXED = 16          # order code of a system with several source orders: MIXED + bit mask


@dataclass
class Workload:
    name: str
    pos: np.ndarray            # (N, 3) float64, C-contiguous
    order: int                 # source order m (0, 1, 2) or MIXED + bit mask of orders
    moments: np.ndarray        # (N,), (N, 3), (N, 6) or (N, w) float64 (mixed)
    p: int
    theta: float
    ncrit: int
    outputs: str               # "pot+field" or "field"
    sample: Optional[np.ndarray] = None   # int64 target indices for sampled checks
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    nrm = np.sqrt((g * g).sum(axis=1))
    nrm[nrm == 0.0] = 1.0
    return np.ascontiguousarray(g / nrm[:, None])


def uniform_cube(rng: np.random.Generator, n: int) -> np.ndarray:
    return np.ascontiguousarray(rng.random((n, 3)))


def plummer(rng: np.random.Generator, n: int, a: float = 0.1, umax: float = 0.999) -> np.ndarray:
    """Plummer sphere: radius from the inverse cumulative mass, cut at mass
    fraction ``umax``; isotropic directions."""
    u = rng.uniform(0.0, umax, n)
    u = np.maximum(u, 1e-12)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    d = _unit_vectors(rng, n)
    return np.ascontiguousarray(d * r[:, None])


def jittered_lattice(rng: np.random.Generator, nx: int, ny: int, nz: int, h: float) -> np.ndarray:
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    jit = rng.uniform(-h / 4.0, h / 4.0, base.shape)
    return np.ascontiguousarray((base + 0.5) * h + jit)


def random_moments(rng: np.random.Generator, order: int, n: int, kind: str = "default") -> np.ndarray:
    if order == 0:
        return np.ascontiguousarray(rng.uniform(-1.0, 1.0, n))
    if order == 1:
        return _unit_vectors(rng, n)
    if order == 2:
        q = rng.standard_normal((n, 6))          # xx, xy, xz, yy, yz, zz
        tr = (q[:, 0] + q[:, 3] + q[:, 5]) / 3.0
        q[:, 0] -= tr
        q[:, 3] -= tr
        q[:, 5] -= tr
        return np.ascontiguousarray(q)
    if order == 3:
        return traceless_octupoles(rng.standard_normal((n, 10)))
    raise ValueError("order must be 0, 1, 2 or 3")


# the ten components of an octupole in the index order of order 3
OCT_INDEX = [(3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 2, 1), (0, 1, 2),
             (0, 0, 3)]


def octupole_full(o: np.ndarray) -> np.ndarray:
    """(n, 10) components -> (n, 3, 3, 3) symmetric tensors"""
    o = np.asarray(o, dtype=np.float64).reshape(-1, 10)
    T = np.empty((o.shape[0], 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                c = [0, 0, 0]
                c[i] += 1
                c[j] += 1
                c[k] += 1
                T[:, i, j, k] = o[:, OCT_INDEX.index(tuple(c))]
    return T


def traceless_octupoles(o: np.ndarray) -> np.ndarray:
    """remove the trace t_k = sum_i O_iik: O - (delta_ij t_k + delta_ik t_j +
    delta_jk t_i) / 5"""
    T = octupole_full(o)
    t = np.einsum("niik->nk", T)
    d = np.eye(3)
    T = T - (np.einsum("ij,nk->nijk", d, t) + np.einsum("ik,nj->nijk", d, t) + np.einsum("jk,ni->nijk", d, t)) / 5.0
    return np.ascontiguousarray(np.stack([T[:, a, b, c] for a, b, c in map(_axes, OCT_INDEX)], axis=1))


def _axes(c):
    return [a for a in range(3) for _ in range(c[a])]


def sample_targets(seed: int, n: int, k: int = 4096) -> np.ndarray:
    rng = np.random.default_rng(seed + 7)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def config(index: int, n_override: Optional[int] = None) -> Workload:
    """The five benchmark configurations (index 1..4; 5 is the serving mix,
    see ``serving_stream``).  ``n_override`` shrinks a config for quick tests
    while keeping its distribution and parameters."""
    seed = SEED_BASE + index
    rng = np.random.default_rng(seed)
    if index == 1:
        n = n_override or 1000
        pos = uniform_cube(rng, n)
        mom = random_moments(rng, 0, n)
        return Workload("C1: 1k monopoles uniform cube p=4", pos, 0, mom, 4, 0.5, 64, "pot+field")
    if index == 2:
        n = n_override or 100_000
        pos = uniform_cube(rng, n)
        mom = random_moments(rng, 1, n)
        return Workload("C2: 100k dipoles uniform cube p=8", pos, 1, mom, 8, 0.5, 64, "pot+field",
                        sample=sample_targets(seed, n))
    if index == 3:
        n = n_override or 1_000_000
        pos = plummer(rng, n)
        mom = random_moments(rng, 1, n)
        return Workload("C3: 1M Plummer dipoles p=6", pos, 1, mom, 6, 0.6, 128, "field",
                        sample=sample_targets(seed, n))
    if index == 4:
        if n_override:
            side = max(2, int(round(n_override ** (1.0 / 3.0))))
            nx, ny, nz = side, side, side
            h = 1.0 / side
        else:
            nx, ny, nz = 125, 125, 128
            h = 1.0 / 125.0
        pos = jittered_lattice(rng, nx, ny, nz, h)
        mom = random_moments(rng, 2, pos.shape[0])
        return Workload("C4: 2M lattice quadrupoles p=10", pos, 2, mom, 10, 0.5, 64, "pot+field",
                        sample=sample_targets(seed, pos.shape[0]))
    if index == 0:
        # The paper's optimisation study: 1e5 charges in a 2e-9 box, theta=0.3, ncrit=128.
        n = n_override or 100_000
        pos = np.ascontiguousarray(rng.uniform(-1e-9, 1e-9, (n, 3)))
        mom = random_moments(rng, 0, n)
        return Workload("C0: 1e5 charges in [-1e-9,1e-9]^3", pos, 0, mom, 8, 0.3, 128, "pot+field",
                        sample=sample_targets(seed, n))
    raise ValueError(f"unknown config {index}")


@dataclass
class Request:
    rid: int
    arrival: float             # seconds since stream start
    workload: Workload


def serving_stream(n_requests: int = 512, rate: float = 100.0, nmax: int = 200_000,
                   nmin: int = 1000, seed: Optional[int] = None) -> list:
    """Poisson arrivals; N log-uniform in [nmin, nmax]; order uniform in
    {0,1,2}; p uniform in {4,6,8}; positions uniform or Plummer (half each);
    theta = 0.5, ncrit = 64."""
    seed = SEED_BASE + 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(np.floor(10.0 ** rng.uniform(np.log10(nmin), np.log10(nmax))))
        order = int(rng.integers(0, 3))
        p = int(rng.choice([4, 6, 8]))
        sub = np.random.default_rng(seed * 1000 + i)
        pos = uniform_cube(sub, n) if rng.random() < 0.5 else plummer(sub, n)
        mom = random_moments(sub, order, n)
        out.append(Request(i, t, Workload(f"req{i}", pos, order, mom, p, 0.5, 64, "pot+field")))
    return out


def small_random(seed: int, n: int, order: int, kind: str = "uniform", p: int = 4,
                 theta: float = 0.5, ncrit: int = 8) -> Workload:
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        pos = uniform_cube(rng, n)
    elif kind == "plummer":
        pos = plummer(rng, n)
    elif kind == "lattice":
        side = max(1, int(round(n ** (1.0 / 3.0))))
        pos = jittered_lattice(rng, side, side, side, 1.0 / side)
    else:
        raise ValueError(kind)
    mom = random_moments(rng, order, pos.shape[0])
    return Workload(f"small-{kind}-{n}-m{order}", pos, order, mom, p, theta, ncrit, "pot+field")


def mixed_moments(rng: np.random.Generator, mask: int, n: int) -> np.ndarray:
    """Rows [q | mu | Q | O] of the orders present in ``mask`` (bit k: order k)."""
    parts = [random_moments(rng, k, n).reshape(n, -1) for k in range(4) if mask & (1 << k)]
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


def small_mixed(seed: int, n: int, mask: int, kind: str = "uniform", p: int = 4,
                theta: float = 0.5, ncrit: int = 8) -> Workload:
    """A system with several source orders at once (charges, dipoles,
    quadrupoles as ``mask`` selects), every particle carrying all of them."""
    w = small_random(seed, n, 0, kind, p, theta, ncrit)
    rng = np.random.default_rng(seed + 1)
    mom = mixed_moments(rng, mask, w.n)
    return Workload(f"mixed-{kind}-{n}-k{mask}", w.pos, MIXED + mask, mom, p, theta, ncrit, "pot+field")
