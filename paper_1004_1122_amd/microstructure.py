"""Seeded synthetic microstructures (phase images) for every workload.

This module only draws inputs: it holds none of the solver's arithmetic and
is the one piece of code shared by the HIP path's callers and the tests that
feed the CPU reference.  A microstructure is a ``uint8`` phase image sampled
at the grid nodes (array index ``j`` at coordinate ``j / N`` of the unit cell)
plus a conductivity per phase; the paper treats "general microstructures
supplied in the form of digital images" (Sec. 1) with isotropic phases
(Sec. 3).

Workloads (all synthetic; the paper's own experiment is synthetic too):

* ``square_inclusion`` - 63x63 cell with a centred square of conductivity 10
  in a matrix of 1; the 31x31 nodes whose centred distance is at most 15
  (volume fraction 961/3969 = 0.242, the closest node set to 0.25).
* ``rsa_inclusions`` - random sequential addition of non-overlapping
  circles (2-D) or spheres (3-D) with uniform radii, periodic distances.
* ``grf_two_phase`` / ``batched_problem`` - thresholded Gaussian random
  fields with a Gaussian covariance of correlation length ``ell``.
* ``circle_array`` - the paper's model problem (Sec. 3): one circular
  particle per square cell at a given volume fraction.
* ``laminate`` - layers along one axis (closed-form effective tensor).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Microstructure",
    "square_inclusion",
    "rsa_inclusions",
    "grf_two_phase",
    "batched_problem",
    "warmstart_train_problem",
    "warmstart_eval_problem",
    "circle_array",
    "laminate",
    "lam_field",
]


@dataclass
class Microstructure:
    """A phase image, its per-phase conductivities and generation facts."""

    phase: np.ndarray                 # uint8, shape N (C order)
    cond: np.ndarray                  # float64, one conductivity per phase
    info: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.phase.shape

    @property
    def d(self):
        return self.phase.ndim

    def lam(self) -> np.ndarray:
        """Nodal conductivity field ``cond[phase]`` (input marshalling)."""
        return lam_field(self.phase, self.cond)


def lam_field(phase, cond) -> np.ndarray:
    return np.asarray(cond, dtype=np.float64)[np.asarray(phase)]


# ---------------------------------------------------------------------------
# Square inclusion (63x63, conductivity 10 in 1)
# ---------------------------------------------------------------------------

def square_inclusion(n: int = 63, half_width: int = 15, rho: float = 10.0) -> Microstructure:
    c = n // 2
    phase = np.zeros((n, n), dtype=np.uint8)
    phase[c - half_width:c + half_width + 1, c - half_width:c + half_width + 1] = 1
    return Microstructure(phase, np.array([1.0, rho]),
                          dict(kind="square", vf=float(phase.mean()), n=n))


# ---------------------------------------------------------------------------
# Random sequential addition of circles / spheres
# ---------------------------------------------------------------------------

def _periodic_dist(a, b):
    diff = np.abs(a - b)
    diff = np.minimum(diff, 1.0 - diff)
    return np.sqrt((diff * diff).sum(axis=-1))


def _rasterise_balls(n: int, d: int, centres, radii) -> np.ndarray:
    """Nodes at ``j / n`` within periodic distance ``r`` of a centre -> 1."""
    phase = np.zeros((n,) * d, dtype=np.uint8)
    for c, r in zip(centres, radii):
        lo = [int(math.floor((c[a] - r) * n)) - 1 for a in range(d)]
        hi = [int(math.ceil((c[a] + r) * n)) + 1 for a in range(d)]
        idx = [np.arange(lo[a], hi[a] + 1) for a in range(d)]
        grids = np.meshgrid(*idx, indexing="ij")
        dist2 = np.zeros(grids[0].shape)
        for a in range(d):
            x = grids[a] / n
            diff = np.abs(x - c[a])
            diff = np.minimum(diff % 1.0, 1.0 - (diff % 1.0))
            dist2 += diff * diff
        inside = dist2 <= r * r
        wrapped = tuple(np.mod(g[inside], n) for g in grids)
        phase[wrapped] = 1
    return phase


def rsa_inclusions(n: int, d: int, count: int, rmin: float, rmax: float,
                   seed: int, rho: float = 10.0,
                   max_attempts: int = 10 ** 6) -> Microstructure:
    """Random sequential addition without overlap in the periodic unit cell.

    Each attempt draws the radius ``r ~ U[rmin, rmax]`` and then the centre
    ``c ~ U[0, 1)^d``; it is accepted when the periodic centre distance to
    every accepted inclusion is at least the sum of the radii.  The stated
    number of inclusions is honoured and the achieved volume fraction is
    reported (``info['vf']``).
    """
    rng = np.random.default_rng(seed)
    centres = np.zeros((0, d))
    radii = np.zeros(0)
    attempts = 0
    while len(radii) < count:
        if attempts >= max_attempts:
            raise RuntimeError(f"RSA placed only {len(radii)} of {count} inclusions "
                               f"in {max_attempts} attempts")
        attempts += 1
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, 1.0, size=d)
        if len(radii) and np.any(_periodic_dist(centres, c[None, :]) < radii + r):
            continue
        centres = np.vstack([centres, c[None, :]])
        radii = np.append(radii, r)
    phase = _rasterise_balls(n, d, centres, radii)
    return Microstructure(phase, np.array([1.0, rho]),
                          dict(kind="rsa", vf=float(phase.mean()), n=n, d=d,
                               count=count, seed=seed, attempts=attempts,
                               centres=centres, radii=radii))


def circles_729(seed: int = 2, rho: float = 10.0) -> Microstructure:
    """729x729 cell with 40 RSA circles, radii U[0.02, 0.06]."""
    return rsa_inclusions(729, 2, 40, 0.02, 0.06, seed, rho)


def spheres_243(seed: int = 3, rho: float = 1e3) -> Microstructure:
    """243^3 cell with 200 RSA spheres, radii U[0.03, 0.08]."""
    return rsa_inclusions(243, 3, 200, 0.03, 0.08, seed, rho)


# ---------------------------------------------------------------------------
# Gaussian random fields
# ---------------------------------------------------------------------------

def _int_freq(n):
    m = np.arange(n)
    return np.where(m <= n // 2, m, m - n).astype(np.float64)


def grf_threshold(noise: np.ndarray, ell: float, vf: float) -> np.ndarray:
    """Filter white noise to a Gaussian covariance and threshold it.

    The amplitude filter ``exp(-pi^2 ell^2 |k|^2)`` (integer frequencies of
    the unit cell) gives a periodised covariance proportional to
    ``exp(-r^2 / (2 ell^2))``.  Phase 1 is given to the ``round(vf |N|)``
    largest values (stable order, ties to the lower flat index), so the volume
    fraction is exact.
    """
    shape = noise.shape
    k2 = np.zeros(shape)
    for a, n in enumerate(shape):
        view = [1] * len(shape)
        view[a] = n
        k2 = k2 + _int_freq(n).reshape(view) ** 2
    filt = np.exp(-math.pi ** 2 * ell ** 2 * k2)
    smooth = np.fft.ifftn(np.fft.fftn(noise) * filt).real
    count = int(round(vf * noise.size))
    order = np.argsort(-smooth.ravel(), kind="stable")
    phase = np.zeros(noise.size, dtype=np.uint8)
    phase[order[:count]] = 1
    return phase.reshape(shape)


def grf_two_phase(n: int, ell: float, vf: float, rho: float, seed: int, d: int = 2) -> Microstructure:
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n,) * d)
    phase = grf_threshold(noise, ell, vf)
    return Microstructure(phase, np.array([1.0, rho]),
                          dict(kind="grf", n=n, ell=ell, vf=float(phase.mean()), rho=rho, seed=seed))


def batched_problem(i: int) -> Microstructure:
    """Problem ``i`` of the 512-problem batch: seed ``400000 + i``.

    Grid size uniform over {81, 243, 729}, ``ell ~ U[0.05, 0.2]``,
    ``vf ~ U[0.2, 0.6]``, ``log10 rho ~ U[1, 4]``; phase 1 carries ``rho``.
    """
    return _grf_problem_fixed_draw(400000 + i, None)


def _grf_problem_fixed_draw(seed: int, forced_n):
    """Draw order: grid size, correlation length, volume fraction, log10 rho,
    noise.  A forced size still consumes the size draw, so the remaining
    draws do not depend on it."""
    rng = np.random.default_rng(seed)
    n_draw = int([81, 243, 729][rng.integers(3)])
    n = n_draw if forced_n is None else int(forced_n)
    ell = float(rng.uniform(0.05, 0.2))
    vf = float(rng.uniform(0.2, 0.6))
    log_rho = float(rng.uniform(1.0, 4.0))
    noise = rng.standard_normal((n, n))
    phase = grf_threshold(noise, ell, vf)
    rho = 10.0 ** log_rho
    return Microstructure(phase, np.array([1.0, rho]),
                          dict(kind="grf", n=n, ell=ell, vf_target=vf,
                               vf=float(phase.mean()), log10_rho=log_rho, rho=rho,
                               seed=seed))


def warmstart_train_problem(i: int) -> Microstructure:
    """Training problem ``i``: seed ``500000 + i``; 81^2 for even i, 243^2 for odd."""
    return _grf_problem_fixed_draw(500000 + i, 81 if i % 2 == 0 else 243)


def warmstart_eval_problem(i: int, n: int) -> Microstructure:
    """Held-out problem: seeds ``600000 + i`` (243^2) or ``610000 + i`` (729^2)."""
    base = 600000 if n == 243 else 610000
    return _grf_problem_fixed_draw(base + i, n)


# ---------------------------------------------------------------------------
# The paper's model problem and a laminate
# ---------------------------------------------------------------------------

def circle_array(n: int = 255, vf: float = 0.5, rho: float = 10.0) -> Microstructure:
    """One centred circular particle per cell at volume fraction ``vf``."""
    r = math.sqrt(vf / math.pi)
    x = np.arange(n) / n
    c = (n // 2) / n
    dx = x[:, None] - c
    dy = x[None, :] - c
    phase = ((dx * dx + dy * dy) <= r * r).astype(np.uint8)
    return Microstructure(phase, np.array([1.0, rho]),
                          dict(kind="circle_array", vf=float(phase.mean()), n=n))


def laminate(shape, layer_phase) -> np.ndarray:
    """Phase image constant across every axis but the first."""
    layer_phase = np.asarray(layer_phase, dtype=np.uint8)
    assert layer_phase.shape == (shape[0],)
    view = [shape[0]] + [1] * (len(shape) - 1)
    return np.broadcast_to(layer_phase.reshape(view), shape).copy()
