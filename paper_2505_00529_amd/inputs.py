"""Seeded synthetic inputs for the second-order adjoint quantum-control workloads.

This module only draws random numbers: Hamiltonians, dipole matrices, initial and
target states, control coefficients and directions.  It holds none of the method's
arithmetic (no basis functions, no propagators, no derivatives), so that both the
device path and the CPU oracle can take their inputs from here without sharing any
computation.

The paper's molecular matrices (H2 and HeH+ in STO-3G / 6-31G, Sec. II) are not
available; these "molecule-shaped" systems stand in for them: a diagonal core
Hamiltonian H0 (diagonal in the full-CI basis, Sec. II, eq. matrixTDSE) with a
negative spectrum, a real symmetric dipole matrix M that does not commute with H0,
the ground state as initial state and a target in a low-lying eigenspace.

Workload recipes (all real FP64 system matrices, complex FP64 states):

* ``tiny``     N=4,   J=500,   dt=0.05, Fourier K=4   (P=8)
* ``molecule`` N=36,  J=4000,  dt=0.02, Fourier K=16  (P=32)
* ``diff``     N=128, J=10000, dt=0.01, Fourier K=64  (P=128)
* ``warm``     N=64,  J=4000,  dt=0.02, Fourier K=32  (P=64)
* ``batched``  256 problems, N in {8,16,36,64,128}, J in [2000, 8000], K in {8,16,32}
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = [
    "System",
    "Workload",
    "spectrum_with_gap",
    "tiny_system",
    "molecule_system",
    "make_workload",
    "draw_thetas",
    "draw_directions",
    "batched_workloads",
    "warm_targets",
    "degenerate_system",
    "DEGENERATE_KINDS",
    "transfer_system",
    "hermitian_system",
    "WORKLOADS",
]


@dataclasses.dataclass
class System:
    """A finite-basis TDSE system i a' = (H0 + f(t) M) a with one control."""

    h0: np.ndarray          # (n, n) float64 real symmetric, or complex128 Hermitian
    m: np.ndarray           # (n, n) float64 real symmetric, or complex128 Hermitian
    psi0: np.ndarray        # (n,) complex128
    psi_target: np.ndarray  # (n,) complex128

    @property
    def n(self) -> int:
        return int(self.h0.shape[0])


@dataclasses.dataclass
class Workload:
    """A system plus time grid, Fourier harmonic count and weights."""

    name: str
    system: System
    nt: int
    dt: float
    k: int                  # Fourier harmonics; P = 2K
    gamma: float
    rho: float
    seed: int

    @property
    def p(self) -> int:
        return 2 * self.k


def spectrum_with_gap(rng: np.random.Generator, n: int, lo: float, gap: float) -> np.ndarray:
    """n sorted points in [lo, 0] with every spacing >= gap.

    Draw n uniform points on [lo, -(n-1) gap], sort, add i*gap to the i-th: exactly the
    uniform order statistics conditioned on all spacings >= gap.
    """
    hi = -(n - 1) * gap
    if hi <= lo:
        raise ValueError("gap too large for the interval")
    x = np.sort(rng.uniform(lo, hi, size=n))
    return x + gap * np.arange(n)


def _sym_normal(rng: np.random.Generator, n: int, sigma: float, zero_diag: bool) -> np.ndarray:
    g = rng.normal(0.0, sigma, size=(n, n))
    m = np.triu(g, 1)
    m = m + m.T
    if not zero_diag:
        m = m + np.diag(np.diag(g))
    return m


def _unit(n: int, i: int) -> np.ndarray:
    v = np.zeros(n, dtype=np.complex128)
    v[i] = 1.0
    return v


def _random_unit_in_span(rng: np.random.Generator, n: int, d: int) -> np.ndarray:
    z = np.zeros(n, dtype=np.complex128)
    z[:d] = rng.normal(size=d) + 1j * rng.normal(size=d)
    return z / np.linalg.norm(z)


def tiny_system(rng: np.random.Generator, n: int = 4) -> System:
    """H0 = diag(sorted U[-1.5, 0]); M zero diagonal, off-diagonal N(0, 0.5^2); e0 -> e1."""
    e = np.sort(rng.uniform(-1.5, 0.0, size=n))
    h0 = np.diag(e)
    m = _sym_normal(rng, n, 0.5, zero_diag=True)
    return System(h0, m, _unit(n, 0), _unit(n, 1))


def molecule_system(rng: np.random.Generator, n: int = 36, target_dim: int = 6) -> System:
    """Spectrum U[-3, 0] with gap >= 1e-3; dense M ~ N(0, 0.3^2) (diagonal included);
    ground state -> random unit vector in the span of the lowest ``target_dim`` states."""
    e = spectrum_with_gap(rng, n, -3.0, 1e-3)
    h0 = np.diag(e)
    m = _sym_normal(rng, n, 0.3, zero_diag=False)
    return System(h0, m, _unit(n, 0), _random_unit_in_span(rng, n, min(target_dim, n)))


def transfer_system(n: int, seed: int = 12) -> System:
    """Stand-in for the paper's optimiser-comparison molecules (Sec. IV-B): the molecule recipe
    (spectrum U[-3, 0] with gap >= 1e-3, dense M ~ N(0, 0.3^2)) driven from the lowest
    state e_0 to the highest e_{n-1}, the paper's alpha and beta."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, n])))
    e = spectrum_with_gap(rng, n, -3.0, 1e-3)
    m = _sym_normal(rng, n, 0.3, zero_diag=False)
    return System(np.diag(e), m, _unit(n, 0), _unit(n, n - 1))


def hermitian_system(n: int, seed: int = 13, sigma: float = 0.3) -> System:
    """Stand-in for the paper's random timing systems (Sec. IV-A): H0 = diag(sorted U[-3, 0]),
    M complex Hermitian with Re and Im of the off-diagonal entries ~ N(0, sigma^2 / 2) and a real
    diagonal ~ N(0, sigma^2); alpha = e_0, beta = e_{n-1}."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, n, 31])))
    h0 = np.diag(np.sort(rng.uniform(-3.0, 0.0, n))).astype(np.complex128)
    z = rng.normal(0.0, sigma / np.sqrt(2.0), (n, n)) + 1j * rng.normal(0.0, sigma / np.sqrt(2.0), (n, n))
    m = np.triu(z, 1)
    m = m + m.conj().T + np.diag(rng.normal(0.0, sigma, n))
    return System(h0, m, _unit(n, 0), _unit(n, n - 1))


def _default_weights(dt: float):
    # C = dt * sum_j f_j^2 + |a_J - beta|^2  ->  gamma = 2 dt, rho = 2
    return 2.0 * dt, 2.0


WORKLOADS = {
    "tiny": dict(n=4, nt=500, dt=0.05, k=4, seed=1, kind="tiny"),
    "molecule": dict(n=36, nt=4000, dt=0.02, k=16, seed=2, kind="molecule"),
    "diff": dict(n=128, nt=10000, dt=0.01, k=64, seed=4, kind="molecule"),
    "warm": dict(n=64, nt=4000, dt=0.02, k=32, seed=5, kind="tiny"),
}


def make_workload(name: str, *, n: Optional[int] = None, nt: Optional[int] = None,
                  dt: Optional[float] = None, k: Optional[int] = None,
                  seed: Optional[int] = None) -> Workload:
    """Build a named workload; keyword overrides allow reduced variants for tests."""
    spec = dict(WORKLOADS[name])
    for key, val in (("n", n), ("nt", nt), ("dt", dt), ("k", k), ("seed", seed)):
        if val is not None:
            spec[key] = val
    rng = np.random.Generator(np.random.PCG64(spec["seed"]))
    if spec["kind"] == "tiny":
        sysm = tiny_system(rng, spec["n"])
    else:
        sysm = molecule_system(rng, spec["n"])
    gamma, rho = _default_weights(spec["dt"])
    return Workload(name, sysm, spec["nt"], spec["dt"], spec["k"], gamma, rho, spec["seed"])


def multi_direction_workload(ndir: int = 3, seed: int = 17):
    """The molecule workload with ndir control directions (Sec. II, the x, y, z dipoles): its M is
    the first operator and the others follow the same recipe (dense N(0, 0.3^2), diagonal
    included); each direction gets its own block of the Fourier model (P = ndir x 2K).
    Returns (workload, [M_1, ..., M_ndir])."""
    w = make_workload("molecule")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, w.system.n, ndir])))
    ms = [w.system.m] + [_sym_normal(rng, w.system.n, 0.3, zero_diag=False) for _ in range(ndir - 1)]
    return w, ms


def draw_thetas(p: int, count: int, seed: int, sigma: float = 0.1) -> np.ndarray:
    """(count, p) control coefficients ~ N(0, sigma^2)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7919])))
    return rng.normal(0.0, sigma, size=(count, p))


def draw_directions(p: int, count: int, seed: int) -> np.ndarray:
    """(count, p) unit-norm directions v ~ N(0, I) / |.| for Hessian-vector products."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 104729])))
    v = rng.normal(size=(count, p))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def batched_workloads(count: int = 256, seed: int = 3,
                      sizes=(8, 16, 36, 64, 128), nt_range=(2000, 8000),
                      ks=(8, 16, 32), dt: float = 0.02) -> List[Workload]:
    """Independent problems of uneven size drawn with the tiny-system recipe."""
    ss = np.random.SeedSequence(seed)
    out = []
    for i, child in enumerate(ss.spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        n = int(rng.choice(sizes))
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        k = int(rng.choice(ks))
        sysm = tiny_system(rng, n)
        gamma, rho = _default_weights(dt)
        out.append(Workload(f"batched[{i}]", sysm, nt, dt, k, gamma, rho, seed))
    return out


def warm_targets(n: int, count: int, spawn: int, seed: int = 5, dim: int = 8) -> np.ndarray:
    """(count, n) complex unit targets in the span of the lowest ``dim`` basis states."""
    child = np.random.SeedSequence(seed).spawn(spawn + 1)[spawn]
    rng = np.random.Generator(np.random.PCG64(child))
    z = np.zeros((count, n), dtype=np.complex128)
    z[:, :dim] = rng.normal(size=(count, dim)) + 1j * rng.normal(size=(count, dim))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


DEGENERATE_KINDS = ("h0zero", "doubled", "near_crossing")


def degenerate_system(kind: str, n: int, seed: int = 11) -> System:
    """Systems whose step Hamiltonians H0 + f M have confluent or nearly confluent spectra.

    * ``h0zero``: H0 = 0 and M dense symmetric N(0, 0.3^2).  Every eigenvalue of f M passes
      through 0 together when the field changes sign, and all coincide at f = 0 (theta = 0).
    * ``doubled`` (n even): H0 = diag(e, e) with e the sorted U[-1.5, 0] draw of size n/2, so
      every level is exactly doubly degenerate, and M = R^T blockdiag(m, m) R with R a product
      of plane rotations by random angles on the pairs (i, i + n/2).  R commutes with H0, so
      every H0 + f M keeps an exactly doubly degenerate spectrum, in a basis that mixes the
      copies.
    * ``near_crossing``: the molecule recipe's spectrum with level 1 moved to 1e-9 above level 0;
      with a weak field the pair stays within about |f| of a crossing.

    psi0 = e0; the target is e1 (a unit vector), as in the tiny recipe.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, n, DEGENERATE_KINDS.index(kind)])))
    if kind == "h0zero":
        h0 = np.zeros((n, n))
        m = _sym_normal(rng, n, 0.3, zero_diag=False)
    elif kind == "doubled":
        if n % 2:
            raise ValueError("doubled system needs an even n")
        k = n // 2
        e = np.sort(rng.uniform(-1.5, 0.0, size=k))
        h0 = np.diag(np.concatenate([e, e]))
        mb = _sym_normal(rng, k, 0.5, zero_diag=True)
        m2 = np.zeros((n, n))
        m2[:k, :k] = mb
        m2[k:, k:] = mb
        r = np.eye(n)
        for i, ang in enumerate(rng.uniform(0.0, np.pi, size=k)):
            c, sn = np.cos(ang), np.sin(ang)
            r[i, i], r[i, i + k], r[i + k, i], r[i + k, i + k] = c, -sn, sn, c
        m = r.T @ m2 @ r
        m = 0.5 * (m + m.T)
    elif kind == "near_crossing":
        e = spectrum_with_gap(rng, n, -3.0, 1e-3)
        e[1] = e[0] + 1e-9
        h0 = np.diag(e)
        m = _sym_normal(rng, n, 0.3, zero_diag=False)
    else:
        raise ValueError(f"unknown degenerate kind {kind!r}")
    return System(h0, m, _unit(n, 0), _unit(n, 1))
