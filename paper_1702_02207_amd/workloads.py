"""Seeded synthetic inputs for the coupled-oscillator integrator.

This module is the only code shared by the GPU path's tests/benchmarks and the
FP64 oracle's tests. It draws random system parameters and initial conditions
and picks the step size; it performs none of the integration, energy or
A-formation arithmetic of the method itself.

Systems follow eq. (1) of the paper, sum_j (m_ij x_j'' + k_ij x_j) = 0.  Two
storage kinds are produced:

* chain: the fixed-free spring chain of eq. (2) (Fig. 1) generalised to ``s``
  masses.  ``m[b, i]`` is the mass of body i, ``k[b, 0]`` the wall spring on
  body 0, ``k[b, i]`` (i >= 1) the spring joining bodies i-1 and i; the last
  body is free.  For s = 2 this is eq. (2) with C1 = k[:, 0], C2 = k[:, 1].
* dense: full symmetric positive definite M and symmetric K, s x s row-major.

Step-size rule (the paper names no step size): dt = 0.01 / omega_max per
instance, where omega_max^2 is the largest generalised eigenvalue of (K, M).
It is computed here in FP64 with LAPACK routines and passed to both sides as
an input, so both integrate with the identical double.

Seeds: numpy PCG64 with seed 1702022070 + config index (0..4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.linalg

SEED_BASE = 1702022070


def _rng(config_index: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_index, salt]))


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


@dataclasses.dataclass
class ChainBatch:
    """A batch of independent fixed-free chains (diagonal M, tridiagonal K)."""
    m: np.ndarray          # [batch, s] float64 masses
    k: np.ndarray          # [batch, s] float64 springs, k[:,0] = wall spring
    dt: np.ndarray         # [batch] float64
    x0: np.ndarray         # [batch, s] float64
    v0: np.ndarray         # [batch, s] float64
    nsteps: int
    out_stride: int

    @property
    def batch(self) -> int:
        return self.m.shape[0]

    @property
    def s(self) -> int:
        return self.m.shape[1]

    def subset(self, idx) -> "ChainBatch":
        idx = np.asarray(idx)
        return ChainBatch(self.m[idx].copy(), self.k[idx].copy(), self.dt[idx].copy(),
                          self.x0[idx].copy(), self.v0[idx].copy(), self.nsteps, self.out_stride)


@dataclasses.dataclass
class DenseBatch:
    """Instances of eq. (1) with full M, K.  If ``shared``, M and K are [s, s]
    and every instance uses them with the single step dt[0]; otherwise they are
    [batch, s, s] with dt[batch]."""
    M: np.ndarray
    K: np.ndarray
    dt: np.ndarray
    x0: np.ndarray         # [batch, s]
    v0: np.ndarray         # [batch, s]
    nsteps: int
    out_stride: int
    shared: bool = True

    @property
    def batch(self) -> int:
        return self.x0.shape[0]

    @property
    def s(self) -> int:
        return self.x0.shape[1]

    def subset(self, idx) -> "DenseBatch":
        idx = np.asarray(idx)
        if self.shared:
            return DenseBatch(self.M, self.K, self.dt, self.x0[idx].copy(), self.v0[idx].copy(),
                              self.nsteps, self.out_stride, True)
        return DenseBatch(self.M[idx].copy(), self.K[idx].copy(), self.dt[idx].copy(),
                          self.x0[idx].copy(), self.v0[idx].copy(), self.nsteps, self.out_stride, False)


# ---------------------------------------------------------------------------
# step-size helpers (input recipe, LAPACK eigenvalues)
# ---------------------------------------------------------------------------

def chain_omega_max(m: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Largest natural frequency of each chain, from the symmetric tridiagonal
    matrix M^-1/2 K M^-1/2 (LAPACK stebz via scipy)."""
    m = np.atleast_2d(m)
    k = np.atleast_2d(k)
    out = np.empty(m.shape[0])
    s = m.shape[1]
    for b in range(m.shape[0]):
        kr = np.r_[k[b, 1:], 0.0]
        d = (k[b] + kr) / m[b]
        if s == 1:
            out[b] = math.sqrt(d[0])
            continue
        e = -k[b, 1:] / np.sqrt(m[b, :-1] * m[b, 1:])
        lam = scipy.linalg.eigh_tridiagonal(d, e, eigvals_only=True, select="i",
                                            select_range=(s - 1, s - 1))
        out[b] = math.sqrt(lam[0])
    return out


def chain2_omega_max(m: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Vectorised largest frequency for s = 2 chains (batched 2x2 eigvalsh)."""
    m1, m2 = m[:, 0], m[:, 1]
    c1, c2 = k[:, 0], k[:, 1]
    S = np.empty((m.shape[0], 2, 2))
    S[:, 0, 0] = (c1 + c2) / m1
    S[:, 1, 1] = c2 / m2
    S[:, 0, 1] = S[:, 1, 0] = -c2 / np.sqrt(m1 * m2)
    return np.sqrt(np.linalg.eigvalsh(S)[:, -1])


def dense_omega_max(M: np.ndarray, K: np.ndarray) -> float:
    lam = scipy.linalg.eigh(K, M, eigvals_only=True)
    return math.sqrt(lam[-1])


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def c1_paper_two_mass(x0=(1.0, 0.0), v0=(0.0, 0.0), nsteps: int = 100_000,
                      out_stride: int = 1) -> ChainBatch:
    """eq. (3) with m = 2, C = 2025 (the dimensionless values read from the
    worked example of section 2), dt = 1e-5, classic RK4 in FP64."""
    m = np.array([[2.0, 2.0]])
    k = np.array([[2025.0, 2025.0]])
    return ChainBatch(m, k, np.array([1e-5]), np.array([x0], dtype=np.float64),
                      np.array([v0], dtype=np.float64), nsteps, out_stride)


def c2_two_dof_ensemble(batch: int = 1 << 20, nsteps: int = 10_000,
                        out_stride: int = 100) -> ChainBatch:
    """2^20 independent eq. (2) systems: m1, m2 ~ LogU[0.5, 5], C1, C2 ~ LogU[1e2, 1e4],
    x0, v0 ~ N(0, 1), dt = 0.01/omega_max.  Instance b is the same for every
    ``batch`` >= b + 1 (each quantity is drawn for the full 2^20 ensemble)."""
    full = 1 << 20
    if batch > full:
        raise ValueError("C2 has at most 2^20 instances")
    rng = _rng(1)
    m = _log_uniform(rng, 0.5, 5.0, (full, 2))[:batch]
    k = _log_uniform(rng, 1e2, 1e4, (full, 2))[:batch]
    x0 = rng.normal(0.0, 1.0, (full, 2))[:batch]
    v0 = rng.normal(0.0, 1.0, (full, 2))[:batch]
    dt = 0.01 / chain2_omega_max(m, k)
    return ChainBatch(m.copy(), k.copy(), dt, x0.copy(), v0.copy(), nsteps, out_stride)


def random_chain(rng, batch: int, s: int):
    m = rng.uniform(0.5, 2.0, (batch, s))
    k = _log_uniform(rng, 1e2, 1e4, (batch, s))
    return m, k


def c3_spring_chain(batch: int = 4096, s: int = 1024, nsteps: int = 100_000,
                    out_stride: int = 1000, instances: Optional[np.ndarray] = None) -> ChainBatch:
    """Fixed-free chains, masses U[0.5, 2], springs LogU[1e2, 1e4], x0 ~ N(0, var 1e-2)
    (sigma = 0.1), v0 = 0.  ``instances`` selects a subset without computing the
    step size of the others."""
    full = 4096
    rng = _rng(2)
    m, k = random_chain(rng, full, s)
    x0 = rng.normal(0.0, 0.1, (full, s))
    idx = np.arange(batch) if instances is None else np.asarray(instances)
    m, k, x0 = m[idx], k[idx], x0[idx]
    dt = 0.01 / chain_omega_max(m, k)
    return ChainBatch(m, k, dt, x0, np.zeros_like(x0), nsteps, out_stride)


@dataclasses.dataclass
class Excitation:
    """Rayleigh damping alpha M + beta K and a force F cos(omega t) per instance."""
    alpha: float
    beta: float
    F: np.ndarray          # [batch, s] float64
    omega: np.ndarray      # [batch] float64

    def subset(self, idx) -> "Excitation":
        idx = np.asarray(idx)
        return Excitation(self.alpha, self.beta, self.F[idx].copy(), self.omega[idx].copy())


def c3_driven_chain(batch: int = 4096, s: int = 1024, nsteps: int = 10_000, out_stride: int = 1000):
    """The C3 chains (same masses, springs, x0) with light Rayleigh damping
    (alpha = 0.05, beta = 1e-5), forces F ~ N(0, 10^2) per DOF and one
    frequency omega ~ U[1, 100] per chain.  Returns (ChainBatch, Excitation)."""
    w = c3_spring_chain(batch=batch, s=s, nsteps=nsteps, out_stride=out_stride)
    rng = _rng(2, salt=1)
    F = rng.normal(0.0, 10.0, (4096, s))[:batch]
    omega = rng.uniform(1.0, 100.0, 4096)[:batch]
    return w, Excitation(0.05, 1e-5, F.copy(), omega.copy())


def c3_vdp_chain(batch: int = 4096, s: int = 1024, nsteps: int = 10_000, out_stride: int = 1000,
                  mu: float = 20.0):
    """The C3 chains (same masses, springs, x0 ~ N(0, 1e-2)) with a Van der
    Pol element on every body, mu = 20: over the run (about 0.36 time units)
    the elements pump the small initial motion towards their limit cycles.
    Returns (ChainBatch, mu)."""
    return c3_spring_chain(batch=batch, s=s, nsteps=nsteps, out_stride=out_stride), mu


def c4_driven_dense(batch: int = 8192, s: int = 256, nsteps: int = 10_000, out_stride: int = 1000):
    """The C4 dense system (one operator shared by every instance, same x0)
    with Rayleigh damping alpha = 0.02, beta = 1e-3, forces F ~ N(0, 1) per
    DOF and one frequency omega ~ U[0.2, 2] per instance (the system's modes
    span about 0.25 to 1.7 rad per unit time).  Returns (DenseBatch, Excitation)."""
    w = c4_dense_shared(batch=batch, s=s, nsteps=nsteps, out_stride=out_stride)
    rng = _rng(3, salt=1)
    F = rng.normal(0.0, 1.0, (8192, s))[:batch]
    omega = rng.uniform(0.2, 2.0, 8192)[:batch]
    return w, Excitation(0.02, 1e-3, F.copy(), omega.copy())


def haar_orthogonal(rng, s: int) -> np.ndarray:
    g = rng.normal(0.0, 1.0, (s, s))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def random_dense_system(rng, s: int):
    """M = I + Q diag(U[0,1]) Q^T (Q Haar), K = G G^T / s + 0.1 I (G ~ N(0,1))."""
    q = haar_orthogonal(rng, s)
    d = rng.uniform(0.0, 1.0, s)
    M = np.eye(s) + (q * d[None, :]) @ q.T
    M = 0.5 * (M + M.T)
    g = rng.normal(0.0, 1.0, (s, s))
    K = g @ g.T / s + 0.1 * np.eye(s)
    K = 0.5 * (K + K.T)
    return M, K


def c4_dense_shared(batch: int = 8192, s: int = 256, nsteps: int = 10_000,
                    out_stride: int = 1000) -> DenseBatch:
    """One dense SPD system shared by ``batch`` instances, x0 ~ N(0,1), v0 = 0."""
    rng = _rng(3)
    M, K = random_dense_system(rng, s)
    x0 = rng.normal(0.0, 1.0, (8192 if batch <= 8192 else batch, s))[:batch]
    dt = np.array([0.01 / dense_omega_max(M, K)])
    return DenseBatch(M, K, dt, x0.copy(), np.zeros((batch, s)), nsteps, out_stride, True)


@dataclasses.dataclass
class Request:
    """One served integration: a single instance of either kind."""
    rid: int
    arrival: float         # seconds after stream start
    kind: str              # "chain" | "dense"
    system: object         # ChainBatch or DenseBatch with batch == 1


def c5_request_stream(n_requests: int = 200, qps: float = 100.0, s_max: int = 2048,
                      nsteps_range=(1_000, 100_000), seed_salt: int = 0):
    """Poisson arrivals at ``qps``; each request is a chain or a dense SPD
    system (50/50), s = round(exp U[ln 2, ln s_max]), nsteps = round(exp
    U[ln 1e3, ln 1e5]), out_stride = ceil(nsteps / 64); parameters as in the
    chain and dense workloads above."""
    rng = _rng(4, seed_salt)
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / qps)
        kind = "chain" if rng.uniform() < 0.5 else "dense"
        s = int(round(math.exp(rng.uniform(math.log(2), math.log(s_max)))))
        nsteps = int(round(math.exp(rng.uniform(math.log(nsteps_range[0]),
                                                math.log(nsteps_range[1])))))
        out_stride = max(1, math.ceil(nsteps / 64))
        sub = np.random.Generator(np.random.PCG64([SEED_BASE + 4, seed_salt, rid + 1]))
        if kind == "chain":
            m, k = random_chain(sub, 1, s)
            x0 = sub.normal(0.0, 0.1, (1, s))
            dt = 0.01 / chain_omega_max(m, k)
            sysm = ChainBatch(m, k, dt, x0, np.zeros_like(x0), nsteps, out_stride)
        else:
            M, K = random_dense_system(sub, s)
            x0 = sub.normal(0.0, 1.0, (1, s))
            dt = np.array([0.01 / dense_omega_max(M, K)])
            sysm = DenseBatch(M, K, dt, x0, np.zeros_like(x0), nsteps, out_stride, True)
        reqs.append(Request(rid, t, kind, sysm))
    return reqs
