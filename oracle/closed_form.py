"""Closed-form results used to pin the oracle (TEST INFRASTRUCTURE ONLY).

* eq. (6): characteristic equation m^2 lam^4 + 3 m C lam^2 + C^2 = 0 of the
  equal-parameter two-mass system eq. (3); its roots are purely imaginary,
  lam = +-j omega.
* eq. (4): the secular system gives the mode shape B/A = (m lam^2 + 2C)/C.
* eq. (7): the general solution is a superposition of the normal modes.  The
  printed form pairs cos(omega_1 t) with sin(omega_2 t); it is read here as the
  standard modal superposition x(t) = sum_k phi_k (a_k cos w_k t + b_k/w_k sin w_k t).
* Exact discrete solutions of the two schemes on the normal modes: classic RK4
  applied to q'' = -w^2 q multiplies u = w q + i p by R(-i w h) per step, with
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24; velocity Verlet applies the 2x2 map
  [[1 - th^2/2, h], [-h w^2 (1 - th^2/4), 1 - th^2/2]] (th = w h), whose n-th
  power follows from Cayley-Hamilton.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


# --------------------------------------------------------------------------
# section 2: the two-mass system
# --------------------------------------------------------------------------

def eq6_lambda_squared(m: float, C: float):
    """Roots in lam^2 of m^2 lam^4 + 3 m C lam^2 + C^2 = 0 (quadratic formula)."""
    a, b, c = m * m, 3.0 * m * C, C * C
    disc = math.sqrt(b * b - 4.0 * a * c)
    return ((-b - disc) / (2.0 * a), (-b + disc) / (2.0 * a))   # (fast, slow)


def eq6_omegas(m: float, C: float):
    """(omega_fast, omega_slow) with lam = +-j omega."""
    l_fast, l_slow = eq6_lambda_squared(m, C)
    return math.sqrt(-l_fast), math.sqrt(-l_slow)


def eq4_mode_ratio(m: float, C: float, omega: float) -> float:
    """B/A from the first row of eq. (4) with lam^2 = -omega^2."""
    return (2.0 * C - m * omega * omega) / C


def two_mass_equal(t, m: float, C: float, x0, v0):
    """Closed-form trajectory of eq. (3): superposition of the two normal modes
    with the eq. (4) shapes (1, r_k) and eq. (6) frequencies.  Returns
    (x [len(t), 2], v [len(t), 2])."""
    t = np.asarray(t, dtype=np.float64)
    wf, ws = eq6_omegas(m, C)
    rf, rs = eq4_mode_ratio(m, C, wf), eq4_mode_ratio(m, C, ws)
    P = np.array([[1.0, 1.0], [rf, rs]])            # columns are mode shapes
    a = np.linalg.solve(P, np.asarray(x0, dtype=np.float64))
    b = np.linalg.solve(P, np.asarray(v0, dtype=np.float64))
    w = np.array([wf, ws])
    ct, st = np.cos(np.outer(t, w)), np.sin(np.outer(t, w))
    q = a * ct + (b / w) * st
    qd = -a * w * st + b * ct
    return q @ P.T, qd @ P.T


# --------------------------------------------------------------------------
# chains as matrices
# --------------------------------------------------------------------------

def chain_matrices(m, k):
    """Diagonal M and tridiagonal K of the fixed-free chain (eq. (2) for s bodies)."""
    m = np.asarray(m, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    s = m.shape[0]
    M = np.diag(m)
    K = np.zeros((s, s))
    for i in range(s):
        K[i, i] += k[i]
        if i >= 1:
            K[i - 1, i - 1] += k[i]
            K[i - 1, i] -= k[i]
            K[i, i - 1] -= k[i]
    return M, K


def uniform_chain_omegas(s: int, k: float, m: float) -> np.ndarray:
    """Natural frequencies of a uniform fixed-free chain:
    omega_j = 2 sqrt(k/m) sin((2j-1) pi / (2(2s+1))), j = 1..s."""
    j = np.arange(1, s + 1)
    return 2.0 * math.sqrt(k / m) * np.sin((2 * j - 1) * math.pi / (2 * (2 * s + 1)))


# --------------------------------------------------------------------------
# modal machinery (generalised symmetric-definite eigenproblem K phi = w^2 M phi)
# --------------------------------------------------------------------------

def modes(M, K):
    """Frequencies and M-orthonormal mode shapes (LAPACK sygv via scipy)."""
    lam, phi = scipy.linalg.eigh(K, M)
    return np.sqrt(lam), phi


def _modal_coords(M, phi, x0, v0):
    return phi.T @ M @ x0, phi.T @ M @ v0


def modal_solution(t, M, K, x0, v0):
    """Exact solution of x'' = -M^-1 K x at the times t: (x [len(t), s], v [len(t), s])."""
    w, phi = modes(M, K)
    a, b = _modal_coords(M, phi, np.asarray(x0, float), np.asarray(v0, float))
    t = np.asarray(t, dtype=np.float64)
    ct, st = np.cos(np.outer(t, w)), np.sin(np.outer(t, w))
    q = a * ct + (b / w) * st
    qd = -a * w * st + b * ct
    return q @ phi.T, qd @ phi.T


def rk4_amplification(theta):
    z = -1j * np.asarray(theta, dtype=np.float64)
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def rk4_discrete(n, h, M, K, x0, v0):
    """State after each step count in ``n`` of classic RK4 with step h, exactly
    (up to rounding): u_n = R(-i w h)^n u_0 per mode, u = w q + i p."""
    w, phi = modes(M, K)
    q0, p0 = _modal_coords(M, phi, np.asarray(x0, float), np.asarray(v0, float))
    u0 = w * q0 + 1j * p0
    R = rk4_amplification(w * h)
    n = np.asarray(n, dtype=np.float64)[:, None]
    un = (np.abs(R) ** n) * np.exp(1j * n * np.angle(R)) * u0
    q = un.real / w
    p = un.imag
    return q @ phi.T, p @ phi.T


def verlet_discrete(n, h, M, K, x0, v0):
    """State after each step count in ``n`` of velocity Verlet (kick-drift-kick)
    with step h, exactly (up to rounding), per mode."""
    w, phi = modes(M, K)
    q0, p0 = _modal_coords(M, phi, np.asarray(x0, float), np.asarray(v0, float))
    th = w * h
    c = 1.0 - th * th / 2.0
    phi_ang = np.arccos(c)
    sphi = np.sin(phi_ang)
    n = np.asarray(n, dtype=np.float64)[:, None]
    cn, sn = np.cos(n * phi_ang), np.sin(n * phi_ang)
    # M^n = cos(n phi) I + sin(n phi)/sin(phi) (Mstep - cos(phi) I); Mstep - c I = [[0, h],[-h w^2 (1 - th^2/4), 0]]
    g = sn / sphi
    q = cn * q0 + g * h * p0
    p = cn * p0 - g * h * w * w * (1.0 - th * th / 4.0) * q0
    return q @ phi.T, p @ phi.T


def rk4_energy_factor(theta):
    """|R(-i theta)|^2 = 1 - theta^6/72 + theta^8/576: the per-step energy factor of RK4."""
    theta = np.asarray(theta, dtype=np.float64)
    return 1.0 - theta ** 6 / 72.0 + theta ** 8 / 576.0


# --------------------------------------------------------------------------
# damped, driven systems: M x'' + (alpha M + beta K) x' + K x = F cos(W t)
# --------------------------------------------------------------------------

def _modes(M, K):
    """omega^2 and M-orthonormal mode shapes of the pencil (K, M) (LAPACK)."""
    w2, Phi = scipy.linalg.eigh(K, M)
    return w2, Phi


def driven_modal_solution(t, M, K, alpha, beta, F, W, x0, v0):
    """Exact solution by normal modes.  Mode k obeys q'' + g_k q' + w_k^2 q =
    f_k cos(W t) with g_k = alpha + beta w_k^2, f = Phi^T F.  Particular part
    Re(G e^{iWt}), G = f / (w^2 - W^2 + i g W) (the receptance); the
    homogeneous part from its initial value by the 2x2 matrix exponential of
    [[0, 1], [-w^2, -g]] (scipy.linalg.expm).  Returns (x, v), [len(t), s]."""
    t = np.asarray(t, dtype=np.float64)
    w2, Phi = _modes(M, K)
    q0 = Phi.T @ (M @ np.asarray(x0, dtype=np.float64))
    p0 = Phi.T @ (M @ np.asarray(v0, dtype=np.float64))
    fk = Phi.T @ (np.zeros(len(w2)) if F is None else np.asarray(F, dtype=np.float64))
    g = alpha + beta * w2
    G = fk / (w2 - W * W + 1j * g * W)
    q = np.empty((len(t), len(w2)))
    p = np.empty_like(q)
    for k in range(len(w2)):
        L = np.array([[0.0, 1.0], [-w2[k], -g[k]]])
        z0 = np.array([q0[k] - G[k].real, p0[k] + W * G[k].imag])
        for i, ti in enumerate(t):
            z = scipy.linalg.expm(L * ti) @ z0
            e = G[k] * np.exp(1j * W * ti)
            q[i, k] = z[0] + e.real
            p[i, k] = z[1] + (1j * W * e).real
    return q @ Phi.T, p @ Phi.T


def steady_amplitude(M, K, alpha, beta, F, W):
    """|G_k| = |f_k| / sqrt((w_k^2 - W^2)^2 + (g_k W)^2) per mode: the
    amplitude of the driven response once the transient has decayed."""
    w2, Phi = _modes(M, K)
    fk = Phi.T @ np.asarray(F, dtype=np.float64)
    g = alpha + beta * w2
    return np.abs(fk) / np.sqrt((w2 - W * W) ** 2 + (g * W) ** 2)


def rk4_damped_discrete(steps, h, M, K, alpha, beta, x0, v0):
    """Exact discrete solution of classic RK4 on the free damped system: per
    mode the step multiplies (q, q') by R(hL_k) = sum_{j<=4} (hL_k)^j / j!,
    L_k = [[0, 1], [-w_k^2, -g_k]]."""
    w2, Phi = _modes(M, K)
    q0 = Phi.T @ (M @ np.asarray(x0, dtype=np.float64))
    p0 = Phi.T @ (M @ np.asarray(v0, dtype=np.float64))
    g = alpha + beta * w2
    steps = np.asarray(steps)
    q = np.empty((len(steps), len(w2)))
    p = np.empty_like(q)
    for k in range(len(w2)):
        hL = h * np.array([[0.0, 1.0], [-w2[k], -g[k]]])
        R = np.eye(2) + hL + hL @ hL / 2 + hL @ hL @ hL / 6 + hL @ hL @ hL @ hL / 24
        for i, n in enumerate(steps):
            z = np.linalg.matrix_power(R, int(n)) @ np.array([q0[k], p0[k]])
            q[i, k], p[i, k] = z
    return q @ Phi.T, p @ Phi.T
