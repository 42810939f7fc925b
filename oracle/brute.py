"""Dense brute force for tiny lattices (a few dozen sites). TEST INFRASTRUCTURE ONLY.

An independent second reading of the model, used to pin the C oracle. The one-step
transition of section 2.1 is written as dense matrices:

  T0[i, j] = sum over links j -> i of p(j->i), plus stay(i) on the diagonal,
  T1[i, j] = sum over links j -> i of p(j->i) d_a(j->i),
  T2[i, j] = sum over links j -> i of p(j->i) d_a(j->i)^2,

with p(j->i) = p0 * min(1, exp(-(F_i - F_j))) (Eq. (1)) and d_a the unwrapped hop
component along axis a. Then one step is rho <- T0 rho, m <- diag(exp(i theta)) T0 m
(Eq. (13)), and the displacement moments follow the block lower-triangular system
[rho, M1, M2] <- [[T0, 0, 0], [T1, T0, 0], [T2, 2 T1, T0]] [rho, M1, M2].

It also gives the velocity autocorrelation of Eq. (4) (Kohn's discretisation of the
Green-Kubo integral, Eq. (3)) and the continuous-time generator whose matrix exponential
is the small-step limit of the chain.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

PERIODIC, CLOSED, RESERVOIR = 0, 1, 2


def _sites(shape_xyz):
    nx, ny, nz = shape_xyz
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                yield x, y, z, x + nx * (y + ny * z)


def links(shape_xyz, bc):
    """All directed links (source j, target i, hop vector) between lattice sites."""
    nx, ny, nz = shape_xyz
    dims = (nx, ny, nz)
    out = []
    for x, y, z, j in _sites(shape_xyz):
        for axis in range(3):
            for sign in (+1, -1):
                c = [x, y, z]
                c[axis] += sign
                if not 0 <= c[axis] < dims[axis]:
                    if bc[axis] != PERIODIC:
                        continue
                    c[axis] %= dims[axis]
                i = c[0] + nx * (c[1] + ny * c[2])
                hop = [0, 0, 0]
                hop[axis] = sign
                out.append((j, i, tuple(hop)))
    return out


def ghost_links(shape_xyz, bc):
    """(site i, face f, hop vector ghost -> i) for every face site of a reservoir axis;
    face f = 2 * axis + side, side 0 below coordinate 0 and 1 above n - 1."""
    dims = tuple(shape_xyz)
    out = []
    for x, y, z, i in _sites(shape_xyz):
        c = (x, y, z)
        for axis in range(3):
            if bc[axis] != RESERVOIR:
                continue
            for side, at, sign in ((0, 0, +1), (1, dims[axis] - 1, -1)):
                if c[axis] == at:
                    hop = [0, 0, 0]
                    hop[axis] = sign
                    out.append((i, 2 * axis + side, tuple(hop)))
    return out


def _acc(Ffrom, Fto):
    """Eq. (1) written as a minimum; 0 into a site of infinite free energy."""
    if math.isinf(Fto) and Fto > 0:
        return 0.0
    return min(1.0, math.exp(-(Fto - Ffrom)))


def matrices(shape_xyz, bc, F, p0, axis=0, mobility=None, ghost=None):
    """T0, T1, T2 for displacement along `axis`; F flattened in x-fastest order, +inf for
    inaccessible sites (no row, no column). With `mobility` the link i-j is scaled by
    min(mu_i, mu_j). With reservoir axes (ghost: 24 values, F, rho, Re m, Im m per face) it
    also returns the per-step sources (s0, sm, s1, s2) that the ghost sites send in, so that
    rho' = T0 rho + s0, m' = diag(e^{i theta}) (T0 m + sm), and so on."""
    F = np.asarray(F, dtype=np.float64).reshape(-1)
    n = F.size
    mu = np.ones(n) if mobility is None else np.asarray(mobility, dtype=np.float64).reshape(-1)
    open_ = ~(np.isinf(F) & (F > 0))
    T0 = np.zeros((n, n))
    T1 = np.zeros((n, n))
    T2 = np.zeros((n, n))
    leave = np.zeros(n)
    for j, i, hop in links(shape_xyz, bc):
        if not (open_[i] and open_[j]):
            continue
        p = p0 * min(mu[i], mu[j]) * _acc(F[j], F[i])
        d = hop[axis]
        T0[i, j] += p
        T1[i, j] += p * d
        T2[i, j] += p * d * d
        leave[j] += p
    s0 = np.zeros(n)
    sm = np.zeros(n, dtype=np.complex128)
    s1 = np.zeros(n)
    s2 = np.zeros(n)
    for i, f, hop in ghost_links(shape_xyz, bc):
        if not open_[i]:
            continue
        Fg, rg, reg, img = ghost[4 * f:4 * f + 4]
        a = min(mu[i], 1.0)
        leave[i] += p0 * a * _acc(F[i], Fg)
        p_in = p0 * a * _acc(Fg, F[i])
        d = hop[axis]
        s0[i] += p_in * rg
        sm[i] += p_in * complex(reg, img)
        s1[i] += p_in * d * rg
        s2[i] += p_in * d * d * rg
    T0[np.arange(n), np.arange(n)] += np.where(open_, 1.0 - leave, 0.0)
    if ghost is None:
        return T0, T1, T2
    return T0, T1, T2, (s0, sm, s1, s2)


def run_affine(T0, T1, T2, src, theta, rho0, m0, n_steps):
    """Steps the dense affine system of a lattice with reservoir faces; returns per step the
    sums of rho, m and the moments along the axis of T1/T2 (each from a zero start)."""
    s0, sm, s1, s2 = src
    A = np.exp(1j * theta)
    rho = np.asarray(rho0, dtype=np.float64).copy()
    m = np.asarray(m0, dtype=np.complex128).copy()
    M1 = np.zeros_like(rho)
    M2 = np.zeros_like(rho)
    out = np.empty((n_steps + 1, 4), dtype=np.complex128)
    out[0] = rho.sum(), m.sum(), 0.0, 0.0
    for t in range(1, n_steps + 1):
        rho, m, M1, M2 = (T0 @ rho + s0, A * (T0 @ m + sm), T0 @ M1 + T1 @ rho + s1,
                          T0 @ M2 + 2.0 * (T1 @ M1) + T2 @ rho + s2)
        out[t] = rho.sum(), m.sum(), M1.sum(), M2.sum()
    return out


def phases(delta_ppm, dt, nu0):
    return 2.0 * math.pi * np.asarray(delta_ppm, dtype=np.float64).reshape(-1) * 1e-6 * nu0 * dt


def fid(T0, theta, m0, n_steps):
    """G(n) = 1^T A^n m0 with A = diag(exp(i theta)) T0, for n = 0..n_steps."""
    A = np.exp(1j * theta)[:, None] * T0
    m = np.asarray(m0, dtype=np.complex128).copy()
    out = np.empty(n_steps + 1, dtype=np.complex128)
    out[0] = m.sum()
    for t in range(1, n_steps + 1):
        m = A @ m
        out[t] = m.sum()
    return out


def fid_power(T0, theta, m0, n):
    """1^T A^n m0 through numpy's matrix power (repeated squaring)."""
    A = np.exp(1j * theta)[:, None] * T0
    return np.linalg.matrix_power(A, n) @ np.asarray(m0, dtype=np.complex128)


def moments(T0, T1, T2, rho0, n_steps):
    """Sums of rho, M1, M2 along the axis of T1/T2 for n = 0..n_steps (M1 = M2 = 0 at start)."""
    n = T0.shape[0]
    Z = np.zeros((n, n))
    B = np.block([[T0, Z, Z], [T1, T0, Z], [T2, 2.0 * T1, T0]])
    v = np.concatenate([np.asarray(rho0, dtype=np.float64), np.zeros(2 * n)])
    out = np.empty((n_steps + 1, 3))
    for t in range(n_steps + 1):
        if t:
            v = B @ v
        out[t] = v[:n].sum(), v[n:2 * n].sum(), v[2 * n:].sum()
    return out


def vacf(T0, T1, T2, rho_eq, t_max):
    """C(0) = <dx^2> per step and C(tau) = <dx_1 dx_{1+tau}> for tau = 1..t_max-1 (Eq. (4)),
    from a stationary start rho_eq: C(tau) = 1^T T1 T0^(tau-1) T1 rho_eq."""
    one = np.ones(T0.shape[0])
    c0 = one @ (T2 @ rho_eq)
    v = T1 @ rho_eq
    w = one @ T1
    C = np.empty(t_max)
    C[0] = c0
    for tau in range(1, t_max):
        C[tau] = w @ v
        v = T0 @ v
    return C


def msd_from_vacf(C, t):
    """Einstein sum of a stationary increment process: t C0 + 2 sum_{tau=1}^{t-1} (t - tau) C(tau)."""
    tau = np.arange(1, t)
    return t * C[0] + 2.0 * np.sum((t - tau) * C[1:t])


def expm_fid(T_ref, theta, m0, t):
    """1^T expm(t (Q + i Theta)) m0 with the generator Q = T_ref - I."""
    n = T_ref.shape[0]
    Gen = (T_ref - np.eye(n)) + 1j * np.diag(theta)
    return (scipy.linalg.expm(t * Gen) @ np.asarray(m0, dtype=np.complex128)).sum()
