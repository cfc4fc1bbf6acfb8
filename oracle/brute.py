"""High-precision brute force for tiny systems (oracle, mpmath).

Test infrastructure only (see ``oracle/__init__.py``).

These routines take no shortcut of the method: the propagators are matrix
exponentials evaluated in multiprecision, the Green's function is the plain
inverse of I + B ... B, and weights are plain determinants.  They pin the
FP64 oracle (QR-stabilized chains, rank-one ratios) on the smallest lattices.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

from . import dqmc


def _mp_matrix(a: np.ndarray):
    return mp.matrix([[mp.mpf(float(x)) for x in row] for row in a])


def mp_propagator(model: dqmc.Model, dps: int = 50):
    """exp(-dtau (K - mu)) in multiprecision."""
    with mp.workdps(dps):
        km = _mp_matrix(model.K) - mp.mpf(model.mu) * mp.eye(model.N)
        return mp.expm(-mp.mpf(model.dtau) * km)


def mp_green(model: dqmc.Model, fields: np.ndarray, l: int, dps: int = 50, e=None) -> np.ndarray:
    """G(l) = [I + B_l ... B_1 B_{L_tau} ... B_{l+1}]^{-1} in multiprecision,
    returned as float64."""
    with mp.workdps(dps):
        if e is None:
            e = mp_propagator(model, dps)
        n = model.N
        a = mp.mpf(model.alpha)
        p = mp.eye(n)
        for j in dqmc.chain_order(l, fields.shape[0]):
            ev = [mp.exp(a * int(x)) for x in fields[j - 1]]
            b = e.copy()
            for c in range(n):
                for r in range(n):
                    b[r, c] *= ev[c]
            p = b * p
        g = (mp.eye(n) + p) ** -1
        return np.array([[float(g[r, c]) for c in range(n)] for r in range(n)])


def mp_log_weight(model: dqmc.Model, fields: np.ndarray, dps: int = 50, e=None):
    """log of prod exp(-alpha s) det(I + B_{L_tau} ... B_1)^2 in multiprecision."""
    with mp.workdps(dps):
        if e is None:
            e = mp_propagator(model, dps)
        n = model.N
        a = mp.mpf(model.alpha)
        p = mp.eye(n)
        for j in range(1, fields.shape[0] + 1):
            ev = [mp.exp(a * int(x)) for x in fields[j - 1]]
            b = e.copy()
            for c in range(n):
                for r in range(n):
                    b[r, c] *= ev[c]
            p = b * p
        det = mp.det(mp.eye(n) + p)
        return 2 * mp.log(abs(det)) - a * int(fields.sum())


def _mp_b(e, a, s_row):
    """B = E diag(exp(alpha s)) in multiprecision."""
    n = e.rows
    ev = [mp.exp(a * int(x)) for x in s_row]
    b = e.copy()
    for c in range(n):
        for r in range(n):
            b[r, c] *= ev[c]
    return b


def mp_pqmc_green(model: dqmc.Model, fields: np.ndarray, p: np.ndarray, l: int, dps: int = 40,
                  e=None) -> np.ndarray:
    """Projector G(l) = I - R (L R)^{-1} L, R = B_l ... B_1 P,
    L = P^T B_{L_tau} ... B_{l+1}, plain products and inverse in
    multiprecision (P given in FP64), returned as float64."""
    with mp.workdps(dps):
        if e is None:
            e = mp_propagator(model, dps)
        a = mp.mpf(model.alpha)
        pm = _mp_matrix(p)
        r = pm.copy()
        for j in range(1, l + 1):
            r = _mp_b(e, a, fields[j - 1]) * r
        lm = pm.T
        for j in range(fields.shape[0], l, -1):   # P^T B_{L_tau}, then B_{L_tau - 1}, ...
            lm = lm * _mp_b(e, a, fields[j - 1])
        g = mp.eye(model.N) - r * ((lm * r) ** -1) * lm
        return np.array([[float(g[i, j]) for j in range(model.N)] for i in range(model.N)])


def mp_pqmc_log_weight(model: dqmc.Model, fields: np.ndarray, p: np.ndarray, dps: int = 40, e=None):
    """log of prod exp(-alpha s) det(P^T B_{L_tau} ... B_1 P)^2 in multiprecision."""
    with mp.workdps(dps):
        if e is None:
            e = mp_propagator(model, dps)
        a = mp.mpf(model.alpha)
        pm = _mp_matrix(p)
        x = pm.copy()
        for j in range(1, fields.shape[0] + 1):
            x = _mp_b(e, a, fields[j - 1]) * x
        det = mp.det(pm.T * x)
        return 2 * mp.log(abs(det)) - a * int(fields.sum())


# ---------------------------------------------------------------------------
# Fock-space brute force (tiny systems): expectation values under a Gaussian
# weight operator, computed from the many-body matrices themselves.
# ---------------------------------------------------------------------------

def fock_annihilators(modes: int):
    """Jordan-Wigner annihilation matrices c_k (2^modes x 2^modes), mode 0 first."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])   # |1> -> |0>
    z = np.diag([1.0, -1.0])
    eye = np.eye(2)
    ops = []
    for k in range(modes):
        m = np.array([[1.0]])
        for j in range(modes):
            m = np.kron(m, z if j < k else (a if j == k else eye))
        ops.append(m)
    return ops


def fock_quadratic(cs, a: np.ndarray, spins: int = 2) -> np.ndarray:
    """sum over spins and sites of c^+_{s,i} A_ij c_{s,j} (mode = s * n + i)."""
    n = a.shape[0]
    out = np.zeros_like(cs[0])
    for s in range(spins):
        for i in range(n):
            for j in range(n):
                if a[i, j] != 0.0:
                    out += a[i, j] * cs[s * n + i].T @ cs[s * n + j]
    return out
