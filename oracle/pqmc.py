"""Projector (zero-temperature) DQMC pieces for the kagome model (oracle, FP64).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. II: the filling is set by a trial wave function that occupies the
lowest N_occ eigenstates of K, with total filling rho = 2 N_occ / N; the
ground state is reached by projecting it over an imaginary time the paper
calls the projection length (Sec. III: beta = 10 for the timings).  Readings
taken where the paper is silent:

* Projection: L_tau = beta / dtau slices B_l = exp(-dtau (K - mu)) exp(V_l)
  (the same B_l and Ising decoupling as the finite-temperature oracle)
  between the trial state on both sides.  With R(l) = B_l ... B_1 P and
  L(l) = P^T B_{L_tau} ... B_{l+1}, the equal-time Green's function between
  slices l and l+1 is G(l) = I - R(l) (L(l) R(l))^{-1} L(l); a flip's weight
  ratio is the same e^{2 alpha s} R^2, R = 1 + Delta (1 - G~_ii), and the
  update and the wrap G(l) = B_l G(l-1) B_l^{-1} are those of the
  finite-temperature case.  mu only rescales every B_l, which G ignores.
* Trial state at an open shell: at the Dirac filling (N_occ = L^2) with
  3 | L the Dirac points are on the momentum grid and the N_occ-th level of
  K is degenerate with the next one, so "the lowest N_occ eigenstates" is
  not one state.  The trial orbitals are therefore the lowest N_occ
  eigenvectors of K_T = K + eps (n_A - n_C) summed over cells, a sublattice
  potential of eps = 0.01 t that splits the Dirac points by 2 eps / sqrt(3)
  and leaves every other level's order unchanged.
* Stabilization: R and L^T are kept as orthonormal N x N_occ panels.  G
  depends on the panels' spans only, so each is replaced by the Q factor of
  its Householder QR after every B (no pivoting or scale factors needed).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import dqmc, lattice

TRIAL_EPS = 0.01


def sublattice_pattern(L: int) -> np.ndarray:
    """(+1, 0, -1) on sublattices (A, B, C) of every cell, site order of Eq. (3)."""
    return np.tile(np.array([1.0, 0.0, -1.0]), L * L)


def trial_K(L: int, t: float = 1.0, eps: float = TRIAL_EPS) -> np.ndarray:
    """K_T = K + eps * diag(sublattice pattern)."""
    return lattice.kagome_K(L, t) + eps * np.diag(sublattice_pattern(L))


def trial_orbitals(L: int, n_occ: int, t: float = 1.0, eps: float = TRIAL_EPS):
    """(P, levels): the lowest n_occ orthonormal eigenvectors of K_T as the
    columns of P (N x n_occ) and all levels of K_T in ascending order.
    Raises if level n_occ is degenerate with level n_occ + 1 (open shell)."""
    w, v = np.linalg.eigh(trial_K(L, t, eps))
    if n_occ < w.size and w[n_occ] - w[n_occ - 1] < 1e-8:
        raise ValueError("open shell: the trial levels n_occ and n_occ+1 are degenerate")
    return v[:, :n_occ].copy(), w


def _orth(x: np.ndarray) -> np.ndarray:
    """An orthonormal basis of span(x) (the Q factor of a Householder QR)."""
    q, _ = scipy.linalg.qr(x, mode="economic")
    return q


def right_panel(model: dqmc.Model, fields: np.ndarray, p: np.ndarray, l: int) -> np.ndarray:
    """Orthonormal basis of span(B_l ... B_1 P) (QR after every B)."""
    r = p.copy()
    for j in range(1, l + 1):
        r = _orth(dqmc.b_matrix(model, fields[j - 1]) @ r)
    return r


def left_panel(model: dqmc.Model, fields: np.ndarray, p: np.ndarray, l: int) -> np.ndarray:
    """Orthonormal basis of span((P^T B_{L_tau} ... B_{l+1})^T), i.e. of
    B_{l+1}^T ... B_{L_tau}^T P (QR after every B^T)."""
    L_tau = fields.shape[0]
    x = p.copy()
    for j in range(L_tau, l, -1):
        x = _orth(dqmc.b_matrix(model, fields[j - 1]).T @ x)
    return x


def green(model: dqmc.Model, fields: np.ndarray, p: np.ndarray, l: int) -> np.ndarray:
    """G(l) = I - R (L R)^{-1} L with the stabilized panels (L = left^T)."""
    r = right_panel(model, fields, p, l)
    lt = left_panel(model, fields, p, l)
    x = np.linalg.solve(lt.T @ r, lt.T)
    return np.eye(model.N) - r @ x


def sweep(model, fields, p, g0, **kw):
    """One upward projector pass l = 1..L_tau from G(0) (dqmc.sweep with the
    projector's G at every stabilization); ends at G(L_tau)."""
    return dqmc.sweep(model, fields, g0, green=lambda f, l: green(model, f, p, l), **kw)


def sweep_down(model, fields, p, g_top, **kw):
    """One downward projector pass l = L_tau..1 from G(L_tau); ends at G(0)."""
    return dqmc.sweep_down(model, fields, g_top, green=lambda f, l: green(model, f, p, l), **kw)
