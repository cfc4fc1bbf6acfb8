"""Equal-time estimators of Secs. IV-V from one configuration's G (oracle, FP64).

Test infrastructure only (see ``oracle/__init__.py``).

For one Hubbard-Stratonovich configuration the weight is a Gaussian operator,
so expectation values of products of fermion operators follow from Wick's
theorem with G_ab = <c_a c_b^+> (the same for both spins under the charge
decoupling).  The Monte-Carlo average of these per-configuration values is
the caller's (the correlation ratio and the order parameter are ratios and
roots of averages).

* Pairing structure factor, symmetric form (Sec. IV):
  S_Pair(Q) = (1/N) sum_ij e^{iQ.(r_i - r_j)} <D_i^+ D_j + D_j D_i^+>,
  D_i = c_{i dn} c_{i up}; with one spin's contractions per factor
  <D_i^+ D_j> = (delta_ij - G_ji)^2 and <D_j D_i^+> = G_ji^2.
* CDW field (Sec. V): phi(Q) = (1/N) sum_cells e^{iQ.R} (n_A + w n_B + w^2 n_C),
  w = e^{2 pi i / 3}, n = n_up + n_dn; D(Q)^2 = <phi^+ phi> with
  <n_a n_b> = 4 (1 - G_aa)(1 - G_bb) + 2 (delta_ab - G_ba) G_ab.

Readings where the paper is silent:
* Positions.  Cell x = (x1, x2) at x1 a1 + x2 a2 with |a1| = |a2| and a 60
  degree angle; the bonds of Eq. (3) then make B sit at -a2/2 and C at -a1/2
  from A (B's two A neighbours are A(x) and A(x - a2); C's are A(x) and
  A(x - a1)), which gives every bond the same length.  Momenta
  Q = (2 pi / L)(m1 b1 + m2 b2) with b_i . a_j = 2 pi delta_ij, so
  Q . r = (2 pi / L)(m1 X1 + m2 X2) for a site at X1 a1 + X2 a2.
* Gamma + delta k: m = (1, 0) and m = (0, 1), both returned.
* K: the Dirac point, m = (L/3, 2L/3) (the momentum (2 pi/3, -2 pi/3) of the
  cell coordinates; on the grid when 3 | L).
* The 1/N of phi is the number of sites N (the paper's symbol), the sum runs
  over cells R (the cell position).
"""
from __future__ import annotations

import numpy as np

OMEGA = np.exp(2j * np.pi / 3)
SUB_OFFSET = np.array([[0.0, 0.0], [0.0, -0.5], [-0.5, 0.0]])  # (X1, X2) offsets of A, B, C


def site_coords(L: int) -> np.ndarray:
    """(N, 2) fractional coordinates (X1, X2) of every site, order of Eq. (3)."""
    out = np.zeros((3 * L * L, 2))
    for x1 in range(L):
        for x2 in range(L):
            for s in range(3):
                out[(x1 * L + x2) * 3 + s] = (x1 + SUB_OFFSET[s, 0], x2 + SUB_OFFSET[s, 1])
    return out


def cell_coords(L: int) -> np.ndarray:
    """(N, 2) coordinates of the cell each site belongs to."""
    out = np.zeros((3 * L * L, 2))
    for x1 in range(L):
        for x2 in range(L):
            out[(x1 * L + x2) * 3:(x1 * L + x2) * 3 + 3] = (x1, x2)
    return out


def phases(coords: np.ndarray, L: int, m) -> np.ndarray:
    """e^{i Q.r} for Q = (2 pi / L)(m1 b1 + m2 b2)."""
    return np.exp(2j * np.pi / L * (m[0] * coords[:, 0] + m[1] * coords[:, 1]))


def pair_correlation(g: np.ndarray) -> np.ndarray:
    """<D_i^+ D_j + D_j D_i^+> for all i, j (element [i, j])."""
    n = g.shape[0]
    gt = g.T                       # gt[i, j] = G_ji
    d = np.eye(n) - gt
    return d * d + gt * gt


def s_pair(g: np.ndarray, L: int, m) -> complex:
    """S_Pair(Q) of one configuration (Sec. IV, symmetric definition)."""
    n = g.shape[0]
    p = phases(site_coords(L), L, m)
    c = pair_correlation(g)
    total = 0.0 + 0.0j
    for i in range(n):
        total += p[i] * np.sum(c[i, :] * np.conj(p))
    return total / n


def density_correlation(g: np.ndarray) -> np.ndarray:
    """<n_a n_b> (both spins) for all a, b."""
    n = g.shape[0]
    occ = 1.0 - np.diag(g)
    return 4.0 * np.outer(occ, occ) + 2.0 * (np.eye(n) - g.T) * g


def cdw_d2(g: np.ndarray, L: int, m) -> complex:
    """<phi^+(Q) phi(Q)> of one configuration (Sec. V)."""
    n = g.shape[0]
    w = np.tile(np.array([1.0, OMEGA, OMEGA ** 2]), L * L)
    coef = phases(cell_coords(L), L, m) * w          # phi = (1/N) sum_a coef_a n_a
    nn = density_correlation(g)
    return np.sum(np.conj(coef)[:, None] * coef[None, :] * nn) / n ** 2


def density(g: np.ndarray) -> float:
    """Particles per site, both spins: (2/N) sum_a (1 - G_aa)."""
    return float(2.0 * np.mean(1.0 - np.diag(g)))


DK1, DK2 = (1, 0), (0, 1)


def k_point(L: int):
    return (L // 3, (2 * L) // 3)


def estimators(g: np.ndarray, L: int) -> dict:
    """The per-configuration values the GPU path returns (real parts)."""
    return {"s_pair_gamma": s_pair(g, L, (0, 0)).real,
            "s_pair_dk1": s_pair(g, L, DK1).real,
            "s_pair_dk2": s_pair(g, L, DK2).real,
            "cdw2_gamma": cdw_d2(g, L, (0, 0)).real,
            "cdw2_k": cdw_d2(g, L, k_point(L)).real,
            "density": density(g)}
