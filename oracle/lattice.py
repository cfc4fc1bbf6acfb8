"""Kagome kinetic matrix and its momentum-space block form (oracle, FP64).

Test infrastructure only (see ``oracle/__init__.py``).

Site order: the Kronecker order of Eq. (3), i.e. the first factor acts on the
slow cell coordinate x1, the second on x2, the third on the sublattice s, so
site index ``i = (x1*L + x2)*3 + s`` with s = 0, 1, 2 for A, B, C.
"""
from __future__ import annotations

import numpy as np


def shift_matrix(L: int) -> np.ndarray:
    """The L x L circulant one-step translation K_s of Eq. (3).

    Sec. II (text after Eq. (3)): non-zero entries only on the first
    subdiagonal and the top-right corner.  0-based: (K_s)[x+1, x] = 1 for
    x < L-1 and (K_s)[0, L-1] = 1.
    """
    ks = np.zeros((L, L))
    for x in range(L - 1):
        ks[x + 1, x] = 1.0
    ks[0, L - 1] = 1.0
    return ks


def intracell_deltas():
    """The 3x3 intra-cell matrices delta_a, delta_b, delta_c of Eq. (3).

    Each has a single unit entry at (2,1), (3,1), (3,2) respectively (1-based
    in the paper; 0-based (1,0), (2,0), (2,1) here).
    """
    da = np.zeros((3, 3)); da[1, 0] = 1.0
    db = np.zeros((3, 3)); db[2, 0] = 1.0
    dc = np.zeros((3, 3)); dc[2, 1] = 1.0
    return da, db, dc


def kagome_K(L: int, t: float = 1.0) -> np.ndarray:
    """Dense N x N kinetic matrix, N = 3 L^2.

    Eq. (3) gives the unit-hopping pattern as a Kronecker sum plus its
    Hermitian conjugate; Eq. (1) fixes K_ij = -t on nearest-neighbour bonds,
    so K = -t * (Eq. (3) matrix).
    """
    eye = np.eye(L)
    ks = shift_matrix(L)
    da, db, dc = intracell_deltas()
    m = (np.kron(np.kron(eye, eye + ks), da)
         + np.kron(np.kron(eye + ks, eye), db)
         + np.kron(np.kron(eye, eye) + np.kron(ks, ks.T), dc))
    return -t * (m + m.T.conj())


def triangular_K(L: int, t: float = 1.0) -> np.ndarray:
    """Dense L^2 x L^2 kinetic matrix of the triangular lattice (App. A1):
    the Kronecker sum I (x) K_s + K_s (x) I + K_s (x) K_s plus its Hermitian
    conjugate, scaled by -t (Eq. (1)).  One site per cell, i = x1 L + x2."""
    eye = np.eye(L)
    ks = shift_matrix(L)
    m = np.kron(eye, ks) + np.kron(ks, eye) + np.kron(ks, ks)
    return -t * (m + m.T.conj())


def honeycomb_K(L: int, t: float = 1.0) -> np.ndarray:
    """Dense 2L^2 x 2L^2 kinetic matrix of the honeycomb lattice (App. A2):
    (I (x) I + I (x) K_s + K_s (x) I) (x) delta plus its Hermitian conjugate,
    delta the 2 x 2 matrix with one unit entry at (2, 1) (1-based); scaled by
    -t.  Site i = (x1 L + x2) 2 + s, s = 0, 1 for the two sublattices."""
    eye = np.eye(L)
    ks = shift_matrix(L)
    d = np.zeros((2, 2))
    d[1, 0] = 1.0
    m = np.kron(np.kron(eye, eye) + np.kron(eye, ks) + np.kron(ks, eye), d)
    return -t * (m + m.T.conj())


LATTICES = {"kagome": (3, kagome_K), "triangular": (1, triangular_K), "honeycomb": (2, honeycomb_K)}


def lattice_K(name: str, L: int, t: float = 1.0) -> np.ndarray:
    """K of a lattice by name (kagome, triangular, honeycomb)."""
    return LATTICES[name][1](L, t)


def triangular_band_energies(L: int, t: float = 1.0) -> np.ndarray:
    """Closed form: -2t (cos k1 + cos k2 + cos(k1 + k2)) on the L x L grid (sorted)."""
    e = []
    for m1 in range(L):
        for m2 in range(L):
            k1, k2 = 2 * np.pi * m1 / L, 2 * np.pi * m2 / L
            e.append(-2 * t * (np.cos(k1) + np.cos(k2) + np.cos(k1 + k2)))
    return np.sort(np.array(e))


def honeycomb_band_energies(L: int, t: float = 1.0) -> np.ndarray:
    """Closed form: +-t |1 + e^{i k1} + e^{i k2}| on the L x L grid (sorted)."""
    e = []
    for m1 in range(L):
        for m2 in range(L):
            k1, k2 = 2 * np.pi * m1 / L, 2 * np.pi * m2 / L
            r = abs(1 + np.exp(1j * k1) + np.exp(1j * k2))
            e.extend([t * r, -t * r])
    return np.sort(np.array(e))


def dft_matrix(L: int) -> np.ndarray:
    """Unitary one-dimensional DFT matrix F, F[m, x] = exp(-2 pi i m x / L) / sqrt(L).

    The paper does not fix the sign or the normalisation of F.  Eq. (2) is a
    similarity transform only when F is unitary, hence the 1/sqrt(L).
    """
    m = np.arange(L)
    return np.exp(-2j * np.pi * np.outer(m, m) / L) / np.sqrt(L)


def momentum_transform(L: int) -> np.ndarray:
    """The N x N unitary F (x) F (x) I_3 of Eqs. (2) and (4)."""
    f = dft_matrix(L)
    return np.kron(np.kron(f, f), np.eye(3))


def block_form_eq4(L: int, t: float = 1.0) -> np.ndarray:
    """Lambda_kag of Eq. (4): the dense N x N matrix made of L^2 3x3 blocks.

    Built from the bracket of Eq. (4) with Lambda_s = F^dagger K_s F (the
    reading under which Eq. (2) and Eq. (4) agree; the sentence after Eq. (3)
    writes the transform the other way round, which diagonalises K_s just as
    well but would swap F and F^dagger in Eq. (4)).
    """
    f = dft_matrix(L)
    lam_s = f.conj().T @ shift_matrix(L) @ f
    lam_s = np.diag(np.diag(lam_s))
    eye = np.eye(L)
    da, db, dc = intracell_deltas()
    m = (np.kron(np.kron(eye, eye + lam_s), da)
         + np.kron(np.kron(eye + lam_s, eye), db)
         + np.kron(np.kron(eye, eye) + np.kron(lam_s, lam_s.conj()), dc))
    return -t * (m + m.T.conj())


def bloch_blocks(L: int, t: float = 1.0) -> np.ndarray:
    """The L^2 independent 3x3 blocks of Eq. (2), shape (L, L, 3, 3).

    Extracted from (F^dagger (x) F^dagger (x) I) K (F (x) F (x) I); block
    (m1, m2) belongs to momentum k = 2 pi (m1, m2) / L.
    """
    ft = momentum_transform(L)
    lam = ft.conj().T @ kagome_K(L, t) @ ft
    out = np.empty((L, L, 3, 3), dtype=complex)
    for m1 in range(L):
        for m2 in range(L):
            c = (m1 * L + m2) * 3
            out[m1, m2] = lam[c:c + 3, c:c + 3]
    return out


def kagome_band_energies(L: int, t: float = 1.0) -> np.ndarray:
    """Closed-form kagome spectrum on the L x L momentum grid (sorted).

    The textbook nearest-neighbour kagome dispersion: a flat band at +2t and
    two dispersive bands -t(1 +- sqrt(3 + 2cos k1 + 2cos k2 + 2cos(k1-k2))),
    with k_j = 2 pi m_j / L.  Used as an independent pin of kagome_K.
    """
    e = []
    for m1 in range(L):
        for m2 in range(L):
            k1 = 2 * np.pi * m1 / L
            k2 = 2 * np.pi * m2 / L
            r = np.sqrt(max(0.0, 3 + 2 * np.cos(k1) + 2 * np.cos(k2) + 2 * np.cos(k1 - k2)))
            e.extend([2 * t, -t * (1 + r), -t * (1 - r)])
    return np.sort(np.array(e))


def dirac_mu(L: int, t: float = 1.0) -> float:
    """Chemical potential at the Dirac energy, read from the spectrum of K.

    Dirac filling rho = 2/3 (Sec. IV) means the lowest L^2 of the N = 3L^2
    single-particle levels are occupied per spin (N_occ = N/3, Sec. II); the
    chemical potential is taken midway between level L^2 and level L^2 + 1.
    When 3 | L the Dirac point is on the momentum grid and both levels equal
    the Dirac energy -t.
    """
    e = np.sort(np.linalg.eigvalsh(kagome_K(L, t)))
    n = L * L
    return 0.5 * (e[n - 1] + e[n])


def _block_function(L: int, t: float, fn) -> np.ndarray:
    """Apply fn to every 3x3 Bloch block (Hermitian), returns shape (L, L, 3, 3)."""
    h = bloch_blocks(L, t)
    out = np.empty_like(h)
    for m1 in range(L):
        for m2 in range(L):
            w, v = np.linalg.eigh(h[m1, m2])
            out[m1, m2] = (v * fn(w)) @ v.conj().T
    return out


def apply_block_operator(L: int, blocks: np.ndarray, m: np.ndarray) -> np.ndarray:
    """The three steps of Eq. (6) applied to every column of M.

    (1) transform each sublattice component with (F^dagger (x) F^dagger),
    (2) multiply by the 3x3 block of momentum k, (3) transform back with
    (F (x) F).  The unitary F of ``dft_matrix`` makes F^dagger the
    unnormalised inverse DFT / L and F the forward DFT / L per axis.
    """
    n = 3 * L * L
    cols = m.reshape(L, L, 3, -1)
    # F^dagger (x) F^dagger on the cell indices: numpy's ifft2 is
    # (1/L^2) sum_x exp(+2 pi i k x / L); F^dagger v = sqrt(L) ifft per axis.
    vk = np.fft.ifft2(cols, axes=(0, 1)) * L
    vk = np.einsum('abst,abtc->absc', blocks, vk)
    out = np.fft.fft2(vk, axes=(0, 1)) / L
    return out.reshape(n, -1)


def expm_blocks(L: int, t: float, scale: float, mu: float = 0.0) -> np.ndarray:
    """exp(scale * (H(k) - mu)) for every Bloch block."""
    return _block_function(L, t, lambda w: np.exp(scale * (w - mu)))


def free_green_blocks(L: int, t: float, beta: float, mu: float) -> np.ndarray:
    """(I + exp(-beta (H(k) - mu)))^{-1} for every Bloch block."""
    return _block_function(L, t, lambda w: 1.0 / (1.0 + np.exp(-beta * (w - mu))))
