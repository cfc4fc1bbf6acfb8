"""Pins of the oracle's lattice module against facts fixed by the paper and
by mathematics (Eqs. (1)-(4), (6); textbook kagome dispersion)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import lattice


def site(L, x1, x2, s):
    return ((x1 % L) * L + (x2 % L)) * 3 + s


@pytest.mark.parametrize("L", [3, 4, 5, 6, 12])
def test_K_symmetric_four_regular(L):
    K = lattice.kagome_K(L, t=1.3)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 0)
    nz = K != 0
    assert np.all(nz.sum(axis=1) == 4)          # kagome coordination number
    assert np.all(K[nz] == -1.3)                 # K_ij = -t on bonds, Eq. (1)


@pytest.mark.parametrize("L", [4, 5, 6])
def test_K_neighbour_lists(L):
    """Neighbours read by hand off the Kronecker terms of Eq. (3):
    A-B bonds along x2, A-C bonds along x1, B-C bonds along (x1+1, x2-1)."""
    K = lattice.kagome_K(L)
    A, B, C = 0, 1, 2
    for x1 in range(L):
        for x2 in range(L):
            want = {
                A: {site(L, x1, x2, B), site(L, x1, x2 + 1, B), site(L, x1, x2, C), site(L, x1 + 1, x2, C)},
                B: {site(L, x1, x2, A), site(L, x1, x2 - 1, A), site(L, x1, x2, C), site(L, x1 + 1, x2 - 1, C)},
                C: {site(L, x1, x2, A), site(L, x1 - 1, x2, A), site(L, x1, x2, B), site(L, x1 - 1, x2 + 1, B)},
            }
            for s in (A, B, C):
                got = set(np.nonzero(K[site(L, x1, x2, s)])[0])
                assert got == want[s], (x1, x2, s)


@pytest.mark.parametrize("L", [3, 4, 5, 6, 12])
def test_K_spectrum_closed_form(L):
    e = np.sort(np.linalg.eigvalsh(lattice.kagome_K(L, t=0.7)))
    assert np.abs(e - lattice.kagome_band_energies(L, t=0.7)).max() < 1e-13


@pytest.mark.parametrize("L", [3, 4, 6])
def test_eq2_block_diagonal(L):
    ft = lattice.momentum_transform(L)
    lam = ft.conj().T @ lattice.kagome_K(L) @ ft
    mask = np.kron(np.eye(L * L), np.ones((3, 3))).astype(bool)
    assert np.abs(lam[~mask]).max() < 1e-13


@pytest.mark.parametrize("L", [3, 4, 6])
def test_eq4_reconstructs_K(L):
    ft = lattice.momentum_transform(L)
    k = ft @ lattice.block_form_eq4(L) @ ft.conj().T
    assert np.abs(k - lattice.kagome_K(L)).max() < 1e-13


@pytest.mark.parametrize("L", [3, 6])
def test_bloch_block_eigenvalues_per_k(L):
    h = lattice.bloch_blocks(L, t=1.0)
    for m1 in range(L):
        for m2 in range(L):
            k1, k2 = 2 * np.pi * m1 / L, 2 * np.pi * m2 / L
            r = np.sqrt(max(0.0, 3 + 2 * np.cos(k1) + 2 * np.cos(k2) + 2 * np.cos(k1 - k2)))
            want = np.sort([2.0, -(1 + r), -(1 - r)])
            got = np.linalg.eigvalsh(h[m1, m2])
            assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("L", [3, 6, 9])
def test_eq6_three_step_product_equals_dense_expm(L):
    """Eq. (6): FFT -> 3x3 block multiply -> inverse FFT equals exp(-dtau K) M."""
    dtau = 0.1
    K = lattice.kagome_K(L)
    m = np.random.default_rng(L).standard_normal((3 * L * L, 7))
    dense = scipy.linalg.expm(-dtau * K) @ m
    fast = lattice.apply_block_operator(L, lattice.expm_blocks(L, 1.0, -dtau), m)
    assert np.abs(fast.imag).max() < 1e-13
    assert np.abs(fast.real - dense).max() < 1e-13


def test_expm_crosscheck():
    from oracle import dqmc
    K = lattice.kagome_K(6)
    a = -0.1 * (K + 0.3 * np.eye(K.shape[0]))
    assert np.abs(scipy.linalg.expm(a) - dqmc.expm_eigh(a)).max() < 1e-14


@pytest.mark.parametrize("L", [3, 6, 9, 12])
def test_dirac_mu_is_minus_t_when_3_divides_L(L):
    assert abs(lattice.dirac_mu(L, t=1.0) + 1.0) < 1e-12
    assert abs(lattice.dirac_mu(L, t=2.0) + 2.0) < 1e-12


def test_dirac_filling_two_thirds():
    """Occupying every level below mu fills N/3 states per spin (rho = 2/3)."""
    L = 12
    e = np.linalg.eigvalsh(lattice.kagome_K(L))
    mu = lattice.dirac_mu(L)
    assert (e < mu - 1e-9).sum() + 0.5 * (np.abs(e - mu) < 1e-9).sum() == L * L


@pytest.mark.parametrize("L", [3, 4, 6])
def test_triangular_K(L):
    """App. A1: symmetric, 6-regular (L >= 3), K_ij = -t, spectrum = the
    closed-form triangular dispersion."""
    k = lattice.triangular_K(L, 1.0)
    assert np.array_equal(k, k.T)
    assert np.all((k == 0) | (k == -1.0))
    assert np.all((k != 0).sum(axis=1) == 6)
    assert np.abs(np.sort(np.linalg.eigvalsh(k)) - lattice.triangular_band_energies(L)).max() < 1e-12


@pytest.mark.parametrize("L", [3, 4, 6])
def test_honeycomb_K(L):
    """App. A2: symmetric, 3-regular, bipartite (no A-A or B-B bonds),
    spectrum = +-t |1 + e^{ik1} + e^{ik2}|."""
    k = lattice.honeycomb_K(L, 1.0)
    assert np.array_equal(k, k.T)
    assert np.all((k != 0).sum(axis=1) == 3)
    assert np.all(k[0::2, 0::2] == 0) and np.all(k[1::2, 1::2] == 0)
    assert np.abs(np.sort(np.linalg.eigvalsh(k)) - lattice.honeycomb_band_energies(L)).max() < 1e-12
