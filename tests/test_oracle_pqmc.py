"""Pins of the oracle's projector (PQMC) module (Sec. II: trial wave function
of the lowest N_occ eigenstates, filling rho = 2 N_occ / N; projection over
beta): the trial orbitals against the Bloch-block spectrum of Eq. (4), the
free-fermion projector G against a closed form assembled per momentum, the
stabilized G and the flip ratio against multiprecision brute force, and the
update/wrap consistency of a pass."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import brute, dqmc, lattice, pqmc


def _model(L, U, beta):
    return dqmc.Model(L=L, t=1.0, U=U, beta=beta, dtau=0.1, mu=-1.0)


@pytest.fixture(scope="module")
def small():
    """L=3, U=-4, beta=1 (10 slices), Dirac filling n_occ = L^2 = 9."""
    m = _model(3, -4.0, 1.0)
    f = si.ising_fields(3, m.L_tau, 33)
    p, _ = pqmc.trial_orbitals(3, 9)
    return m, f, p


def _bloch_trial_levels(L, eps):
    """Levels of K_T from the 3x3 blocks of Eq. (4) plus the sublattice
    potential (translation invariant, so it adds diag(eps, 0, -eps) to every
    block)."""
    h = lattice.bloch_blocks(L, 1.0)
    d = np.diag([eps, 0.0, -eps])
    return np.sort(np.concatenate([np.linalg.eigvalsh(h[a, b] + d) for a in range(L) for b in range(L)]))


@pytest.mark.parametrize("L", [3, 6])
def test_trial_orbitals(L):
    n = L * L
    p, w = pqmc.trial_orbitals(L, n)
    kt = pqmc.trial_K(L)
    assert np.abs(p.T @ p - np.eye(n)).max() < 1e-13
    assert np.abs(kt @ p - p * w[:n][None, :]).max() < 1e-12
    # the dense levels are the Bloch levels (an independent route, Eq. (4))
    assert np.abs(w - _bloch_trial_levels(L, pqmc.TRIAL_EPS)).max() < 1e-12
    # the potential splits the Dirac points by 2 eps / sqrt(3) to first order
    gap = w[n] - w[n - 1]
    assert abs(gap / (2 * pqmc.TRIAL_EPS / np.sqrt(3)) - 1) < 0.01
    # without it the shell is open at the Dirac filling (3 | L)
    with pytest.raises(ValueError):
        pqmc.trial_orbitals(L, n, eps=0.0)


@pytest.mark.parametrize("L,beta,l", [(3, 2.0, 7), (6, 3.0, 0), (6, 3.0, 30)])
def test_free_projector_green_closed_form(L, beta, l):
    """U = 0: every B_l = exp(-dtau (K - mu)), and per momentum
    G_k = I - e^{-l dtau H_k} V_k (V_k^+ e^{-beta H_k} V_k)^{-1} V_k^+ e^{-(beta - l dtau) H_k}
    with V_k the occupied trial vectors of H_k + diag(eps, 0, -eps)
    (mu cancels); assembled through the unitary momentum transform of Eq. (2)."""
    m = _model(L, 0.0, beta)
    assert m.alpha == 0.0
    n = L * L
    p, w = pqmc.trial_orbitals(L, n)
    f = si.ising_fields(L, m.L_tau, 5)
    g = pqmc.green(m, f, p, l)
    h = lattice.bloch_blocks(L, 1.0)
    d = np.diag([pqmc.TRIAL_EPS, 0.0, -pqmc.TRIAL_EPS])
    # occupied (k, band) pairs: the lowest n levels of all blocks of K_T
    lev = []
    for a in range(L):
        for b in range(L):
            ew, ev = np.linalg.eigh(h[a, b] + d)
            for j in range(3):
                lev.append((ew[j], a, b, ev[:, j]))
    lev.sort(key=lambda x: x[0])
    occ = {}
    for e, a, b, v in lev[:n]:
        occ.setdefault((a, b), []).append(v)
    tau = l * m.dtau
    blocks = np.zeros((L, L, 3, 3), dtype=complex)
    for a in range(L):
        for b in range(L):
            ew, ev = np.linalg.eigh(h[a, b])
            ex = lambda s: (ev * np.exp(-s * ew)) @ ev.conj().T  # noqa: E731
            if (a, b) not in occ:
                blocks[a, b] = np.eye(3)
                continue
            v = np.array(occ[(a, b)]).T
            blocks[a, b] = np.eye(3) - ex(tau) @ v @ np.linalg.solve(
                v.conj().T @ ex(beta) @ v, v.conj().T @ ex(beta - tau))
    ft = lattice.momentum_transform(L)
    lam = np.zeros((m.N, m.N), dtype=complex)
    for a in range(L):
        for b in range(L):
            c = (a * L + b) * 3
            lam[c:c + 3, c:c + 3] = blocks[a, b]
    gk = ft @ lam @ ft.conj().T
    assert np.abs(gk.imag).max() < 1e-12
    assert np.abs(g - gk.real).max() < 1e-12


def test_projector_green_vs_multiprecision(small):
    m, f, p = small
    e = brute.mp_propagator(m, dps=40)
    for l in (0, 4, 10):
        g = pqmc.green(m, f, p, l)
        gm = brute.mp_pqmc_green(m, f, p, l, dps=40, e=e)
        assert np.abs(g - gm).max() < 1e-12, l


def test_projector_flip_ratio_vs_determinants(small):
    """The rank-one ratio from G~ = e^{V_l} G(l-1) e^{-V_l} equals the ratio of
    the weights prod e^{-alpha s} det(P^T B_{L_tau} ... B_1 P)^2."""
    m, f, p = small
    e = brute.mp_propagator(m, dps=30)
    lw0 = brute.mp_pqmc_log_weight(m, f, p, dps=30, e=e)
    for (l, i) in [(1, 0), (4, 13), (10, 26)]:
        g_prev = pqmc.green(m, f, p, l - 1)
        ev = np.exp(m.alpha * f[l - 1])
        gt = ev[:, None] * g_prev / ev[None, :]
        ratio, _, _ = dqmc.flip_ratio(m.alpha, int(f[l - 1, i]), gt[i, i])
        f2 = f.copy()
        f2[l - 1, i] *= -1
        rb = float(brute.mp.exp(brute.mp_pqmc_log_weight(m, f2, p, dps=30, e=e) - lw0))
        assert abs(ratio / rb - 1) < 1e-11, (l, i, ratio, rb)


def test_projector_wrap_relation(small):
    m, f, p = small
    for l in (1, 6, 10):
        g_prev = pqmc.green(m, f, p, l - 1)
        assert np.abs(dqmc.wrap(m, g_prev, f[l - 1]) - pqmc.green(m, f, p, l)).max() < 1e-12


def test_projector_not_cyclic(small):
    """Unlike the finite-temperature G, G(L_tau) differs from G(0)."""
    m, f, p = small
    assert np.abs(pqmc.green(m, f, p, 0) - pqmc.green(m, f, p, m.L_tau)).max() > 1e-3


@pytest.mark.parametrize("k", [1, 4])
def test_projector_pass_consistency(small, k):
    """An upward Metropolis pass (delay k): decisions follow the rule, every
    slice's G is the fresh projector G of the fields so far, delayed equals
    undelayed; the downward pass from its end returns to the fresh G(0)."""
    m, f, p = small
    u = si.metropolis_uniforms(3, m.L_tau, 7, n_sweeps=2)
    r = pqmc.sweep(m, f, p, pqmc.green(m, f, p, 0), uniforms=u[0], k=k, n_stab=5)
    assert np.array_equal(r["fields"] != f, r["accepted"])
    assert np.array_equal(u[0] < r["ratios"], r["accepted"])
    assert r["accepted"].any()
    for l, g in enumerate(r["G_slices"], start=1):
        f_at = np.concatenate([r["fields"][:l], f[l:]])
        assert np.abs(g - pqmc.green(m, f_at, p, l)).max() < 1e-10, l
    r1 = pqmc.sweep(m, f, p, pqmc.green(m, f, p, 0), uniforms=u[0], k=1, n_stab=5)
    assert np.array_equal(r1["accepted"], r["accepted"])
    rd = pqmc.sweep_down(m, r["fields"], p, r["G"], uniforms=u[1], k=k, n_stab=5)
    assert np.abs(rd["G"] - pqmc.green(m, rd["fields"], p, 0)).max() < 1e-12
    assert np.array_equal(u[1] < rd["ratios"], rd["accepted"])
