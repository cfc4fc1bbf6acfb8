"""Planted mistakes in the oracle (CPU only): each plausible slip must make at
least one pin fail, so the pins are not tautologies of the oracle's code."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import dqmc, lattice
import test_oracle_dqmc as tdq
import test_oracle_lattice as tla


def _c1():
    w = si.C1
    m = dqmc.Model.from_workload(w)
    return w, m, si.ising_fields(w.L, m.L_tau, w.seed)


def test_transposed_shift_is_caught(monkeypatch):
    orig = lattice.shift_matrix
    monkeypatch.setattr(lattice, "shift_matrix", lambda L: orig(L).T.copy())
    with pytest.raises(AssertionError):
        tla.test_K_neighbour_lists(4)


def test_wrong_intracell_entry_is_caught(monkeypatch):
    orig = lattice.intracell_deltas

    def bad():
        da, db, dc = orig()
        return da, db, dc.T.copy()
    monkeypatch.setattr(lattice, "intracell_deltas", bad)
    with pytest.raises(AssertionError):
        tla.test_K_neighbour_lists(5)


def test_missing_kron_term_is_caught(monkeypatch):
    def bad(L, t=1.0):
        eye = np.eye(L)
        ks = lattice.shift_matrix(L)
        da, db, dc = lattice.intracell_deltas()
        m = (np.kron(np.kron(eye, eye + ks), da) + np.kron(np.kron(eye + ks, eye), db)
             + np.kron(np.kron(eye, eye), dc))
        return -t * (m + m.T)
    monkeypatch.setattr(lattice, "kagome_K", bad)
    with pytest.raises(AssertionError):
        tla.test_K_spectrum_closed_form(6)


def test_wrong_alpha_is_caught(monkeypatch):
    monkeypatch.setattr(dqmc, "hs_alpha", lambda U, dtau: float(np.arccosh(np.exp(dtau * abs(U)))))
    with pytest.raises(AssertionError):
        tdq.test_hs_decoupling_identity(-4.0)


def test_wrong_delta_sign_is_caught(monkeypatch):
    monkeypatch.setattr(dqmc, "flip_delta", lambda a, s: float(np.exp(2.0 * a * s) - 1.0))
    with pytest.raises(AssertionError):
        tdq.test_flip_ratio_vs_determinants(_c1())


def test_missing_sign_factor_in_ratio_is_caught(monkeypatch):
    def bad(alpha, s, g_ii):
        delta = dqmc.flip_delta(alpha, s)
        r = 1.0 + delta * (1.0 - g_ii)
        return r * r, r, delta
    monkeypatch.setattr(dqmc, "flip_ratio", bad)
    with pytest.raises(AssertionError):
        tdq.test_flip_ratio_vs_determinants(_c1())


def test_wrap_sides_swapped_is_caught(monkeypatch):
    def bad(model, g, s_l):
        ev = np.exp(model.alpha * s_l.astype(float))
        gt = ev[:, None] * g / ev[None, :]
        return model.EKinv @ gt @ model.EK
    monkeypatch.setattr(dqmc, "wrap", bad)
    with pytest.raises(AssertionError):
        tdq.test_wrap_relation(_c1())


def test_dropped_small_scales_is_caught(monkeypatch):
    def bad(u, d, t):
        db = np.maximum(d, 1.0)
        rhs = u.T / db[:, None]
        return np.linalg.solve(rhs + t, rhs)
    monkeypatch.setattr(dqmc, "green_from_udt", bad)
    with pytest.raises(AssertionError):
        tdq.test_green_scratch_vs_multiprecision(_c1())


def test_wrong_chain_order_is_caught(monkeypatch):
    monkeypatch.setattr(dqmc, "chain_order", lambda l, Lt: list(range(1, Lt + 1)))
    with pytest.raises(AssertionError):
        tdq.test_wrap_relation(_c1())


def test_wrong_update_row_is_caught(monkeypatch):
    orig = dqmc.update_slice

    def bad(gt, s, alpha, u=None, forced=None, k=1):
        gt = gt.T.copy()   # rows and columns exchanged in the rank-one factor
        g, a, r = orig(gt, s, alpha, u, forced, k)
        return g.T.copy(), a, r
    monkeypatch.setattr(dqmc, "update_slice", bad)
    with pytest.raises(AssertionError):
        tdq.test_rank_one_update_then_wrap_equals_scratch(_c1())


def test_down_pass_old_field_scaling_is_caught(monkeypatch):
    """Downward pass that scales back with the fields from before the flips."""
    def bad(model, fields, g_top, uniforms=None, forced=None, k=1, n_stab=10, record=True,
            l_stop=None, l_start=None):
        fields = fields.copy()
        L_tau, n = fields.shape
        acc = np.zeros((L_tau, n), dtype=bool)
        g = g_top.copy()
        top = L_tau if l_start is None else l_start
        for l in range(top, (1 if l_stop is None else l_stop) - 1, -1):
            s = fields[l - 1]
            ev = np.exp(model.alpha * s.astype(float))   # taken before the flips
            gt = model.EKinv @ g @ model.EK
            gt, acc[l - 1], _ = dqmc.update_slice(gt, s, model.alpha,
                                                  None if uniforms is None else uniforms[l - 1],
                                                  None if forced is None else forced[l - 1], k)
            g = gt / ev[:, None] * ev[None, :]
        return dict(fields=fields, G=g, accepted=acc)
    monkeypatch.setattr(dqmc, "sweep_down", bad)
    with pytest.raises(AssertionError):
        tdq.test_down_slice_update_equals_scratch(_c1())


# ---- projector (PQMC) pieces -------------------------------------------------
import test_oracle_pqmc as tpq  # noqa: E402
from oracle import pqmc  # noqa: E402


def _pq_small():
    m = dqmc.Model(L=3, t=1.0, U=-4.0, beta=1.0, dtau=0.1, mu=-1.0)
    f = si.ising_fields(3, m.L_tau, 33)
    p, _ = pqmc.trial_orbitals(3, 9)
    return m, f, p


def test_pqmc_left_chain_untransposed_is_caught(monkeypatch):
    """Left panel built from B instead of B^T."""
    def bad(model, fields, p, l):
        x = p.copy()
        for j in range(fields.shape[0], l, -1):
            x = pqmc._orth(dqmc.b_matrix(model, fields[j - 1]) @ x)
        return x
    monkeypatch.setattr(pqmc, "left_panel", bad)
    with pytest.raises(AssertionError):
        tpq.test_projector_green_vs_multiprecision(_pq_small())


def test_pqmc_right_chain_short_is_caught(monkeypatch):
    """Right panel missing the last B."""
    def bad(model, fields, p, l):
        r = p.copy()
        for j in range(1, l):
            r = pqmc._orth(dqmc.b_matrix(model, fields[j - 1]) @ r)
        return r
    monkeypatch.setattr(pqmc, "right_panel", bad)
    with pytest.raises(AssertionError):
        tpq.test_projector_wrap_relation(_pq_small())


def test_pqmc_highest_orbitals_is_caught(monkeypatch):
    """Trial orbitals taken from the top of the spectrum."""
    def bad(L, n_occ, t=1.0, eps=pqmc.TRIAL_EPS):
        w, v = np.linalg.eigh(pqmc.trial_K(L, t, eps))
        return v[:, -n_occ:].copy(), w
    monkeypatch.setattr(pqmc, "trial_orbitals", bad)
    with pytest.raises(AssertionError):
        tpq.test_free_projector_green_closed_form(3, 2.0, 7)


# ---- equal-time estimators -----------------------------------------------------
import test_oracle_measure as tms  # noqa: E402
from oracle import measure  # noqa: E402


def _gaussian():
    return tms.gaussian.__wrapped__()


def test_pair_correlation_untransposed_is_caught(monkeypatch):
    def bad(g):
        n = g.shape[0]
        d = np.eye(n) - g
        return d * d + g * g
    monkeypatch.setattr(measure, "pair_correlation", bad)
    with pytest.raises(AssertionError):
        tms.test_pair_correlation_wick(_gaussian())


def test_density_exchange_term_untransposed_is_caught(monkeypatch):
    def bad(g):
        n = g.shape[0]
        occ = 1.0 - np.diag(g)
        return 4.0 * np.outer(occ, occ) + 2.0 * (np.eye(n) - g) * g
    monkeypatch.setattr(measure, "density_correlation", bad)
    with pytest.raises(AssertionError):
        tms.test_density_correlation_wick(_gaussian())


def test_swapped_sublattice_offsets_are_caught(monkeypatch):
    monkeypatch.setattr(measure, "SUB_OFFSET", np.array([[0.0, 0.0], [-0.5, 0.0], [0.0, -0.5]]))
    with pytest.raises(AssertionError):
        tms.test_geometry_bonds(3)
