"""Plain FP64 CPU oracle for the kagome attractive-Hubbard DQMC hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU path
(``paper_2608_03894_amd``) never imports, links or calls anything here, and
nothing here imports the GPU path: the two share only the seeded input
generators in ``seeded_inputs.py``.

What it computes, following the paper (Zhang, Li, Wang, "Accelerated quantum
Monte Carlo simulations of the attractive Hubbard model on the kagome
lattice"):

* ``lattice``: the kinetic matrix K of Eq. (1)/(3) built from the Kronecker
  sum of Eq. (3) (scaled by -t, the hopping of Eq. (1)), the unitary DFT
  matrix F, and the momentum-space blocks of Eq. (2)/(4).  The block form is
  used by the pins only; the oracle's propagators are dense.
* ``dqmc``: dense propagators expm(-dtau (K - mu)) (the product of Eq. (5)),
  the discrete charge-channel Ising decoupling, single-flip ratios,
  Sherman-Morrison and delayed rank-k Green's-function updates (the
  delay-update algorithm cited in Sec. II), column-pivoted QR (UDT)
  stabilized equal-time Green's functions, and one Metropolis sweep.

Every function is FP64.  Where the paper is silent (decoupling, ensemble,
stabilization, visiting order) the reading adopted is stated in the
function's docstring.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against a
closed form, a brute-force determinant, a textbook identity or an exact
algebraic relation.  The physics observables of Secs. IV-V are not part of
the oracle (parity unpinned there; not built).
"""
