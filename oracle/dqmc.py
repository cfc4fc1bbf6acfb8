"""Finite-temperature DQMC for the attractive kagome Hubbard model (oracle, FP64).

Test infrastructure only (see ``oracle/__init__.py``).

Readings adopted where the paper is silent (each one is listed with its
reason in the design notes):

* Ensemble: grand canonical at inverse temperature beta with L_tau = beta/dtau
  slices (the paper's runs are projector QMC; the propagator product of
  Eq. (5) and the update are the same in both).
* Decoupling: the interaction U (n_up - 1/2)(n_dn - 1/2), U < 0, is written
  with a discrete charge-channel Ising field s = +-1 per site and slice,
  exp(-dtau U (n_up-1/2)(n_dn-1/2)) = (1/2) exp(-dtau|U|/4)
  sum_s exp(alpha s (n_up + n_dn - 1)), cosh(alpha) = exp(dtau |U| / 2).
  V_l = diag(alpha s_l) acts identically on both spins, so G_up = G_dn = G.
* Propagator: B_l = exp(-dtau (K - mu)) exp(V_l) (kinetic factor of Eq. (5)
  to the left of the field factor).
* Equal-time Green's function:
  G(l) = [I + B_l ... B_1 B_{L_tau} ... B_{l+1}]^{-1}, G(0) = G(L_tau).
* Update of slice l: G~ = exp(V_l) G(l-1) exp(-V_l); sites i = 0..N-1 are
  visited in order; a flip s -> -s is accepted (Metropolis) iff
  u < exp(2 alpha s) R^2 with R = 1 + Delta (1 - G~_ii),
  Delta = exp(-2 alpha s) - 1; then G(l) = exp(-dtau K) G~ exp(+dtau K).
* Delay: k counts accepted flips; the accumulated rank-k factors are added to
  G~ when k have been accepted and at the end of the slice (the delay-update
  algorithm cited in Sec. II).  k = 1 is plain Sherman-Morrison.
* Stabilization: every n_stab slices G is replaced by the QR-stabilized
  G(l) (column-pivoted Householder QR after every B, Loh-Gubernatis scale
  separation for the final inverse) and the largest |difference| is logged.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import lattice


def hs_alpha(U: float, dtau: float) -> float:
    """Ising coupling alpha with cosh(alpha) = exp(dtau |U| / 2)."""
    return float(np.arccosh(np.exp(dtau * abs(U) / 2.0)))


@dataclasses.dataclass
class Model:
    """Kagome lattice plus the Hubbard and discretisation parameters."""

    L: int
    t: float
    U: float
    beta: float
    dtau: float
    mu: float
    lattice: str = "kagome"   # or "triangular", "honeycomb" (App. A)

    def __post_init__(self):
        self.K = lattice.lattice_K(self.lattice, self.L, self.t)
        self.N = self.K.shape[0]
        self.L_tau = int(round(self.beta / self.dtau))
        km = self.K - self.mu * np.eye(self.N)
        # Dense propagators: the plain definition of the product of Eq. (5).
        self.E = scipy.linalg.expm(-self.dtau * km)
        self.Einv = scipy.linalg.expm(self.dtau * km)
        # The wrap exp(-dtau K) G exp(dtau K): mu cancels between the factors.
        self.EK = scipy.linalg.expm(-self.dtau * self.K)
        self.EKinv = scipy.linalg.expm(self.dtau * self.K)
        self.alpha = hs_alpha(self.U, self.dtau)

    @classmethod
    def from_workload(cls, w, mu=None):
        if mu is None:
            mu = lattice.dirac_mu(w.L, w.t)
        return cls(L=w.L, t=w.t, U=w.U, beta=w.beta, dtau=w.dtau, mu=mu)


def expm_eigh(a: np.ndarray) -> np.ndarray:
    """exp(a) for real symmetric a via its eigendecomposition (cross-check of expm)."""
    w, v = np.linalg.eigh(a)
    return (v * np.exp(w)) @ v.T


def b_matrix(model: Model, s_l: np.ndarray) -> np.ndarray:
    """B_l = exp(-dtau (K - mu)) diag(exp(alpha s_l))."""
    return model.E * np.exp(model.alpha * s_l.astype(float))[None, :]


def wrap(model: Model, g: np.ndarray, s_l: np.ndarray) -> np.ndarray:
    """G(l) = B_l G(l-1) B_l^{-1} with unchanged fields."""
    ev = np.exp(model.alpha * s_l.astype(float))
    gt = ev[:, None] * g / ev[None, :]
    return model.EK @ gt @ model.EKinv


# ----------------------------------------------------------------------------
# QR-stabilized products (UDT form) and the stable inverse
# ----------------------------------------------------------------------------

def udt_step(b: np.ndarray, u: np.ndarray, d: np.ndarray, t: np.ndarray):
    """Given X = U diag(D) T, return the UDT form of B X.

    Column-pivoted Householder QR of C = (B U) diag(D): C P = Q R, then
    U' = Q, D' = |diag R|, T' = diag(D')^{-1} R P^T T.
    """
    c = (b @ u) * d[None, :]
    q, r, piv = scipy.linalg.qr(c, pivoting=True)
    dn = np.abs(np.diag(r))
    tn = (r / dn[:, None]) @ t[piv, :]
    return q, dn, tn


def udt_product(bs):
    """UDT form of bs[-1] @ ... @ bs[1] @ bs[0] (bs[0] is the rightmost factor)."""
    n = bs[0].shape[0]
    u, d, t = np.eye(n), np.ones(n), np.eye(n)
    for b in bs:
        u, d, t = udt_step(b, u, d, t)
    return u, d, t


def green_from_udt(u: np.ndarray, d: np.ndarray, t: np.ndarray) -> np.ndarray:
    """(I + U diag(D) T)^{-1} with the Loh-Gubernatis scale separation.

    With D = Db Ds, Db = max(D, 1), Ds = min(D, 1):
    I + U D T = U Db (Db^{-1} U^T + Ds T) (U^T U = I), hence
    (I + U D T)^{-1} = (Db^{-1} U^T + Ds T)^{-1} Db^{-1} U^T.
    """
    db = np.maximum(d, 1.0)
    ds = np.minimum(d, 1.0)
    rhs = u.T / db[:, None]
    return np.linalg.solve(rhs + ds[:, None] * t, rhs)


def chain_order(l: int, L_tau: int):
    """Slice indices of B_l ... B_1 B_{L_tau} ... B_{l+1}, rightmost first."""
    return list(range(l + 1, L_tau + 1)) + list(range(1, l + 1))


def green_scratch(model: Model, fields: np.ndarray, l: int) -> np.ndarray:
    """QR-stabilized G(l) = [I + B_l ... B_1 B_{L_tau} ... B_{l+1}]^{-1}.

    ``fields`` has shape (L_tau, N); row l-1 holds slice l (1-based slices).
    """
    L_tau = fields.shape[0]
    bs = [b_matrix(model, fields[j - 1]) for j in chain_order(l, L_tau)]
    return green_from_udt(*udt_product(bs))


def green_dense(model: Model, fields: np.ndarray, l: int) -> np.ndarray:
    """Unstabilized G(l): plain product and inverse (only for short, warm chains)."""
    L_tau = fields.shape[0]
    p = np.eye(model.N)
    for j in chain_order(l, L_tau):
        p = b_matrix(model, fields[j - 1]) @ p
    return np.linalg.inv(np.eye(model.N) + p)


def green_free(model: Model) -> np.ndarray:
    """U = 0 closed form (I + exp(-beta (K - mu)))^{-1} in the eigenbasis of K."""
    w, v = np.linalg.eigh(model.K)
    f = 1.0 / (1.0 + np.exp(-model.beta * (w - model.mu)))
    return (v * f) @ v.T


# ----------------------------------------------------------------------------
# Single-flip ratio and the updates of one slice
# ----------------------------------------------------------------------------

def flip_delta(alpha: float, s: int) -> float:
    """Delta = exp(-2 alpha s) - 1: exp(V) changes by (1 + Delta) at the site."""
    return float(np.exp(-2.0 * alpha * s) - 1.0)


def flip_ratio(alpha: float, s: int, g_ii: float):
    """Weight ratio of flipping s at a site with current G~_ii.

    The determinant of each spin changes by R = 1 + Delta (1 - G~_ii); the
    factor prod exp(-alpha s) of the decoupling changes by exp(2 alpha s).
    Returns (ratio, R, Delta).
    """
    delta = flip_delta(alpha, s)
    r = 1.0 + delta * (1.0 - g_ii)
    return float(np.exp(2.0 * alpha * s) * r * r), r, delta


def update_slice(gt: np.ndarray, s: np.ndarray, alpha: float, u=None, forced=None, k: int = 1):
    """Sequential Metropolis over the sites of one slice with delay k.

    ``gt`` is G~ = exp(V_l) G(l-1) exp(-V_l) (modified copy returned), ``s``
    the slice's fields (flipped in place), ``u`` the uniforms, ``forced`` an
    optional 0/1 decision per site that replaces the Metropolis test.

    Delayed update (classic form): with pending factors U (N x m), W (m x N),
    G~cur = G~ + U W.  An accepted flip at i appends
    u = -(Delta/R) G~cur[:, i] and w = e_i - G~cur[i, :]; when m reaches k
    the factors are added to G~.  Returns (G~, accepted, ratios).
    """
    gt = gt.copy()
    n = gt.shape[0]
    acc = np.zeros(n, dtype=bool)
    ratios = np.zeros(n)
    uu = np.zeros((n, k))
    ww = np.zeros((k, n))
    m = 0
    for i in range(n):
        g_ii = gt[i, i] + uu[i, :m] @ ww[:m, i]
        ratio, r, delta = flip_ratio(alpha, int(s[i]), g_ii)
        ratios[i] = ratio
        if forced is not None:
            a = bool(forced[i])
        else:
            a = bool(u[i] < ratio)
        if not a:
            continue
        acc[i] = True
        col = gt[:, i] + uu[:, :m] @ ww[:m, i]
        row = gt[i, :] + uu[i, :m] @ ww[:m, :]
        uu[:, m] = -(delta / r) * col
        ww[m, :] = -row
        ww[m, i] += 1.0
        m += 1
        s[i] = -s[i]
        if m == k:
            gt += uu[:, :m] @ ww[:m, :]
            m = 0
    if m:
        gt += uu[:, :m] @ ww[:m, :]
    return gt, acc, ratios


def sweep(model: Model, fields: np.ndarray, g0: np.ndarray, uniforms=None, forced=None,
          k: int = 1, n_stab: int = 10, record: bool = True, l_stop=None, green=None):
    """One upward pass l = 1..L_tau over the slices.

    Per slice: G~ = exp(V_l) G exp(-V_l); sequential updates (delay k);
    G = exp(-dtau K) G~ exp(dtau K); every n_stab slices G is replaced by the
    QR-stabilized G(l) and max|G - G_fresh| is logged as the wrap error.

    ``l_stop`` ends the pass after that slice (a partial sweep).  ``green``
    (fields, l) -> G(l) gives the fresh G at the stabilizations (default: the
    finite-temperature green_scratch; the projector passes its own).

    Returns a dict with the final fields, G after every slice (``G_slices``,
    index l-1, taken after the stabilization of that slice when there is one),
    the wrapped G before each stabilization (``G_prestab``), accept flags,
    ratios and wrap errors.
    """
    if green is None:
        green = lambda f, l: green_scratch(model, f, l)  # noqa: E731
    fields = fields.copy()
    L_tau, n = fields.shape
    acc = np.zeros((L_tau, n), dtype=bool)
    ratios = np.zeros((L_tau, n))
    wrap_err = {}
    g_slices, g_pre = [], {}
    g = g0.copy()
    for l in range(1, (L_tau if l_stop is None else l_stop) + 1):
        s = fields[l - 1]
        ev = np.exp(model.alpha * s.astype(float))
        gt = ev[:, None] * g / ev[None, :]
        gt, acc[l - 1], ratios[l - 1] = update_slice(
            gt, s, model.alpha,
            None if uniforms is None else uniforms[l - 1],
            None if forced is None else forced[l - 1], k)
        g = model.EK @ gt @ model.EKinv
        if l % n_stab == 0:
            g_pre[l] = g.copy()
            gf = green(fields, l)
            wrap_err[l] = float(np.max(np.abs(g - gf)))
            g = gf
        if record:
            g_slices.append(g.copy())
    return dict(fields=fields, G=g, G_slices=g_slices, G_prestab=g_pre,
                accepted=acc, ratios=ratios, wrap_err=wrap_err)


def sweep_down(model: Model, fields: np.ndarray, g_top: np.ndarray, uniforms=None, forced=None,
               k: int = 1, n_stab: int = 10, record: bool = True, l_stop=None, l_start=None,
               green=None):
    """One downward pass l = L_tau..1 over the slices, starting from
    G(L_tau) = G(0).

    Per slice, read off the same relation as the upward pass backwards:
    G~ = exp(dtau K) G(l) exp(-dtau K) is exp(V_l) G(l-1) exp(-V_l), the matrix
    on which the flips of slice l act; after the sequential updates (delay k),
    G(l-1) = exp(-V_l) G~ exp(V_l) with the new fields.  Whenever l-1 is a
    multiple of n_stab (l-1 = 0 included) G is replaced by the QR-stabilized
    G(l-1) and max|G - G_fresh| is logged.

    ``l_start`` begins at another slice (then ``g_top`` is G(l_start)) and
    ``l_stop`` ends the pass after the slice of that index; ``green`` as in
    ``sweep``.  Returns the same
    dict as ``sweep``; ``G_slices`` holds G(l-1) in visiting order (index
    L_tau - l), and ``G_prestab`` / ``wrap_err`` are keyed by l-1.
    """
    if green is None:
        green = lambda f, l: green_scratch(model, f, l)  # noqa: E731
    fields = fields.copy()
    L_tau, n = fields.shape
    acc = np.zeros((L_tau, n), dtype=bool)
    ratios = np.zeros((L_tau, n))
    wrap_err = {}
    g_slices, g_pre = [], {}
    g = g_top.copy()
    top = L_tau if l_start is None else l_start
    for l in range(top, (1 if l_stop is None else l_stop) - 1, -1):
        s = fields[l - 1]
        gt = model.EKinv @ g @ model.EK
        gt, acc[l - 1], ratios[l - 1] = update_slice(
            gt, s, model.alpha,
            None if uniforms is None else uniforms[l - 1],
            None if forced is None else forced[l - 1], k)
        ev = np.exp(model.alpha * s.astype(float))
        g = gt / ev[:, None] * ev[None, :]
        if (l - 1) % n_stab == 0:
            g_pre[l - 1] = g.copy()
            gf = green(fields, l - 1)
            wrap_err[l - 1] = float(np.max(np.abs(g - gf)))
            g = gf
        if record:
            g_slices.append(g.copy())
    return dict(fields=fields, G=g, G_slices=g_slices, G_prestab=g_pre,
                accepted=acc, ratios=ratios, wrap_err=wrap_err)

