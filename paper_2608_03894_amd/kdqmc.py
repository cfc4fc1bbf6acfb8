"""ctypes binding of libkdqmc.so (include/kdqmc.h): argument marshalling only.

Every computation happens in the HIP library.  PyTorch supplies device
memory (the caller-owned workspace and the input/output tensors) and the HIP
stream; no array here is ever computed on the host.  If the shared library is
missing, ``load()`` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkdqmc.so")

FP64, MIXED_F16, MIXED_BF16 = 0, 1, 2
KAGOME, TRIANGULAR, HONEYCOMB = 0, 1, 2
LATTICE = {"kagome": KAGOME, "triangular": TRIANGULAR, "honeycomb": HONEYCOMB}
NSUB = {KAGOME: 3, TRIANGULAR: 1, HONEYCOMB: 2}
PREC = {"fp64": FP64, "mixed_f16": MIXED_F16, "mixed_bf16": MIXED_BF16, "fp32": MIXED_F16}

OK, EINVAL, EUNSUPPORTED, ESTATE, EHIP, ENUMERIC, ENOSPACE = 0, -1, -2, -3, -4, -5, -6


class KdqmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kdqmc error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int),
        ("t", ctypes.c_double),
        ("U", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("dtau", ctypes.c_double),
        ("n_stab", ctypes.c_int),
        ("delay_k", ctypes.c_int),
        ("window", ctypes.c_int),
        ("fft_tile", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("n_occ", ctypes.c_int),
        ("lattice", ctypes.c_int),
    ]


_lib = None

_vp = ctypes.c_void_p
_SIGS = {
    "kdqmc_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Params)]),
    "kdqmc_workspace_bytes_batch": (ctypes.c_size_t, [ctypes.POINTER(Params), ctypes.c_int]),
    "kdqmc_init_batch": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(Params), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_size_t, _vp]),
    "kdqmc_num_chains": (ctypes.c_int, [_vp]),
    "kdqmc_dirac_mu": (ctypes.c_double, [ctypes.c_int, ctypes.c_double]),
    "kdqmc_init_lattice": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(Params), _vp,
                                          ctypes.c_size_t, _vp]),
    "kdqmc_set_fields": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_get_fields": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_set_G": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "kdqmc_wrap_slice": (ctypes.c_int, [_vp, ctypes.c_int]),
    "kdqmc_sweep_slice": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "kdqmc_stabilize": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_sweep": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "kdqmc_sweep_slice_down": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "kdqmc_sweep_down": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "kdqmc_measure_G": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_current_slice": (ctypes.c_int, [_vp]),
    "kdqmc_sync": (ctypes.c_int, [_vp]),
    "kdqmc_destroy": (None, [_vp]),
    "kdqmc_last_error": (ctypes.c_char_p, []),
    "kdqmc_gemm_f64": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, _vp, ctypes.c_int, _vp,
                                      ctypes.c_int, ctypes.c_double, _vp, ctypes.c_int]),
    "kdqmc_qr_f64": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "kdqmc_expK_f64": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "kdqmc_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "kdqmc_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int)]),
    "kdqmc_phase_name": (ctypes.c_char_p, [ctypes.c_int]),
    "kdqmc_use_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "kdqmc_set_wrap_tolerance": (ctypes.c_int, [_vp, ctypes.c_double]),
    "kdqmc_set_slice_launch": (ctypes.c_int, [_vp, ctypes.c_int]),
    "kdqmc_trial_orbitals": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_double)]),
    "kdqmc_set_trial": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_measure": (ctypes.c_int, [_vp, _vp]),
    "kdqmc_qr_f64_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "kdqmc_health": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
}

NPHASE = 12
NOBS = 6
OBS_NAMES = ("s_pair_gamma", "s_pair_dk1", "s_pair_dk2", "cdw2_gamma", "cdw2_k", "density")


def load():
    """Loads the in-tree libkdqmc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() or "
                           "python paper_2608_03894_amd/build.py")
    # torch's HIP runtime must be in the process first: the library's
    # dependency libamdhip64.so.7 then binds to that same runtime by soname,
    # so device memory and streams from torch are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def gpu_available() -> bool:
    import torch
    return torch.cuda.is_available()


def last_error() -> str:
    return load().kdqmc_last_error().decode()


def _check(rc):
    if rc != OK:
        raise KdqmcError(rc, last_error())


def make_params(L, U, beta, dtau=0.1, t=1.0, mu=None, n_stab=10, delay_k=32, window=0,
                fft_tile=0, prec="fp64", n_occ=0, lattice="kagome") -> Params:
    """n_occ = 0: finite temperature; n_occ > 0: the projector form with n_occ
    trial orbitals projected over beta."""
    if mu is None:
        mu = dirac_mu(L, t)
    if isinstance(prec, str):
        prec = PREC[prec]
    if isinstance(lattice, str):
        lattice = LATTICE[lattice]
    return Params(L=L, t=t, U=U, mu=mu, beta=beta, dtau=dtau, n_stab=n_stab, delay_k=delay_k,
                  window=window, fft_tile=fft_tile, prec=prec, n_occ=n_occ, lattice=lattice)


TRIAL_EPS = 0.01


def trial_orbitals(L, n_occ, t=1.0, eps=TRIAL_EPS):
    """The library's trial orbitals (host): numpy array N x n_occ."""
    import numpy as np
    N = 3 * L * L
    out = np.zeros((N, n_occ), dtype=np.float64)
    _check(load().kdqmc_trial_orbitals(L, t, n_occ, eps,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def workspace_bytes(p: Params, n_chains: int = 1) -> int:
    return int(load().kdqmc_workspace_bytes_batch(ctypes.byref(p), n_chains))


def dirac_mu(L: int, t: float = 1.0) -> float:
    return float(load().kdqmc_dirac_mu(L, t))


def qr_f64_noalloc(n, ld, A, Q, stream=None):
    """kdqmc_qr_f64_noalloc: the QR building block without a context (its
    scratch is the library's static device array); A, Q: device tensors with
    row stride ld."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _check(load().kdqmc_qr_f64_noalloc(n, ld, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(Q.data_ptr()),
                                       ctypes.c_void_p(s.cuda_stream)))


def _ptr(x):
    if x is None:
        return None
    return ctypes.c_void_p(x.data_ptr())


class Chain:
    """A context with its workspace tensor and stream: one Markov chain, or
    n_chains chains of one shape (per-chain interaction U) run together.

    For n_chains > 1 every array argument holds one record per chain (leading
    dimension n_chains), each shaped as for a single chain."""

    def __init__(self, params: Params, device="cuda:0", stream=None, n_chains=1, U=None):
        import torch
        self.torch = torch
        self.p = params
        self.lib = load()
        self.device = torch.device(device)
        self.N = NSUB[params.lattice] * params.L * params.L
        self.L_tau = int(round(params.beta / params.dtau))
        self.n_chains = int(n_chains)
        nbytes = workspace_bytes(params, self.n_chains)
        if nbytes == 0:
            raise KdqmcError(EINVAL, last_error())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        u_arr = None
        if U is not None:
            if len(U) != self.n_chains:
                raise KdqmcError(EINVAL, "need one U per chain")
            u_arr = (ctypes.c_double * self.n_chains)(*[float(x) for x in U])
        _check(self.lib.kdqmc_init_batch(ctypes.byref(ctx), ctypes.byref(params), self.n_chains,
                                         u_arr, _ptr(self.ws), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    # -- the calls of the C ABI, same names ---------------------------------
    def set_trial(self, P):
        _check(self.lib.kdqmc_set_trial(self.ctx, _ptr(P)))

    def set_fields(self, s):
        _check(self.lib.kdqmc_set_fields(self.ctx, _ptr(s)))

    def get_fields(self, out):
        _check(self.lib.kdqmc_get_fields(self.ctx, _ptr(out)))

    def set_G(self, G, l):
        _check(self.lib.kdqmc_set_G(self.ctx, _ptr(G), l))

    def wrap_slice(self, l):
        _check(self.lib.kdqmc_wrap_slice(self.ctx, l))

    def sweep_slice(self, l, u=None, forced=None, accepted=None, ratio=None):
        _check(self.lib.kdqmc_sweep_slice(self.ctx, l, _ptr(u), _ptr(forced), _ptr(accepted),
                                          _ptr(ratio)))

    def sweep_slice_down(self, l, u=None, forced=None, accepted=None, ratio=None):
        _check(self.lib.kdqmc_sweep_slice_down(self.ctx, l, _ptr(u), _ptr(forced), _ptr(accepted),
                                               _ptr(ratio)))

    def sweep_down(self, u=None, forced=None, accepted=None, ratio=None, wrap_err=None):
        _check(self.lib.kdqmc_sweep_down(self.ctx, _ptr(u), _ptr(forced), _ptr(accepted), _ptr(ratio),
                                         _ptr(wrap_err)))

    def stabilize(self, wrap_err=None):
        _check(self.lib.kdqmc_stabilize(self.ctx, _ptr(wrap_err)))

    def sweep(self, u=None, forced=None, accepted=None, ratio=None, wrap_err=None):
        _check(self.lib.kdqmc_sweep(self.ctx, _ptr(u), _ptr(forced), _ptr(accepted), _ptr(ratio),
                                    _ptr(wrap_err)))

    def measure(self, out):
        """kdqmc_measure: the NOBS estimators of the current G into out (device)."""
        _check(self.lib.kdqmc_measure(self.ctx, _ptr(out)))

    def observables(self):
        """The estimators as a dict (or one dict per chain); synchronizes."""
        t = self.torch
        shape = (NOBS,) if self.n_chains == 1 else (self.n_chains, NOBS)
        out = t.zeros(shape, dtype=t.float64, device=self.device)
        self.measure(out)
        self.sync()
        v = out.cpu().numpy()
        if self.n_chains == 1:
            return dict(zip(OBS_NAMES, v.tolist()))
        return [dict(zip(OBS_NAMES, r.tolist())) for r in v]

    def measure_G(self, out):
        _check(self.lib.kdqmc_measure_G(self.ctx, _ptr(out)))

    def current_slice(self) -> int:
        r = self.lib.kdqmc_current_slice(self.ctx)
        if r < 0:
            _check(r)
        return r

    def sync(self):
        _check(self.lib.kdqmc_sync(self.ctx))

    def gemm_f64(self, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc):
        _check(self.lib.kdqmc_gemm_f64(self.ctx, int(ta), int(tb), M, N, K, alpha, _ptr(A), lda,
                                       _ptr(B), ldb, beta, _ptr(C), ldc))

    def expK_f64(self, A, lda=None, ncols=None, sign=-1):
        _check(self.lib.kdqmc_expK_f64(self.ctx, _ptr(A), lda or self.N, ncols or self.N, sign))

    def qr_f64(self, n, A, Q):
        _check(self.lib.kdqmc_qr_f64(self.ctx, n, _ptr(A), _ptr(Q)))

    def set_wrap_tolerance(self, tol):
        _check(self.lib.kdqmc_set_wrap_tolerance(self.ctx, float(tol)))

    def set_slice_launch(self, persistent):
        """True: one resident launch per slice where the shape allows it;
        False: one launch per window.  Returns whether the persistent launch
        is in use."""
        rc = self.lib.kdqmc_set_slice_launch(self.ctx, 1 if persistent else 0)
        if rc < 0:
            _check(rc)
        return rc == 1

    def health(self, raise_on_error=True):
        """Largest wrap error since the last call (synchronizes); raises
        KdqmcError(ENUMERIC) when a chain drifted or went non-finite, unless
        raise_on_error is False (then returns (worst, ok))."""
        worst = ctypes.c_double(0.0)
        rc = self.lib.kdqmc_health(self.ctx, ctypes.byref(worst))
        if raise_on_error:
            _check(rc)
            return worst.value
        if rc not in (OK, ENUMERIC):
            _check(rc)
        return worst.value, rc == OK

    def use_graphs(self, on=True):
        _check(self.lib.kdqmc_use_graphs(self.ctx, 1 if on else 0))

    def profile_enable(self, on=True):
        _check(self.lib.kdqmc_profile_enable(self.ctx, 1 if on else 0))

    def profile_read(self):
        """{phase: (milliseconds, launches)} recorded since the last enable/read."""
        ms = (ctypes.c_double * NPHASE)()
        n = (ctypes.c_int * NPHASE)()
        _check(self.lib.kdqmc_profile_read(self.ctx, ms, n))
        return {self.lib.kdqmc_phase_name(i).decode(): (ms[i], n[i]) for i in range(NPHASE)}

    # -- conveniences ---------------------------------------------------------
    def G(self):
        shape = (self.N, self.N) if self.n_chains == 1 else (self.n_chains, self.N, self.N)
        out = self.torch.empty(shape, dtype=self.torch.float64, device=self.device)
        self.measure_G(out)
        self.sync()
        return out

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.kdqmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent Markov chains of uneven shape (L, beta, U may all differ).

    Chains whose parameters agree except for U form one batched context
    (one launch per kernel for all of them); each such group runs on its own
    HIP stream, so the groups' sweeps overlap on the GPU.  Inputs are given
    per chain in the caller's order and packed per group once (set_inputs);
    sweep() then enqueues every group's sweep and makes the caller's current
    stream wait for all of them."""

    def __init__(self, params_list, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = list(params_list)
        groups = {}
        for i, p in enumerate(self.params):
            key = (p.L, p.t, p.mu, p.beta, p.dtau, p.n_stab, p.delay_k, p.window, p.fft_tile, p.prec,
                   p.n_occ, p.lattice)
            groups.setdefault(key, []).append(i)
        self.groups = []
        for key, idx in groups.items():
            stream = torch.cuda.Stream(self.device)
            ch = Chain(self.params[idx[0]], device=self.device, stream=stream, n_chains=len(idx),
                       U=[self.params[i].U for i in idx])
            self.groups.append({"idx": idx, "chain": ch, "stream": stream})
        self.n_chains = len(self.params)

    def set_inputs(self, fields, uniforms):
        """fields[c]: int8 (L_tau, N) device tensor; uniforms[c]: float64
        (n_sweeps, L_tau, N) device tensor of the chain's Metropolis draws."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        for g in self.groups:
            idx = g["idx"]
            g["fields"] = t.stack([fields[i] for i in idx]).contiguous()
            g["u"] = t.stack([uniforms[i] for i in idx], dim=1).contiguous()  # (sweeps, chains, L_tau, N)
            # one fixed buffer per group: every sweep passes the same pointers,
            # so its captured graphs are replayed rather than captured again
            g["ub"] = t.empty_like(g["u"][0])
            ch = g["chain"]
            g["acc"] = t.zeros((len(idx), ch.L_tau, ch.N), dtype=t.uint8, device=self.device)
            g["err"] = t.zeros((len(idx), ch.L_tau // ch.p.n_stab), dtype=t.float64, device=self.device)
            g["stream"].wait_stream(cur)
            with t.cuda.stream(g["stream"]):
                ch.set_fields(g["fields"])
        for g in self.groups:
            cur.wait_stream(g["stream"])

    def sweep(self, s, down=False):
        """One pass of every chain with its uniforms of sweep s (upward, or
        downward with down=True)."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        for g in self.groups:
            g["stream"].wait_stream(cur)
            with t.cuda.stream(g["stream"]):
                g["ub"].copy_(g["u"][s])
            fn = g["chain"].sweep_down if down else g["chain"].sweep
            fn(g["ub"], None, g["acc"], None, g["err"])
        for g in self.groups:
            cur.wait_stream(g["stream"])

    def accepted(self):
        return sum(int(g["acc"].sum().item()) for g in self.groups)

    def max_wrap_err(self):
        return max(float(g["err"].max().item()) for g in self.groups)

    def health(self):
        """(largest wrap error of any chain since the last call, all healthy)."""
        worst, ok = 0.0, True
        for g in self.groups:
            w, good = g["chain"].health(raise_on_error=False)
            worst = w if (w != w or w > worst) else worst
            ok = ok and good
        return worst, ok

    def field_updates_per_sweep(self):
        return sum(NSUB[p.lattice] * p.L * p.L * int(round(p.beta / p.dtau)) for p in self.params)

    def close(self):
        for g in self.groups:
            g["chain"].close()
