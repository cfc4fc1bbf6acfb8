"""GPU parity at the full lattice sizes of the workloads, through the C ABI,
against the oracle on identical seeded fields with its decisions replayed:

* L=24 (N=1728): the first ten slices and the first stabilization (window
  launches over 27 x 27 tiles, 512-thread QR panels, the triangular solve at
  n = 1728);
* L=18 (N=972), U=-5: the same in FP64, and the mixed precision at its tuned
  stabilization interval against the 1e-5 target;
* L=12 at beta=24 (240 slices): G from the stacks at the widest range of
  scales, where ordering the columns by norm before an unpivoted QR stands
  in for the oracle's column-pivoted QR.

Between stabilizations every FP64 implementation drifts from the exact G(l)
(the wrap amplifies rounding from one slice to the next); the drift grows
monotonically over an interval and the oracle's own drift at the end of the
interval is its wrap error there.  Per slice the GPU must therefore agree
with the oracle within max(1e-10, 2 x that drift), and right after the
stabilization, where both sides are fresh, within 1e-10 (Sec. II, Eqs. 5-6:
the wrap is the propagator product applied on both sides of G)."""
import numpy as np
import pytest

import seeded_inputs as si
from gpu_helpers import chain, dev, model, say, torch
from oracle import dqmc

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _ten_slices(L, U, beta, seed, k=32, prec="fp64", n_stab=10, tol=None, slices=10):
    """Oracle's first `slices` slices (Metropolis), replayed on the GPU slice by
    slice; returns the per-slice differences and the oracle's record."""
    m = model(L, U, beta)
    f = si.ising_fields(L, m.L_tau, seed)
    u = si.metropolis_uniforms(L, m.L_tau, seed)[0]
    say(f"full-size L={L} U={U} beta={beta}: oracle G(0)")
    g0 = dqmc.green_scratch(m, f, 0)
    say(f"full-size L={L}: oracle sweep of {slices} slices")
    r = dqmc.sweep(m, f, g0, uniforms=u, k=k, n_stab=10, l_stop=slices)
    t = torch()
    ch = chain(L, U, beta, delay_k=k, prec=prec, n_stab=n_stab)
    if tol is not None:
        ch.set_wrap_tolerance(tol)
    say(f"full-size L={L}: GPU set_fields")
    ch.set_fields(dev(f))
    d0 = float(np.abs(ch.G().cpu().numpy() - g0).max())
    forced = dev(r["accepted"][:slices].astype(np.uint8))
    ratio = t.zeros((slices, m.N), dtype=t.float64, device="cuda:0")
    acc = t.zeros((slices, m.N), dtype=t.uint8, device="cuda:0")
    diffs, post = [], {}
    err = t.zeros(1, dtype=t.float64, device="cuda:0")
    for l in range(1, slices + 1):
        ch.sweep_slice(l, None, forced[l - 1], acc[l - 1], ratio[l - 1])
        ref = r["G_prestab"][l] if l in r["G_prestab"] else r["G_slices"][l - 1]
        diffs.append(float(np.abs(ch.G().cpu().numpy() - ref).max()))
        if l % n_stab == 0:
            ch.stabilize(err)
            if l in r["G_prestab"]:
                post[l] = (float(np.abs(ch.G().cpu().numpy() - r["G_slices"][l - 1]).max()),
                           float(err.cpu()[0]))
    rr = ratio.cpu().numpy()
    rel = float(np.abs(rr - r["ratios"][:slices]).max() / np.abs(r["ratios"][:slices]).max())
    same_acc = bool(np.array_equal(acc.cpu().numpy().astype(bool), r["accepted"][:slices]))
    ch.close()
    return dict(d0=d0, diffs=diffs, post=post, ratio_rel=rel, same_acc=same_acc, r=r, m=m)


@pytest.mark.timeout(600)
def test_l24_ten_slices_and_stabilization(gpu_lib):
    """L=24, U=-4, beta=2 (N=1728, 20 slices), delay k=32 in 32-site windows."""
    res = _ten_slices(24, -4.0, 2.0, 24)
    drift = res["r"]["wrap_err"][10]
    tol = max(TOL64, 2.0 * drift)
    say("L24 G(0)", res["d0"], "per-slice", res["diffs"], "oracle drift", drift, "post", res["post"],
        "ratio rel", res["ratio_rel"])
    assert res["d0"] < TOL64
    assert max(res["diffs"]) < tol
    d_post, e_gpu = res["post"][10]
    assert d_post < TOL64
    assert e_gpu < tol
    assert res["ratio_rel"] < 1e-9
    assert res["same_acc"]


@pytest.mark.timeout(600)
def test_l18_fp64_ten_slices_and_stabilization(gpu_lib):
    """The L=18 lattice at its coupling U=-5 and beta=12 (L_tau=120), FP64."""
    res = _ten_slices(18, -5.0, 12.0, 18)
    drift = res["r"]["wrap_err"][10]
    tol = max(TOL64, 2.0 * drift)
    say("L18 G(0)", res["d0"], "per-slice", res["diffs"], "oracle drift", drift, "post", res["post"],
        "ratio rel", res["ratio_rel"])
    assert res["d0"] < TOL64
    assert max(res["diffs"]) < tol
    assert res["post"][10][0] < TOL64
    assert res["ratio_rel"] < 1e-9


@pytest.mark.timeout(600)
def test_l18_mixed_at_tuned_interval(gpu_lib):
    """Mixed precision (FP32 G and wrap, split FP16 flush; FP64 ratios and
    stabilization) on the L=18, U=-5 lattice at the stabilization interval the
    autotuner chose for it: every slice's G and every flip ratio within the
    1e-5 target of the oracle (beta=2: the first 20 slices)."""
    from paper_2608_03894_amd import autotune
    e = autotune.lookup_interval(18, -5.0, 12.0, 0.1, "mixed_f16")
    assert e is not None, "the L=18 mixed-precision interval has not been tuned"
    ns = e["n_stab"]
    say("L18 mixed interval", ns, e["table"])
    res = _ten_slices(18, -5.0, 2.0, 18, prec="mixed_f16", n_stab=ns, slices=20)
    say("L18 mixed n_stab", ns, "per-slice", res["diffs"], "ratio rel", res["ratio_rel"])
    assert max(res["diffs"]) < 1e-5
    assert res["ratio_rel"] < 1e-5


@pytest.mark.timeout(600)
def test_l12_beta24_stacks(gpu_lib):
    """L=12 at beta=24 (240 slices, the widest scale range of the workloads):
    G(0) from set_fields' full-length left stack, and the stabilized G at
    slices 10, 120 and 240 of an upward pass without flips (the right stack
    grown to full length), against the oracle's column-pivoted QR chains."""
    L, U, beta = 12, -4.0, 24.0
    m = model(L, U, beta)
    f = si.ising_fields(L, m.L_tau, 12)
    t = torch()
    ch = chain(L, U, beta, delay_k=32)
    say("L12 beta24: set_fields")
    ch.set_fields(dev(f))
    g0 = dqmc.green_scratch(m, f, 0)
    d0 = float(np.abs(ch.G().cpu().numpy() - g0).max())
    say("L12 beta24 G(0)", d0)
    assert d0 < TOL64
    zeros = t.zeros(m.N, dtype=t.uint8, device="cuda:0")
    worst = {}
    for l in range(1, m.L_tau + 1):
        ch.sweep_slice(l, None, zeros)
        if l % 10 == 0:
            ch.stabilize()
            if l in (10, 120, 240):
                g = ch.G().cpu().numpy()
                ref = dqmc.green_scratch(m, f, l % m.L_tau)
                worst[l] = float(np.abs(g - ref).max())
                say("L12 beta24 stabilized G at slice", l, worst[l])
    assert max(worst.values()) < TOL64


def test_graph_replay_new_pointers_without_sync(gpu_lib):
    """Four alternating passes, each handed a different uniform buffer with no
    host synchronization in between (every pass captures new graphs while the
    previous ones may still be queued), equal bit for bit to the same passes
    of direct launches."""
    say("graph: new pointers, no sync")
    t = torch()
    L, Lt = 6, 20
    N = 3 * L * L
    f = si.ising_fields(L, Lt, 11)
    u = dev(si.metropolis_uniforms(L, Lt, 11, n_sweeps=4))
    outs = []
    for graphs in (False, True):
        ch = chain(L, -4.0, 2.0, delay_k=16)
        ch.use_graphs(graphs)
        ch.set_fields(dev(f))
        accs = [t.zeros((Lt, N), dtype=t.uint8, device="cuda:0") for _ in range(4)]
        errs = [t.zeros(2, dtype=t.float64, device="cuda:0") for _ in range(4)]
        for s in range(4):
            (ch.sweep_down if s % 2 else ch.sweep)(u[s], None, accs[s], None, errs[s])
        res = (ch.G().cpu().numpy(), [a.cpu().numpy() for a in accs], [e.cpu().numpy() for e in errs])
        outs.append(res)
        ch.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][2], outs[1][2]):
        assert np.array_equal(a, b)


def test_health_flags_drift(gpu_lib):
    """The numeric-health checks, forced from the host: a perturbation loaded
    into G is caught by the next stabilization (ENUMERIC, with G replaced by
    the fresh value), a NaN is caught the same way, kdqmc_health reports the
    largest wrap error since the last call and clears it, and a clean chain
    passes."""
    from paper_2608_03894_amd import kdqmc
    say("health")
    t = torch()
    L = 3
    m = model(L, -4.0, 2.0)
    f = si.ising_fields(L, m.L_tau, 3)
    ch = chain(L, -4.0, 2.0, delay_k=8)
    ch.set_fields(dev(f))
    zeros = t.zeros(m.N, dtype=t.uint8, device="cuda:0")
    for l in range(1, 11):
        ch.sweep_slice(l, None, zeros)
    ch.stabilize()
    worst = ch.health()
    assert worst < 1e-6
    # a perturbation of 1e-3 at slice 10, wrapped to slice 20
    g = ch.G()
    g[0, 1] += 1e-3
    ch.set_G(g, 10)
    for l in range(11, 21):
        ch.sweep_slice(l, None, zeros)
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.stabilize()
    assert e.value.code == kdqmc.ENUMERIC
    fresh = dqmc.green_scratch(m, f, 0)
    assert np.abs(ch.G().cpu().numpy() - fresh).max() < TOL64   # replaced by the fresh G
    w, ok = ch.health(raise_on_error=False)
    assert not ok and w > 1e-6
    w2, ok2 = ch.health(raise_on_error=False)                   # cleared by the read
    assert ok2 and w2 == 0.0
    # a NaN
    g = ch.G()
    g[2, 2] = float("nan")
    ch.set_G(g, 10)
    for l in range(11, 21):
        ch.sweep_slice(l, None, zeros)
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.stabilize()
    assert e.value.code == kdqmc.ENUMERIC
    w, ok = ch.health(raise_on_error=False)
    assert not ok and w != w
    # a tolerance below every wrap error flags a clean chain too
    ch.set_fields(dev(f))
    ch.set_wrap_tolerance(1e-300)
    for l in range(1, 11):
        ch.sweep_slice(l, None, zeros)
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.stabilize()
    assert e.value.code == kdqmc.ENUMERIC
    with pytest.raises(kdqmc.KdqmcError):
        ch.set_wrap_tolerance(0.0)


def test_mixed_at_ten_slices_is_flagged(gpu_lib):
    """Mixed precision at a 10-slice interval on the L=12 lattice drifts beyond
    the default tolerance of 1e-4 (FP32 rounding amplified over ten wraps),
    and the stabilization says so instead of returning silently."""
    from paper_2608_03894_amd import kdqmc
    say("mixed n_stab=10 flagged")
    L, U, beta = 12, -4.0, 8.0
    m = model(L, U, beta)
    f = si.ising_fields(L, m.L_tau, 12)
    u = dev(si.metropolis_uniforms(L, m.L_tau, 12)[0])
    ch = chain(L, U, beta, delay_k=32, prec="mixed_f16", n_stab=10)
    ch.set_fields(dev(f))
    err = torch().zeros(1, dtype=torch().float64, device="cuda:0")
    for l in range(1, 11):
        ch.sweep_slice(l, u[l - 1])
    with pytest.raises(kdqmc.KdqmcError) as e:
        ch.stabilize(err)
    say("mixed n_stab=10 wrap error", float(err.cpu()[0]))
    assert e.value.code == kdqmc.ENUMERIC
    assert float(err.cpu()[0]) > 1e-4
