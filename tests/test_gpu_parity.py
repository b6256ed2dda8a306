"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: SINR within 0.05 dB of the oracle; reconstruction within 1e-5 relative (FP32
arithmetic); the objective trace within 1e-5 of ||X||^2; NMSE within 1e-5 relative plus
1e-10 absolute; integer layout bit-exact.
"""

import numpy as np
import pytest
import torch

import synthgen
from oracle import metrics, sinr as osinr, tucker
from tests.gpu_util import announce, crandn, db, desc, dev_c64, host, unpack

pytestmark = pytest.mark.gpu

SNRS = (-5.0, 0.0, 10.0, 20.0)


def _plan(api, descs, iters=10, **kw):
    return api.Plan(descs, iters=iters, **kw)


@pytest.fixture(scope="module")
def small_case():
    cfg = synthgen.CONFIGS["small"]
    X = synthgen.make_channel(cfg)
    r = tucker.fit(X, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.iters)
    Ht, Xh = tucker.reconstruct(r["A"], r["B"], r["C"], r["G"], cfg.group_size)
    return cfg, X, r, Ht, Xh


def test_sinr_compressed_matches_oracle(gpu_lib, small_case):
    cfg, X, r, Ht, _ = small_case
    announce("sinr compressed small")
    plan = _plan(gpu_lib, [gpu_lib.desc_from_config(cfg)])
    s2 = synthgen.snr_to_sigma2(SNRS)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = host(plan.sinr(dev_c64(r["C"]), dev_c64(r["G"]), s2, status=st))
    ref = osinr.sinr(Ht, s2, cfg.ns)
    assert out.shape == (4, cfg.nsc, cfg.ns)
    err = np.abs(db(out) - db(ref))
    assert err.max() <= 0.05, err.max()
    assert int(st.item()) & ~8 == 0


def test_sinr_full_matches_oracle(gpu_lib, small_case):
    cfg, X, r, Ht, _ = small_case
    announce("sinr full small")
    plan = _plan(gpu_lib, [gpu_lib.desc_from_config(cfg)])
    s2 = synthgen.snr_to_sigma2(SNRS)
    out = host(plan.sinr_full(dev_c64(X), s2))
    ref = osinr.sinr(X, s2, cfg.ns)
    assert np.abs(db(out) - db(ref)).max() <= 0.05


def test_reconstruct_matches_oracle(gpu_lib, small_case):
    cfg, X, r, Ht, Xh = small_case
    announce("reconstruct small")
    plan = _plan(gpu_lib, [gpu_lib.desc_from_config(cfg)])
    ht, xh = plan.reconstruct(dev_c64(r["A"]), dev_c64(r["B"]), dev_c64(r["C"]), dev_c64(r["G"]))
    ht = unpack(plan, 0, host(ht), "ht")
    xh = unpack(plan, 0, host(xh), "x")
    assert np.linalg.norm(ht - Ht) <= 1e-5 * np.linalg.norm(Ht)
    assert np.linalg.norm(xh - Xh) <= 1e-5 * np.linalg.norm(Xh)


def _gpu_fit_and_check(api, X, gs, m, n, p, ns, iters, orc=None, xhat_tol=1e-4, trace=True,
                       **plan_kw):
    # trace=False fits without the objective trace: with m == nr that runs only the last A-step
    nsc, nr, nt = X.shape
    plan = _plan(api, [desc(nr, nt, nsc, gs, m, n, p, ns)], iters=iters, **plan_kw)
    res = plan.fit(dev_c64(X), trace=trace)
    torch.cuda.synchronize()
    ht, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"])
    A = unpack(plan, 0, host(res["A"]), "a")
    Bm = unpack(plan, 0, host(res["B"]), "b")
    Cm = unpack(plan, 0, host(res["C"]), "c")
    Xh = unpack(plan, 0, host(xh), "x")
    if orc is None:
        orc = tucker.fit(X, gs, m, n, p, iters)
    _, Xh_o = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"], gs)
    nx = np.sum(np.abs(X) ** 2)
    # factors orthonormal
    assert np.abs(A.conj().T @ A - np.eye(m)).max() < 1e-5
    assert np.abs(Bm.conj().T @ Bm - np.eye(n)).max() < 1e-5
    starts, sizes = tucker.group_layout(nsc, gs)
    for s0, sz in zip(starts, sizes):
        Cg = Cm[s0:s0 + sz, :min(p, sz)]
        assert np.abs(Cg.conj().T @ Cg - np.eye(Cg.shape[1])).max() < 1e-5
        assert np.all(Cm[s0:s0 + sz, min(p, sz):] == 0)
    nm_g = metrics.nmse(X, Xh)
    nm_o = metrics.nmse(X, Xh_o)
    assert abs(nm_g - nm_o) <= 1e-5 * nm_o + 1e-10, (nm_g, nm_o)
    assert np.linalg.norm(Xh - Xh_o) <= xhat_tol * np.sqrt(nx), np.linalg.norm(Xh - Xh_o) / np.sqrt(nx)
    if trace:
        tr = host(res["trace"])[0]
        assert np.abs(tr - orc["trace"]).max() <= 1e-5 * nx, np.abs(tr - orc["trace"]).max() / nx
    else:
        assert "trace" not in res
    assert int(res["status"].item()) == 0
    return plan, res, orc


def test_fit_small_config(gpu_lib, small_case):
    cfg, X, r, _, _ = small_case
    announce("fit small")
    _gpu_fit_and_check(gpu_lib, X, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.ns, cfg.iters, orc=r)


@pytest.mark.parametrize("case", [
    # (nsc, nr, nt, gs, m, n, p, iters, seed)
    (30, 6, 10, 8, 3, 4, 3, 6, 7),        # lossy, short last group of 6
    (40, 8, 16, 12, 4, 6, 6, 5, 11),      # last group of 4 < p: p_g = 4
    (25, 4, 32, 5, 2, 8, 2, 4, 13),       # many small groups
    # m > 8: the B-step's 32 x 32 x 2 step 2 with a per-channel slot stride (1280 floats), and
    # the T pass's vector-ALU Yh
    (60, 12, 40, 12, 10, 8, 6, 5, 17),
    # groups of 24 (the B-step pass's 24-slice variant, two T tiles per wave), short last group
    (70, 8, 32, 24, 4, 8, 10, 5, 29),
    # groups of 32 (past the all-matrix-core B-step pass's limit)
    (64, 4, 16, 32, 3, 6, 8, 5, 31),
    # nr = 16, the largest receive array of the fused passes
    (70, 16, 16, 12, 12, 6, 6, 5, 37),
])
def test_fit_lossy_random(gpu_lib, case):
    nsc, nr, nt, gs, m, n, p, iters, seed = case
    announce(f"fit lossy {case}")
    rng = np.random.default_rng(seed)
    # decaying spectra keep the eigengaps at the cuts well separated
    X = crandn(rng, nsc, nr, nt)
    X = X * (0.6 ** np.arange(nr))[None, :, None] * (0.8 ** np.arange(nt))[None, None, :]
    _gpu_fit_and_check(gpu_lib, X, gs, m, n, p, min(m, n, 2), iters, xhat_tol=1e-4)


def test_fit_planted_exact(gpu_lib):
    announce("fit planted exact")
    rng = np.random.default_rng(6)
    X, *_ = synthgen.planted_tucker(rng, 8, 16, 40, 12, 3, 5, 4)
    _gpu_fit_and_check(gpu_lib, X, 12, 3, 5, 4, 2, 3)


def test_fit_deterministic(gpu_lib, small_case):
    cfg, X, _, _, _ = small_case
    announce("fit determinism")
    plan = _plan(gpu_lib, [gpu_lib.desc_from_config(cfg)], iters=cfg.iters)
    Xd = dev_c64(X)
    a = plan.fit(Xd)
    a = {k: v.clone() for k, v in a.items()}
    b = plan.fit(Xd)
    for k in ("A", "B", "C", "G", "trace"):
        assert torch.equal(a[k], b[k]), k


def test_batch_of_two_shapes(gpu_lib):
    announce("fit batch of two shapes")
    rng = np.random.default_rng(21)
    X0 = crandn(rng, 20, 4, 8) * (0.7 ** np.arange(8))[None, None, :]
    X1, *_ = synthgen.planted_tucker(rng, 6, 12, 36, 9, 3, 4, 3)
    d0 = desc(4, 8, 20, 6, 2, 3, 2, 2)
    d1 = desc(6, 12, 36, 9, 3, 4, 3, 3)
    plan = _plan(gpu_lib, [d0, d1], iters=4)
    Xp = np.concatenate([X0.reshape(-1), X1.reshape(-1)])
    res = plan.fit(dev_c64(Xp))
    _, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"])
    xh = host(xh)
    s2 = [0.1, 1.0]
    sg = host(plan.sinr(res["C"], res["G"], s2))
    for c, (X, d) in enumerate(((X0, d0), (X1, d1))):
        orc = tucker.fit(X, d["group_size"], d["m"], d["n"], d["p"], 4)
        Ht_o, Xh_o = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"], d["group_size"])
        Xh = unpack(plan, c, xh, "x")
        assert np.linalg.norm(Xh - Xh_o) <= 1e-4 * np.linalg.norm(X)
        o = plan.offsets(c)
        ref = osinr.sinr(Ht_o, s2, d["ns"])
        got = sg[:, o.sc:o.sc + d["nsc"], :d["ns"]]
        assert np.abs(db(got) - db(ref)).max() <= 0.05
        if d["ns"] < plan.ns_max:
            assert np.all(sg[:, o.sc:o.sc + d["nsc"], d["ns"]:] == 0)


def test_zero_stream_status(gpu_lib):
    announce("sinr zero stream status")
    d = desc(4, 8, 12, 12, 3, 4, 2, 3)
    plan = _plan(gpu_lib, [d])
    rng = np.random.default_rng(3)
    Cm = np.zeros((12, 2), np.complex128)
    Cm[:, :2] = synthgen.random_unitary(rng, 12, 2)
    G = np.zeros((1, 2, 3, 4), np.complex128)
    G[0, :, 0, :] = crandn(rng, 2, 4)            # rank-1 compressed channels
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = host(plan.sinr(dev_c64(Cm), dev_c64(G), [0.5], status=st))
    assert int(st.item()) & 8
    assert np.all(out[..., 1:] == 0) and np.all(out[..., 0] > 0)


def test_sinr_full_mixed_arrays(gpu_lib):
    # the full-channel SINR on 4-, 8- and 16-lane groups (one plan per array size), and the
    # three channels in one plan (16-lane groups for all), against the oracle per channel
    announce("sinr full mixed arrays")
    rng = np.random.default_rng(41)
    shapes = [(4, 32, 20, 2), (6, 40, 18, 3), (12, 64, 16, 4)]  # nr, nt, nsc, ns
    descs = [desc(nr, nt, nsc, 8, min(nr, 4), 8, 4, ns) for nr, nt, nsc, ns in shapes]
    Xs = [crandn(rng, nsc, nr, nt) for nr, nt, nsc, _ in shapes]
    s2 = synthgen.snr_to_sigma2(SNRS)
    plans = [([d], [x]) for d, x in zip(descs, Xs)] + [(descs, Xs)]
    for ds, xs in plans:
        plan = _plan(gpu_lib, ds, iters=2)
        out = host(plan.sinr_full(dev_c64(np.concatenate([x.reshape(-1) for x in xs])), s2))
        for c, (d, X) in enumerate(zip(ds, xs)):
            o = plan.offsets(c)
            ref = osinr.sinr(X, s2, d["ns"])
            got = out[:, o.sc:o.sc + d["nsc"], :d["ns"]]
            err = np.abs(db(got) - db(ref)).max()
            print(f"[sinr full] {len(ds)} channel(s), nr {d['nr']}: max error {err:.3e} dB", flush=True)
            assert err <= 0.05, (len(ds), c, err)


def test_reconstruct_ht_only_matches(gpu_lib):
    # Ht alone (one block per group) against Ht from the per-subcarrier kernel that also forms
    # Xhat: the same sums in the same order (the compiler may contract them into different fused
    # multiply-adds, so rounding-level differences remain); uneven groups in a batch of two
    announce("reconstruct Ht only")
    rng = np.random.default_rng(43)
    d0, d1 = desc(6, 16, 29, 12, 4, 6, 5, 2), desc(8, 32, 40, 8, 6, 10, 7, 3)
    plan = _plan(gpu_lib, [d0, d1], iters=2)
    t = plan.totals
    A, Bm, C, G = (dev_c64(crandn(rng, k)) for k in (t.a, t.b, t.c, t.g))
    ht_full, _ = plan.reconstruct(A, Bm, C, G, ht=True, xhat=True)
    ht_only, xh = plan.reconstruct(A, Bm, C, G, ht=True, xhat=False)
    assert xh is None
    a, b = host(ht_only), host(ht_full)
    err = np.abs(a - b).max() / np.abs(b).max()
    print(f"[reconstruct] Ht only vs with Xhat: {err:.3e} of max |Ht|", flush=True)
    assert err <= 1e-6, err


@pytest.mark.parametrize("case", [
    # (nsc, nr, nt, gs, m, n, p, iters, seed), all with m == nr: without the trace the fit runs
    # only the last A-step, the B-step skips its A^H product and the T pass takes the mode-3
    # Gram of T (A is square and unitary, so A A^H = I)
    (40, 6, 16, 12, 6, 6, 6, 5, 41),      # nt < 64: the B-step's zero columns past nt
    (70, 8, 32, 24, 8, 8, 10, 5, 43),     # groups of 24, short last group
    (50, 8, 64, 12, 8, 16, 12, 6, 47),    # the 8 x 64 shape of the headline workload
    (30, 4, 16, 8, 4, 4, 3, 1, 53),       # one sweep: its A-step is the last
])
def test_fit_full_mode1_untraced(gpu_lib, case):
    nsc, nr, nt, gs, m, n, p, iters, seed = case
    announce(f"fit m == nr without trace {case}")
    rng = np.random.default_rng(seed)
    X = crandn(rng, nsc, nr, nt)
    X = X * (0.6 ** np.arange(nr))[None, :, None] * (0.8 ** np.arange(nt))[None, None, :]
    orc = tucker.fit(X, gs, m, n, p, iters)
    plan, res, _ = _gpu_fit_and_check(gpu_lib, X, gs, m, n, p, min(m, n, 2), iters, orc=orc,
                                      xhat_tol=1e-4, trace=False)
    # the same plan with the trace runs every A-step: the reconstructions agree
    full = plan.fit(dev_c64(X), trace=True)
    _, xa = plan.reconstruct(res["A"], res["B"], res["C"], res["G"])
    _, xb = plan.reconstruct(full["A"], full["B"], full["C"], full["G"])
    xa, xb = host(xa), host(xb)
    rel = np.linalg.norm(xa - xb) / np.linalg.norm(xb)
    print(f"[full mode 1] untraced vs traced X-hat {rel:.3e}", flush=True)
    assert rel <= 1e-5, rel


def test_fit_full_mode1_warm_start_non_unitary_a(gpu_lib):
    # a caller's A need not be unitary: with m == nr and no trace the first A-step still runs
    # before the first B-step, so the continuation matches the oracle's (whose A-step does not
    # read A)
    announce("fit m == nr warm start from a non-unitary A")
    rng = np.random.default_rng(59)
    nsc, nr, nt, gs, m, n, p = 40, 6, 16, 12, 6, 6, 6
    X = crandn(rng, nsc, nr, nt)
    X = X * (0.6 ** np.arange(nr))[None, :, None] * (0.8 ** np.arange(nt))[None, None, :]
    d = desc(nr, nt, nsc, gs, m, n, p, 2)
    r1 = _plan(gpu_lib, [d], iters=3).fit(dev_c64(X))
    warm = _plan(gpu_lib, [d], iters=3, warm_start=True)
    f = {k: r1[k].clone() for k in ("A", "B", "C", "G")}
    f["A"] *= 2.0
    r2 = warm.fit(dev_c64(X), factors=f, trace=False)
    _, xh = warm.reconstruct(r2["A"], r2["B"], r2["C"], r2["G"])
    Xh = unpack(warm, 0, host(xh), "x")
    half = tucker.fit(X, gs, m, n, p, 3)
    half["A"] = 2.0 * half["A"]
    rest = tucker.fit(X, gs, m, n, p, 3, warm=half)
    _, Xh_o = tucker.reconstruct(rest["A"], rest["B"], rest["C"], rest["G"], gs)
    rel = np.linalg.norm(Xh - Xh_o) / np.linalg.norm(X)
    print(f"[full mode 1 warm] X-hat {rel:.3e} of ||X||", flush=True)
    assert int(r2["status"].item()) == 0
    assert rel <= 1e-4, rel


def test_fit_warm_start_resume(gpu_lib):
    # GT_FIT_WARM_START: three sweeps resumed from the factors of a three-sweep fit follow the
    # oracle's warm continuation (which the oracle pins equal to an uninterrupted six-sweep fit)
    announce("fit warm start resume")
    rng = np.random.default_rng(51)
    nsc, nr, nt, gs, m, n, p = 40, 8, 16, 12, 4, 6, 6
    X = crandn(rng, nsc, nr, nt)
    X = X * (0.6 ** np.arange(nr))[None, :, None] * (0.8 ** np.arange(nt))[None, None, :]
    d = desc(nr, nt, nsc, gs, m, n, p, 2)
    r1 = _plan(gpu_lib, [d], iters=3).fit(dev_c64(X))
    warm = _plan(gpu_lib, [d], iters=3, warm_start=True)
    f = {k: r1[k].clone() for k in ("A", "B", "C", "G")}
    r2 = warm.fit(dev_c64(X), factors=f)
    _, xh = warm.reconstruct(r2["A"], r2["B"], r2["C"], r2["G"])
    Xh = unpack(warm, 0, host(xh), "x")
    half = tucker.fit(X, gs, m, n, p, 3)
    rest = tucker.fit(X, gs, m, n, p, 3, warm=half)
    _, Xh_o = tucker.reconstruct(rest["A"], rest["B"], rest["C"], rest["G"], gs)
    nx = float(np.sum(np.abs(X) ** 2))
    rel = np.linalg.norm(Xh - Xh_o) / np.sqrt(nx)
    tr = host(r2["trace"])[0]
    tr_err = np.abs(tr[1:] - rest["trace"][1:]).max() / nx
    print(f"[warm] X-hat {rel:.3e} of ||X||, trace {tr_err:.3e} of ||X||^2", flush=True)
    assert int(r2["status"].item()) == 0
    assert rel <= 1e-4, rel
    assert tr_err <= 1e-5, tr_err
