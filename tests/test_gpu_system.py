"""The multi-cell system of the groupwise model (equation "three matrix factorization"): the
fit with A shared per UE and B per base station, and the per-subcarrier SINR of every UE with
interference (equations "signal receiving", "covariance matrix", "Cov", "reduced inversion of
interference matrix", "SINR formula"), through the C ABI, against the FP64 oracle on a
synthetic system of 3 base stations with 2 UEs each (18 links).

Bars: reconstruction within 1e-4 of ||X|| over the system (the tensors have decaying spectra so
that the rank cuts have gaps), NMSE within 1e-5 relative plus 1e-10, and SINR within 0.05 dB
on every stream of every UE, for the single-link, the paper's inter-cell protocol and the full
intra- plus inter-cell interference.
"""

import numpy as np
import pytest
import torch

import synthgen
from oracle import metrics, multicell as mc, tucker
from tests.gpu_util import announce, crandn, db, dev_c64, host, unpack

pytestmark = pytest.mark.gpu

J, K = 3, 2
NR, NT, NSC, GS, M, N, P, NS, ITERS = 8, 32, 40, 12, 4, 8, 6, 2, 6
SNRS = (-5.0, 10.0, 20.0)


def system_descs(J, K, nr, nt, nsc, gs, m, n, p, ns):
    return [dict(nr=nr, nt=nt, nsc=nsc, group_size=gs, m=m, n=n, p=p, ns=ns, a_id=u + 1,
                 b_id=k + 1, serving=int(u // K == k)) for u, k in synthgen.system_links(J, K)]


@pytest.fixture(scope="module")
def system_case():
    rng = np.random.default_rng(91)
    links = synthgen.system_links(J, K)
    X = {}
    for lk in links:
        X[lk] = crandn(rng, NSC, NR, NT) * (0.6 ** np.arange(NR))[None, :, None] \
            * (0.85 ** np.arange(NT))[None, None, :]
    orc = mc.fit(X, GS, M, N, P, ITERS)
    Ht = {lk: tucker.compressed_channels(orc["C"][lk], orc["G"][lk], GS) for lk in links}
    return links, X, orc, Ht


def _pack(plan, links, arrs, what):
    t = getattr(plan.totals, what)
    buf = np.zeros(t, np.complex128)
    for c, lk in enumerate(links):
        o = getattr(plan.offsets(c), what)
        a = arrs[lk].reshape(-1)
        buf[o:o + a.size] = a
    return buf


def test_system_fit_matches_oracle(gpu_lib, system_case):
    links, X, orc, _ = system_case
    announce("system fit 3 BS x 2 UE")
    plan = gpu_lib.Plan(system_descs(J, K, NR, NT, NSC, GS, M, N, P, NS), iters=ITERS)
    res = plan.fit(dev_c64(_pack(plan, links, X, "x")))
    _, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"])
    xh = host(xh)
    A = host(res["A"])
    Bm = host(res["B"])
    assert np.all(host(res["status"]) == 0)
    err2 = tot2 = 0.0
    nm_g = nm_o = 0.0
    for c, (u, k) in enumerate(links):
        o = plan.offsets(c)
        Xh = unpack(plan, c, xh, "x")
        _, Xh_o = tucker.reconstruct(orc["A"][u], orc["B"][k], orc["C"][(u, k)],
                                     orc["G"][(u, k)], GS)
        err2 += np.sum(np.abs(Xh - Xh_o) ** 2)
        tot2 += np.sum(np.abs(X[(u, k)]) ** 2)
        nm_g += np.sum(np.abs(X[(u, k)] - Xh) ** 2)
        nm_o += np.sum(np.abs(X[(u, k)] - Xh_o) ** 2)
        # the shared factors are the same in every channel that shares them
        Au = unpack(plan, c, A, "a")
        Bk = unpack(plan, c, Bm, "b")
        c_ref = links.index((u, 0))
        assert np.array_equal(Au, unpack(plan, c_ref, A, "a")), (u, k)
        c_refb = links.index((0, k))
        assert np.array_equal(Bk, unpack(plan, c_refb, Bm, "b")), (u, k)
        assert np.abs(Au.conj().T @ Au - np.eye(M)).max() < 1e-5
        assert np.abs(Bk.conj().T @ Bk - np.eye(N)).max() < 1e-5
    rel = np.sqrt(err2 / tot2)
    nm_g, nm_o = nm_g / tot2, nm_o / tot2
    print(f"[system fit] X-hat {rel:.3e} of ||X||; NMSE {nm_g:.6e} vs oracle {nm_o:.6e}", flush=True)
    assert rel <= 1e-4, rel
    assert abs(nm_g - nm_o) <= 1e-5 * nm_o + 1e-10


@pytest.mark.parametrize("mode", ["none", "paper", "all"])
def test_system_sinr_of_oracle_factors(gpu_lib, system_case, mode):
    # the oracle's compressed system through the GPU's system SINR
    links, X, orc, Ht = system_case
    announce(f"system SINR of the oracle's factors, {mode}")
    plan = gpu_lib.Plan(system_descs(J, K, NR, NT, NSC, GS, M, N, P, NS), iters=ITERS)
    Cb = dev_c64(_pack(plan, links, orc["C"], "c"))
    Gb = dev_c64(_pack(plan, links, orc["G"], "g"))
    s2 = synthgen.snr_to_sigma2(SNRS)
    st = torch.zeros(plan.n_channels, dtype=torch.int32, device="cuda")
    out = host(plan.sinr_system(Cb, Gb, s2, mode=mode, status=st))
    ref = mc.sinr_system(Ht, J, K, s2, NS, mode)
    worst = 0.0
    for c, (u, k) in enumerate(links):
        o = plan.offsets(c)
        got = out[:, o.sc:o.sc + NSC, :NS]
        if u // K == k:
            err = np.abs(db(got) - db(ref[u])).max()
            worst = max(worst, err)
        else:
            assert np.all(got == 0), (u, k)
    print(f"[system sinr] {mode}: max error {worst:.3e} dB", flush=True)
    assert worst <= 0.05, worst
    assert np.all(host(st) & ~8 == 0)


@pytest.mark.parametrize("mode", ["paper", "all"])
def test_system_fit_and_sinr_against_oracle(gpu_lib, system_case, mode):
    # the whole path: the GPU fit with sharing, then the system SINR, against the oracle's
    links, X, orc, Ht = system_case
    announce(f"system fit + SINR, {mode}")
    plan = gpu_lib.Plan(system_descs(J, K, NR, NT, NSC, GS, M, N, P, NS), iters=ITERS)
    res = plan.fit(dev_c64(_pack(plan, links, X, "x")))
    s2 = synthgen.snr_to_sigma2(SNRS)
    out = host(plan.sinr_system(res["C"], res["G"], s2, mode=mode))
    ref = mc.sinr_system(Ht, J, K, s2, NS, mode)
    worst = 0.0
    for c, (u, k) in enumerate(links):
        if u // K != k:
            continue
        o = plan.offsets(c)
        worst = max(worst, np.abs(db(out[:, o.sc:o.sc + NSC, :NS]) - db(ref[u])).max())
    print(f"[system fit + sinr] {mode}: max error {worst:.3e} dB", flush=True)
    assert worst <= 0.05, worst


def test_system_without_sharing_is_per_channel(gpu_lib):
    # labels 0 (no sharing): every channel keeps its own factors, as in a batch of single links
    announce("no-sharing plan equals the single-link fits")
    rng = np.random.default_rng(93)
    Xs = [crandn(rng, 24, 4, 16) * (0.6 ** np.arange(4))[None, :, None] for _ in range(2)]
    d = dict(nr=4, nt=16, nsc=24, group_size=8, m=2, n=4, p=3, ns=2)
    plan = gpu_lib.Plan([d, d], iters=3)
    res = plan.fit(dev_c64(np.concatenate([x.reshape(-1) for x in Xs])))
    for c, X in enumerate(Xs):
        orc = tucker.fit(X, 8, 2, 4, 3, 3)
        _, Xh_o = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"], 8)
        _, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"])
        Xh = unpack(plan, c, host(xh), "x")
        assert np.linalg.norm(Xh - Xh_o) <= 1e-4 * np.linalg.norm(X)
