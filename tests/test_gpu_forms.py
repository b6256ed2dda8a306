"""The batched and differentiation forms on the GPU: graph capture and replay of a whole fit +
SINR evaluation, and SINR-aware refinement of the cores through the hand-written adjoint."""

import numpy as np
import pytest
import torch

import synthgen
from oracle import grad as ograd, sinr as osinr, tucker
from tests.gpu_util import announce, desc, dev_c64, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("split", [1, 2])
def test_fit_and_sinr_graph_replay(gpu_lib, split):
    # eight 8 x 64 x 3276 channels (a batch the fit splits over concurrent streams, in both split
    # modes): eager run, then a captured graph replayed three times with eager work in between;
    # every replay must reproduce the eager outputs bit for bit
    cfg = synthgen.CONFIGS["rb273"]
    announce(f"graph capture fit + sinr, 8 x rb273, split mode {split}")
    X = torch.cat([dev_c64(synthgen.make_channel(cfg, c)) for c in range(8)])
    plan = gpu_lib.Plan([gpu_lib.desc_from_config(cfg)] * 8, iters=cfg.iters)
    plan.set_tuning(split=split)
    s2 = [float(v) for v in synthgen.snr_to_sigma2(cfg.snr_db)]
    f_eager = plan.empty_factors()
    r = plan.fit(X, factors=f_eager, trace=False)
    sg_eager = plan.sinr(r["C"], r["G"], s2).clone()
    eager = {k: v.clone() for k, v in r.items()}
    torch.cuda.synchronize()

    f_graph = plan.empty_factors()
    sg_out = torch.empty_like(sg_eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        plan.fit(X, factors=f_graph, trace=False)
        plan.sinr(f_graph["C"], f_graph["G"], s2, out=sg_out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rg = plan.fit(X, factors=f_graph, trace=False)
        plan.sinr(f_graph["C"], f_graph["G"], s2, out=sg_out)
    for rep in range(3):
        for v in f_graph.values():
            v.zero_()
        sg_out.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k in ("A", "B", "C", "G"):
            assert torch.equal(f_graph[k], eager[k]), (rep, k)
        assert torch.equal(rg["status"], eager["status"])
        assert torch.equal(sg_out, sg_eager), rep
        # unrelated eager work between replays
        plan.reconstruct(eager["A"], eager["B"], eager["C"], eager["G"])
        torch.cuda.synchronize()


def test_sinr_aware_refinement(gpu_lib):
    # 8 x 128 channel with 32 paths compressed at mode-2 rank 24 (lossy): refine (C, G) with
    # Adam on the squared dB error of the compressed SINR against the full-channel SINR; the
    # gradient comes from the library's adjoint through SinrFn
    announce("sinr-aware refinement 8 x 128 x 96")
    rng = np.random.default_rng(61)
    nr, nt, nsc, L = 8, 128, 96, 32
    X = synthgen.build_channel(synthgen.draw_paths(rng, L, 3.0), nr, nt, nsc)
    gs, m, n, p, ns = 12, 8, 24, 12, 4
    s2 = [0.1]
    orc = tucker.fit(X, gs, m, n, p, 10)
    target = torch.tensor(10.0 * np.log10(osinr.sinr(X, s2, ns)), dtype=torch.float32,
                          device="cuda")
    plan = gpu_lib.Plan([desc(nr, nt, nsc, gs, m, n, p, ns)], iters=10)
    Ct = dev_c64(orc["C"]).requires_grad_(True)
    Gt = dev_c64(orc["G"]).requires_grad_(True)
    # loss at the oracle's starting point, the same quantity in FP64 on the CPU
    y0 = ograd.sinr_compressed_t(torch.tensor(orc["C"]), torch.tensor(orc["G"]), gs, s2, ns)
    loss0_ref = float(((10 * torch.log10(y0) - target.double().cpu()) ** 2).mean())
    opt = torch.optim.Adam([Ct, Gt], lr=3e-3)
    losses = []
    for it in range(50):
        y = gpu_lib.SinrFn.apply(plan, Ct, Gt, s2)[:, :, :ns]
        loss = ((10 * torch.log10(y) - target) ** 2).mean()
        losses.append(float(loss.detach()))
        opt.zero_grad()
        loss.backward()
        opt.step()
    assert abs(losses[0] - loss0_ref) <= 1e-3 * loss0_ref + 1e-7, (losses[0], loss0_ref)
    assert losses[-1] < 0.1 * losses[0], losses[::10]
    y = host(gpu_lib.SinrFn.apply(plan, Ct, Gt, s2)[:, :, :ns].detach())
    err = np.abs(10 * np.log10(y) - host(target))
    assert err.max() < 0.1, err.max()


def test_heterogeneous_batch(gpu_lib):
    # 48 channels of uneven antenna counts (4..16 x 32..256), subcarrier counts (624..3276),
    # group sizes (12, 24) and ranks in one plan: properties on every channel, FP64 oracle
    # parity on the three smallest
    announce("heterogeneous batch of 48 channels")
    specs = synthgen.heterogeneous_batch(48)
    iters = 6
    descs = [dict(nr=d["nr"], nt=d["nt"], nsc=d["nsc"], group_size=d["group_size"], m=d["m"],
                  n=d["n"], p=d["p"], ns=d["ns"]) for d in specs]
    X = torch.cat([synthgen.build_channel_torch(d["paths"], d["nr"], d["nt"], d["nsc"],
                                                torch.device("cuda"),
                                                dtype=torch.complex64).reshape(-1)
                   for d in specs])
    plan = gpu_lib.Plan(descs, iters=iters)
    res = plan.fit(X)
    _, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"], ht=False)
    torch.cuda.synchronize()
    assert np.all(host(res["status"]) == 0)
    tr = host(res["trace"])
    Xh_all = host(xh)
    X_all = host(X)
    sizes = []
    for c, d in enumerate(descs):
        o = plan.offsets(c)
        nx = d["nsc"] * d["nr"] * d["nt"]
        Xc = X_all[o.x:o.x + nx].astype(np.complex128)
        Xhc = Xh_all[o.x:o.x + nx].astype(np.complex128)
        n2 = float(np.sum(np.abs(Xc) ** 2))
        A = host(res["A"])[o.a:o.a + d["nr"] * d["m"]].reshape(d["nr"], d["m"])
        Bm = host(res["B"])[o.b:o.b + d["nt"] * d["n"]].reshape(d["nt"], d["n"])
        assert np.abs(A.conj().T @ A - np.eye(d["m"])).max() < 1e-4, c
        assert np.abs(Bm.conj().T @ Bm - np.eye(d["n"])).max() < 1e-4, c
        assert np.all(np.diff(tr[c]) <= 1e-5 * n2), (c, np.diff(tr[c]).max() / n2)
        resid = float(np.sum(np.abs(Xc - Xhc) ** 2))
        assert abs(resid - tr[c, -1]) <= 1e-5 * n2, (c, resid / n2, tr[c, -1] / n2)
        sizes.append((nx, c))
    for _, c in sorted(sizes)[:3]:
        d = specs[c]
        Xo = synthgen.build_channel(d["paths"], d["nr"], d["nt"], d["nsc"])
        orc = tucker.fit(Xo, d["group_size"], d["m"], d["n"], d["p"], iters)
        n2 = float(np.sum(np.abs(Xo) ** 2))
        assert np.abs(tr[c] - orc["trace"]).max() <= 1e-5 * n2, c


@pytest.mark.parametrize("split,trace", [(1, True), (2, True), (2, False)])
def test_split_batch_matches_single_channel_fits(gpu_lib, split, trace):
    # a batch of 16 channels runs as four parts on concurrent streams (B-step over the batch, or
    # pipelined parts); every channel's factors, cores, objective trace and status must equal
    # those of a plan holding that channel alone.  Untraced, the pipelined parts make the
    # starting mode-2 factor on the last part's stream while the first B-steps run.
    announce(f"split batch of 16 vs single-channel plans, split mode {split}, trace {trace}")
    rng = np.random.default_rng(91)
    nr, nt, nsc = 8, 64, 240
    Xs = [synthgen.build_channel(synthgen.draw_paths(rng, 8, 6.0), nr, nt, nsc) for _ in range(16)]
    d = desc(nr, nt, nsc, 12, 8, 16, 12, 4)
    plan = gpu_lib.Plan([d] * 16, iters=8)
    plan.set_tuning(split=split)
    res = plan.fit(torch.cat([dev_c64(x) for x in Xs]), trace=trace)
    torch.cuda.synchronize()
    for c, x in enumerate(Xs):
        one = gpu_lib.Plan([d], iters=8).fit(dev_c64(x), trace=trace)
        torch.cuda.synchronize()
        o = plan.offsets(c)
        for k, off, size in (("A", o.a, nr * 8), ("B", o.b, nt * 16), ("C", o.c, nsc * 12),
                             ("G", o.g, one["G"].numel())):
            assert torch.equal(res[k][off:off + size], one[k]), (c, k)
        if trace:
            assert torch.equal(res["trace"][c], one["trace"][0]), c
        assert int(res["status"][c].item()) == 0 and int(one["status"][0].item()) == 0


def test_autotune_keeps_a_valid_fit(gpu_lib):
    # the autotuner times the pass variants on 16 rb273-shaped channels (fused passes, split
    # batch); every variant it may keep must give the same fit up to FP32 rounding: the tuned
    # plan's factors reconstruct X as well as the default plan's, the objective traces agree
    announce("autotune 16 channels")
    rng = np.random.default_rng(93)
    nr, nt, nsc = 8, 64, 480
    Xs = [synthgen.build_channel(synthgen.draw_paths(rng, 8, 6.0), nr, nt, nsc) for _ in range(16)]
    X = torch.cat([dev_c64(x) for x in Xs])
    d = desc(nr, nt, nsc, 12, 8, 16, 12, 4)
    ref = gpu_lib.Plan([d] * 16, iters=6)
    r0 = ref.fit(X)
    tuned = gpu_lib.Plan([d] * 16, iters=6)
    choice = tuned.autotune(X)
    print(f"[autotune] {choice}")
    assert choice["probe_ms"] > 0
    r1 = tuned.fit(X)
    torch.cuda.synchronize()
    assert np.all(host(r1["status"]) == 0)
    tr0, tr1 = host(r0["trace"]), host(r1["trace"])
    for c, x in enumerate(Xs):
        nx = float(np.sum(np.abs(x) ** 2))
        assert np.abs(tr0[c] - tr1[c]).max() <= 1e-5 * nx, c
    # every variant in turn gives the reference fit up to rounding
    for bstep in (0, 1, 2):
        for tpass in (0, 1):
            for split in (0, 1, 2):
                p = gpu_lib.Plan([d] * 16, iters=6)
                p.set_tuning(bstep=bstep, tpass=tpass, split=split)
                r = p.fit(X)
                torch.cuda.synchronize()
                assert np.all(host(r["status"]) == 0), (bstep, tpass, split)
                tr = host(r["trace"])
                for c, x in enumerate(Xs):
                    nx = float(np.sum(np.abs(x) ** 2))
                    assert np.abs(tr0[c] - tr[c]).max() <= 1e-5 * nx, (bstep, tpass, split, c)
