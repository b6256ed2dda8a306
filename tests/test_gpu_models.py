"""The paper's three compression models on a synthetic multi-cell system (Section 4 and its
table of compression results): Individual (every link its own A and B, model "Tucker
decomposition"), Shared (one A and one B for every link, model "MT1") and Groupwise (A per
UE, B per base station, model "MT_origin"), each a labelling of the same plan layout.  The
mean relative SINR error e_c of equation "SINR error" (compressed against uncompressed
channels, the paper's inter-cell protocol) from the GPU's fits and SINRs is checked against
the e_c of the FP64 oracle's fits and SINRs.

The uncompressed SINR runs on the same system kernels through the exact representation
(groups of one subcarrier, p = 1, m = nr, n = nt, C = 1, G = X).  The Individual model's
factors do not cancel in the interference terms (each link has its own B), so its SINR is
evaluated on the reconstructed channels, as the paper's time ratio for that model implies.

Bar: |e_c(GPU) - e_c(oracle)| <= 2 % of e_c(oracle) + 1e-5 (each SINR agrees to 0.05 dB, about
1.2 % relative, and e_c averages relative errors of about 10 %).
"""

import numpy as np
import pytest
import torch

import synthgen
from oracle import metrics, multicell as mc, tucker
from tests.gpu_util import announce, crandn, dev_c64, host, unpack

pytestmark = pytest.mark.gpu

J, K = 3, 2
NR, NT, NSC, GS, M, N, P, NS, ITERS = 8, 32, 40, 12, 4, 8, 6, 2, 6
S2 = [0.1]  # 10 dB
LINKS = synthgen.system_links(J, K)


def labels(model, u, k):
    if model == "individual":
        return 0, 0
    if model == "shared":
        return 1, 1
    return u + 1, k + 1


def fit_descs(model):
    out = []
    for u, k in LINKS:
        a, b = labels(model, u, k)
        out.append(dict(nr=NR, nt=NT, nsc=NSC, group_size=GS, m=M, n=N, p=P, ns=NS, a_id=a, b_id=b))
    return out


def system_descs(m=M, n=N, gs=GS, p=P):
    return [dict(nr=NR, nt=NT, nsc=NSC, group_size=gs, m=m, n=n, p=p, ns=NS, a_id=u + 1,
                 b_id=k + 1, serving=int(u // K == k)) for u, k in LINKS]


def exact_descs():
    return system_descs(m=NR, n=NT, gs=1, p=1)


@pytest.fixture(scope="module")
def models_case():
    rng = np.random.default_rng(97)
    X = {lk: crandn(rng, NSC, NR, NT) * (0.7 ** np.arange(NR))[None, :, None]
         * (0.9 ** np.arange(NT))[None, None, :] for lk in LINKS}
    full = mc.sinr_system(X, J, K, S2, NS, "paper")
    orc = {}
    for model in ("individual", "shared", "groupwise"):
        if model == "individual":
            a_of = b_of = (lambda lk: lk)
        elif model == "shared":
            a_of = b_of = (lambda lk: 0)
        else:
            a_of, b_of = None, None
        r = mc.fit(X, GS, M, N, P, ITERS, a_of=a_of, b_of=b_of)
        if model == "individual":
            Xh = {lk: tucker.reconstruct(r["A"][lk], r["B"][lk], r["C"][lk], r["G"][lk], GS)[1]
                  for lk in LINKS}
            comp = mc.sinr_system(Xh, J, K, S2, NS, "paper")
        else:
            Ht = {lk: tucker.compressed_channels(r["C"][lk], r["G"][lk], GS) for lk in LINKS}
            comp = mc.sinr_system(Ht, J, K, S2, NS, "paper")
        orc[model] = np.mean([np.abs((full[u] - comp[u]) / full[u]).mean() for u in full])
    return X, orc


def _packed(plan, arrs, what):
    buf = np.zeros(getattr(plan.totals, what), np.complex128)
    for c, lk in enumerate(LINKS):
        o = getattr(plan.offsets(c), what)
        a = arrs[lk].reshape(-1)
        buf[o:o + a.size] = a
    return buf


def _ue_values(plan, out):
    vals = {}
    for c, (u, k) in enumerate(LINKS):
        if u // K == k:
            o = plan.offsets(c)
            vals[u] = out[:, o.sc:o.sc + NSC, :NS].astype(np.float64)
    return vals


@pytest.mark.parametrize("model", ["individual", "shared", "groupwise"])
def test_model_sinr_error_matches_oracle(gpu_lib, models_case, model):
    X, orc = models_case
    announce(f"compression model {model}: e_c against the oracle")
    exact = gpu_lib.Plan(exact_descs(), iters=1)
    Xb = dev_c64(_packed(exact, X, "x"))
    ones = torch.ones(exact.totals.c, dtype=torch.complex64, device="cuda")
    full = _ue_values(exact, host(exact.sinr_system(ones, Xb, S2, mode="paper")))
    fplan = gpu_lib.Plan(fit_descs(model), iters=ITERS)
    res = fplan.fit(Xb)
    assert np.all(host(res["status"]) == 0)
    if model == "individual":
        _, xh = fplan.reconstruct(res["A"], res["B"], res["C"], res["G"])
        comp = _ue_values(exact, host(exact.sinr_system(ones, xh, S2, mode="paper")))
    else:
        splan = gpu_lib.Plan(system_descs(), iters=1)
        comp = _ue_values(splan, host(splan.sinr_system(res["C"], res["G"], S2, mode="paper")))
    e_c = np.mean([np.abs((full[u] - comp[u]) / full[u]).mean() for u in full])
    print(f"[models] {model}: e_c GPU {e_c:.5f}, oracle {orc[model]:.5f}", flush=True)
    assert abs(e_c - orc[model]) <= 0.02 * orc[model] + 1e-5, (e_c, orc[model])


@pytest.mark.parametrize("ranks", [(4, 4, 3), (4, 16, 6), (8, 32, 12)])
def test_rank_sweep_point_matches_oracle(gpu_lib, models_case, ranks):
    # one point of the rank sweep of the groupwise model (Section 4, the figure that varies
    # the mode-2 and mode-3 ranks): the storage ratio R_s of equation "compression ratio" for
    # this system and the e_c of the GPU's fit and SINR against the oracle's
    X, _ = models_case
    m, n, p = ranks
    announce(f"rank sweep point {ranks}")
    full = mc.sinr_system(X, J, K, S2, NS, "paper")
    r = mc.fit(X, GS, m, n, p, ITERS)
    Ht = {lk: tucker.compressed_channels(r["C"][lk], r["G"][lk], GS) for lk in LINKS}
    comp = mc.sinr_system(Ht, J, K, S2, NS, "paper")
    e_orc = np.mean([np.abs((full[u] - comp[u]) / full[u]).mean() for u in full])
    descs = system_descs(m=m, n=n, p=p)
    plan = gpu_lib.Plan(descs, iters=ITERS)
    res = plan.fit(dev_c64(_packed(plan, X, "x")))
    got = _ue_values(plan, host(plan.sinr_system(res["C"], res["G"], S2, mode="paper")))
    e_gpu = np.mean([np.abs((full[u] - got[u]) / full[u]).mean() for u in full])
    rs = mc.storage_ratio_system(J, K, NR, NT, NSC, GS, m, n, p)
    print(f"[rank sweep] (m, n, p) = {ranks}: R_s {rs:.3f}, e_c GPU {e_gpu:.5f}, "
          f"oracle {e_orc:.5f}", flush=True)
    assert abs(e_gpu - e_orc) <= 0.02 * e_orc + 1e-5, (e_gpu, e_orc)
