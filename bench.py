"""Benchmark of the groupwise Tucker hot path on one MI355X.

Workload: channels of 8 receive x 64 transmit antennas x 3276 subcarriers (273 resource
blocks of 12), 8 paths (LOS at K = 6 dB), groups of 12 subcarriers, Tucker ranks (8, 16, 12),
20 alternating sweeps, 4 SVD-precoded streams, SNR in {-5, 0, 10, 20} dB.  Synthetic seeded
channels (the paper's 3GPP TR 38.901 data is not available).

One step = one pass of the whole path over a batch of channels resident in HBM:
    fit (HOSVD init + 20 sweeps + cores)  ->  compressed channels Ht  ->
    per-subcarrier SINR at 4 SNRs  ->  adjoint of the SINR with respect to (C, G).
Prints one JSON line.  `value` is Tucker fits/s of the whole step; the SINR-evaluation
rate of the SINR kernel is reported beside it.

The headline steps run with the library's kernel timing off; a second pass of the same steps
brackets every kernel with HIP events on its own stream for the per-kernel durations behind
the rooflines (the B-step on FP32 matrix cores, the SINR kernel on the vector ALU and in HBM
bytes, reconstruction in HBM bytes).  The line also carries the single-channel latency, a
256-channel batch, the oracle on the host (all BLAS threads and one thread) and, unless
`--no-forms`, the precision, graph-replay, differentiation and heterogeneous-batch forms.

`--workload wide` times the same step on channels of 16 x 256 x 3276 (16 paths, K = 3 dB,
ranks (12, 32, 12), 8 streams at 10 dB), 8 channels per step, for the profiles of the
wide-array passes; the default run is the workload above.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# vector ALU without packed FP32 instructions (disabled in this build): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops per FMA x 2.4 GHz
PEAK_VALU_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# algorithmic work per unit of each timed kernel: CMAC = 8 real flops
CMAC = 8.0


def sweep_cmacs(nr, nt, nsc, gs, m, n, p):
    """Complex multiply-adds of one alternating sweep in the kernels' matrix form (A, B and
    C steps), counting Hermitian Grams once per unordered pair.  With m == nr the mode-1
    factor is square and unitary (A A^H = I): the B- and C-step Grams need no product with A
    (t_b, t_c below), and only the last sweep's A-step affects the result."""
    ng = -(-nsc // gs)
    t_a = nsc * nr * nt * n + ng * p * gs * nr * n + ng * p * nr * nr * n / 2
    if m == nr:
        t_b = ng * p * gs * nr * nt + ng * p * m * nt * nt / 2
        t_c = nsc * nr * nt * n + ng * gs * gs * nr * n / 2
    else:
        t_b = nsc * m * nr * nt + ng * p * gs * m * nt + ng * p * m * nt * nt / 2
        t_c = nsc * m * nt * n + ng * gs * gs * m * n / 2
    return t_a, t_b, t_c


def fit_cmacs(nr, nt, nsc, gs, m, n, p, iters):
    """Complex multiply-adds of a whole fit's sweeps (one A-step when m == nr)."""
    t_a, t_b, t_c = sweep_cmacs(nr, nt, nsc, gs, m, n, p)
    return iters * (t_b + t_c) + (1 if m == nr else iters) * t_a


def gram_rows_flops(ng, p, m, nt):
    """Algorithmic flops of the mode-2 Gram S2 = sum over rows of W^H W (Hermitian half)."""
    return CMAC * ng * p * m * nt * nt / 2


def bstep_group_cmacs(nr, nt, gs, m, p):
    """Complex MACs of one group's B-step: Hc_q = sum_s conj(C[s,q]) H_s (p gs nr nt), W_q =
    A^H Hc_q (p m nr nt; none when m == nr, where A A^H = I and the Gram of Hc is the Gram of
    W) and the Hermitian Gram sum_q W_q^H W_q (p m nt^2 / 2)."""
    return p * gs * nr * nt + (0 if m == nr else p * m * nr * nt) + p * m * nt * nt / 2


def sinr_unit_flops(m, n, p, ns, n_snr):
    """Flops of one (subcarrier, SNR) SINR evaluation from the compressed form: Ht (m n p),
    its Gram (m^2 n / 2) amortised over the SNRs, then the MMSE chain.  With ns < m the chain
    runs in the ns x ns push-through form: M = HV^H HV (m ns^2 / 2) once per subcarrier, and per
    SNR the Cholesky of M + s2 I (ns^3 / 6) and, per stream, two triangular solves and z = M y
    (2 ns^2).  With ns = m it is the m x m chain: the covariance (m^2 ns / 2), Cholesky
    (m^3 / 6), two triangular solves (m^2 ns) and the stream products (m ns^2 + m ns).
    Iterative eigensolver sweeps are excluded."""
    per_sub = m * n * p + m * m * n / 2
    if ns < m:
        per_sub += m * ns * ns / 2
        per_snr = ns ** 3 / 6 + 2 * ns ** 3
    else:
        per_snr = m * m * ns / 2 + m ** 3 / 6 + m * m * ns + m * ns * ns + m * ns
    return CMAC * (per_sub / n_snr + per_snr)


def sinr_unit_bytes(m, n, p, gs, n_snr, ns):
    """HBM bytes per (subcarrier, SNR): the group's core read once per group, the C row, the
    SINR output."""
    return (8 * m * n * p / gs + 8 * p) / n_snr + 4 * ns


def measured_traffic(kernel: str, workload: str = "rb273"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy of known size), or None when the
    summary is absent or was taken on a different revision of the kernel's source file."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and not ln.startswith(" "):
                k, v = ln.split(":", 1)
                fields[k.strip()] = v.strip()
    src = fields.get("source")
    if not src or "traffic_bytes_per_launch" not in fields:
        return None
    # one or more source files (comma-separated) with their hashes in the same order
    files = [f.strip() for f in src.split(",")]
    hashes = [h.strip() for h in fields.get("source_sha256", "").split(",")]
    if len(files) != len(hashes):
        return None
    for f, h in zip(files, hashes):
        with open(os.path.join(ROOT, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != h:
                return None
    return float(fields["traffic_bytes_per_launch"])


KERNEL_NAMES = [
    "k_eigA", "k_eigB", "k_eigC", "k_eigA_rows", "k_eigC_rows", "k_gram_rows", "k_reduce_S1", "k_reduce_S2", "k_reduce_S2_mfma",
    "k_init_group", "k_init_group_lds", "k_stepA_group", "k_S3", "k_core", "k_objC", "k_trace",
    "k_norm_total", "k_fused_t", "k_fused_t_mfma", "k_fused_z", "k_fused_b", "k_fused_b_mfma",
    "k_fused_b_mm", "k_eigB_sub", "k_sub_prod", "k_sub_rr", "k_sub_rot", "k_rows_times_b",
    "k_w_rows", "k_yh_from_t", "k_gram_rows_st", "k_reduce_S2_st", "k_reconstruct",
    "k_reconstruct_ht", "k_sinr_rows", "k_sinr_lane", "k_sinr", "k_sinr_bwd_rows",
    "k_sinr_bwd_lane", "k_sinr_bwd", "k_sinr_bwd_reduce"]


def profile_steps(api, fn, steps):
    """Runs fn `steps` times with every library kernel bracketed by HIP events on its own
    stream; returns per-kernel totals per step, launches per step and average durations."""
    import torch

    torch.cuda.synchronize()
    api.profile_enable(True)
    api.profile_reset()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    kern = {}
    for nm in KERNEL_NAMES:
        ms, cnt = api.profile_query(nm)
        if cnt:
            kern[nm] = dict(total_ms=ms / steps, launches=cnt // steps, avg_us=1e3 * ms / cnt)
    api.profile_enable(False)
    api.profile_reset()
    return kern


def _channels(synthgen, cfg, count, dev, torch):
    xs = []
    for c in range(count):
        pp = synthgen.draw_paths(synthgen.channel_rng(cfg.seed_index, c), cfg.n_paths, cfg.k_db)
        xs.append(synthgen.build_channel_torch(pp, cfg.nr, cfg.nt, cfg.nsc, dev,
                                               dtype=torch.complex64).reshape(-1))
    return torch.cat(xs)


def single_channel_latency(api, synthgen, cfg, s2, dev, torch, reps=10):
    """Latency of one channel through the whole step (fit, Ht, SINR, adjoint), median of reps."""
    X = _channels(synthgen, cfg, 1, dev, torch)
    plan = api.Plan([api.desc_from_config(cfg)], iters=cfg.iters)
    f = plan.empty_factors()
    gs = torch.full((len(s2), plan.totals.sc, plan.ns_max), 1.0e-3, dtype=torch.float32, device=dev)

    def one():
        r = plan.fit(X, factors=f, trace=False)
        plan.reconstruct(r["A"], r["B"], r["C"], r["G"], ht=True, xhat=False)
        plan.sinr(r["C"], r["G"], s2)
        plan.sinr_backward(r["C"], r["G"], s2, gs)

    one()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        one()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return dict(ms=times[len(times) // 2], ms_min=times[0], reps=reps,
                what="one 8x64x3276 channel: fit + Ht + SINR at 4 SNRs + SINR adjoint")


def batch_throughput(api, synthgen, cfg, s2, dev, torch, count, steps=3):
    """The same step over `count` seeded channels (fits/s)."""
    X = _channels(synthgen, cfg, count, dev, torch)
    plan = api.Plan([api.desc_from_config(cfg)] * count, iters=cfg.iters)
    f = plan.empty_factors()
    gs = torch.full((len(s2), plan.totals.sc, plan.ns_max), 1.0e-3, dtype=torch.float32, device=dev)

    def one():
        r = plan.fit(X, factors=f, trace=False)
        plan.reconstruct(r["A"], r["B"], r["C"], r["G"], ht=True, xhat=False)
        plan.sinr(r["C"], r["G"], s2)
        plan.sinr_backward(r["C"], r["G"], s2, gs)

    one()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        one()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del X, plan, f
    return dict(channels=count, ms_per_step=ms, fits_per_s=count / (ms / 1e3),
                sinr_evals_per_s_step=count * cfg.nsc * len(s2) / (ms / 1e3))


def host_description():
    """nproc and the CPU model of the host the oracle runs on."""
    desc = dict(nproc=os.cpu_count())
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket",
                             "Socket(s)"):
                desc[k.strip()] = v.strip()
    except Exception:  # lscpu missing: nproc alone
        pass
    return desc


def copy_calibration(mib: int) -> None:
    """Plain device copy of a known size, the reference for scaling HBM byte counters."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 3}))


def time_models(api, synthgen, torch, dev, reps=5):
    """The paper's three compression models on a synthetic multi-cell system (the layout of its
    table of compression results): 3 base stations with 2 UEs each, links of 8 x 64 x 624
    (8 paths, K 6 dB), groups of 12, ranks (8, 16, 6), 20 sweeps, 2 streams at 10 dB with the
    paper's inter-cell protocol.  Per model: R_s (equation "compression ratio" for this
    structure), R_t = SINR time of the uncompressed channels / SINR time from the compressed form
    (both on this GPU; the Individual model's factors do not cancel, so its SINR runs on the
    reconstructed channels), e_c (equation "SINR error"); then a rank sweep of the groupwise
    model (R_s and e_c against n and p)."""
    import numpy as np

    J, K, nr, nt, nsc, gs = 3, 2, 8, 64, 624, 12
    m, n, p, ns, iters = 8, 16, 6, 2, 20
    s2 = [0.1]
    links = synthgen.system_links(J, K)
    Xs = synthgen.make_system(J, K, nr, nt, nsc, 8, 6.0)

    def descs(mm, nn, gg, pp, model):
        out = []
        for u, k in links:
            if model == "individual":
                a, b = 0, 0
            elif model == "shared":
                a, b = 1, 1
            else:
                a, b = u + 1, k + 1
            out.append(dict(nr=nr, nt=nt, nsc=nsc, group_size=gg, m=mm, n=nn, p=pp, ns=ns, a_id=a,
                            b_id=b, serving=int(u // K == k and model == "groupwise")))
        return out

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[len(ts) // 2], out

    def ue_values(plan, out):
        o = out.cpu().numpy()
        vals = []
        for c, (u, k) in enumerate(links):
            if u // K == k:
                sc = plan.offsets(c).sc
                vals.append(o[:, sc:sc + nsc, :ns].astype(np.float64))
        return np.stack(vals)

    exact = api.Plan(descs(nr, nt, 1, 1, "groupwise"), iters=1)
    X = torch.cat([torch.as_tensor(Xs[lk].reshape(-1), dtype=torch.complex64) for lk in links]).to(dev)
    ones = torch.ones(exact.totals.c, dtype=torch.complex64, device=dev)
    ms_full, out_full = timed(lambda: exact.sinr_system(ones, X, s2, mode="paper"))
    full = ue_values(exact, out_full)
    sysplan = api.Plan(descs(m, n, gs, p, "groupwise"), iters=iters)
    ng = -(-nsc // gs)
    per_link = sum(m * n * min(p, min(gs, nsc - g * gs)) + min(gs, nsc - g * gs) * min(p, gs)
                   for g in range(ng))
    orig = J * J * K * nr * nt * nsc
    stored = {"individual": J * J * K * (per_link + nr * m + nt * n),
              "shared": J * J * K * per_link + nr * m + nt * n,
              "groupwise": J * J * K * per_link + J * K * nr * m + J * nt * n}
    res = {}
    for model in ("individual", "shared", "groupwise"):
        fplan = api.Plan(descs(m, n, gs, p, model), iters=iters)
        f = fplan.empty_factors()
        ms_fit, r = timed(lambda: fplan.fit(X, factors=f, trace=False))
        if model == "individual":
            def comp_fn():
                _, xh = fplan.reconstruct(f["A"], f["B"], f["C"], f["G"], ht=False, xhat=True)
                return exact.sinr_system(ones, xh, s2, mode="paper")
            ms_sinr, out = timed(comp_fn)
            comp = ue_values(exact, out)
        else:
            ms_sinr, out = timed(lambda: sysplan.sinr_system(f["C"], f["G"], s2, mode="paper"))
            comp = ue_values(sysplan, out)
        res[model] = dict(R_s=orig / stored[model], R_t=ms_full / ms_sinr,
                          e_c=float(np.mean(np.abs((full - comp) / full))),
                          ms_fit=ms_fit, ms_sinr=ms_sinr, status_ok=bool((r["status"] == 0).all()))
        del fplan, f
    sweep = []
    for nn, pp in ((4, 3), (8, 3), (8, 6), (16, 6), (16, 12), (32, 12)):
        plan = api.Plan(descs(m, nn, gs, pp, "groupwise"), iters=iters)
        f = plan.empty_factors()
        plan.fit(X, factors=f, trace=False)
        comp = ue_values(plan, plan.sinr_system(f["C"], f["G"], s2, mode="paper"))
        pl = sum(m * nn * min(pp, min(gs, nsc - g * gs)) + min(gs, nsc - g * gs) * min(pp, gs)
                 for g in range(ng))
        sweep.append(dict(m=m, n=nn, p=pp, R_s=orig / (J * J * K * pl + J * K * nr * m + J * nt * nn),
                          e_c=float(np.mean(np.abs((full - comp) / full)))))
        del plan, f
    return dict(workload="3 BS x 2 UE, 18 links of 8 x 64 x 624 (8 paths, K 6 dB), groups of 12, "
                         "ranks (8, 16, 6), 20 sweeps, Ns 2 at 10 dB, inter-cell from the first UE "
                         "of each other cell", ms_sinr_uncompressed=ms_full, models=res,
                rank_sweep_groupwise=sweep)


def time_submatrix(api, synthgen, torch, dev, reps=5):
    """The paper's 8 x 256 x 401 shape with mode 3 = path / delay submatrices (Section 2.2):
    8 channels of clustered rays (20 clusters x 20 rays + LOS, one submatrix per ray), groups of
    20 (one cluster each, the LOS alone), ranks (8, 48, 12), 10 sweeps, Ns 4 at 10 dB.  The
    channels are evaluated at 512 OFDM points (combining rows exp(-j 2 pi t tau_l / 512)):
    compressed = combine the factors (equation "compressed matrix SINR reduction") + the SINR
    chain on the m x n channels; full = combine the submatrices + the chain on the nr x nt
    channels.  R_t = full time / compressed time, e_c = mean relative SINR error of the
    compressed evaluation (equation "SINR error"), R_s = stored elements of X / of the
    factors and cores (equation "compression ratio" for one link)."""
    import numpy as np

    nch, nr, nt, gs, m, n, p, ns, iters, n_pts = 8, 8, 256, 20, 8, 48, 12, 4, 10, 512
    s2 = [float(v) for v in synthgen.snr_to_sigma2([10.0])]
    pps = [synthgen.draw_submatrix_paths(synthgen.channel_rng(12, c)) for c in range(nch)]
    X = torch.cat([torch.as_tensor(synthgen.build_submatrices(pp, nr, nt).reshape(-1),
                                   dtype=torch.complex64) for pp in pps]).to(dev)
    U = torch.cat([torch.as_tensor(synthgen.submatrix_weights(pp, n_pts, 512).reshape(-1),
                                   dtype=torch.complex64) for pp in pps]).to(dev)
    P = 20 * 20 + 1
    plan = api.Plan([dict(nr=nr, nt=nt, nsc=P, group_size=gs, m=m, n=n, p=p, ns=ns)] * nch,
                    iters=iters)
    f = plan.empty_factors()
    comp_plan = api.Plan(plan.combined_descs(n_pts, compressed=True), iters=0)
    full_plan = api.Plan(plan.combined_descs(n_pts, compressed=False), iters=0)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[len(ts) // 2], out

    ms_fit, r = timed(lambda: plan.fit(X, factors=f, trace=False))
    ms_comb_c, Ht = timed(lambda: plan.combine_compressed(f["C"], f["G"], U, n_pts))
    ms_comb_f, H = timed(lambda: plan.combine_full(X, U, n_pts))
    ms_sinr_c, sc = timed(lambda: comp_plan.sinr_full(Ht, s2))
    ms_sinr_f, sf = timed(lambda: full_plan.sinr_full(H, s2))
    a, b = sc.cpu().numpy().astype(np.float64), sf.cpu().numpy().astype(np.float64)
    live = (a > 0) & (b > 0)
    ng = -(-P // gs)
    stored = nr * m + nt * n + sum(min(gs, P - g * gs) * min(p, min(gs, P - g * gs))
                                   + m * n * min(p, min(gs, P - g * gs)) for g in range(ng))
    ms_c, ms_f = ms_comb_c + ms_sinr_c, ms_comb_f + ms_sinr_f
    return dict(
        workload="8 x (8 x 256 x 401) submatrix tensors (20 clusters x 20 rays + LOS), groups of "
                 "20, ranks (8, 48, 12), 10 sweeps, 512 OFDM points, Ns 4 at 10 dB",
        fits_per_s=nch / (ms_fit / 1e3), ms_fit=ms_fit,
        ms_compressed=ms_c, ms_combine_compressed=ms_comb_c, ms_sinr_compressed=ms_sinr_c,
        ms_full=ms_f, ms_combine_full=ms_comb_f, ms_sinr_full=ms_sinr_f,
        R_t=ms_f / ms_c, R_s=P * nr * nt / stored, e_c=float(np.mean(np.abs(a[live] - b[live]) / b[live])),
        evals_per_s_compressed=nch * n_pts / (ms_c / 1e3),
        status_ok=bool((r["status"] == 0).all()))


def time_forms(api, synthgen, cfg, X, B, s2, ms_fp32, sg_fp32, torch, steps):
    """The precision, batched (graph replay) and differentiation forms on the same GPU:
    throughput of fit + SINR (eager FP32 first, as the reference) and SINR error against the
    plain FP32 step's output."""
    import numpy as np

    forms = {}

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    def db_err(a, b):
        a = a[:, :cfg.nsc * B, :cfg.ns].cpu().numpy()
        b = b[:, :cfg.nsc * B, :cfg.ns].cpu().numpy()
        live = (a > 0) & (b > 0)
        return float(np.abs(10 * np.log10(a[live]) - 10 * np.log10(b[live])).max())

    for prec in ("fp32", "bf16", "fp16", "split_bf16"):
        plan = api.Plan([api.desc_from_config(cfg)] * B, iters=cfg.iters, ttm_prec=prec)
        f = plan.empty_factors()
        out = {}

        def step_p():
            r = plan.fit(X, factors=f, trace=False)
            out["sg"] = plan.sinr(r["C"], r["G"], s2)

        ms = timed(step_p, steps)
        forms[prec] = dict(fits_per_s=B / (ms / 1e3), ms_per_fit_batch=ms,
                           max_sinr_err_db_vs_fp32=db_err(out["sg"], sg_fp32))
        del plan, f
    # the FP32 fit + SINR after the autotuner has picked the pass variants on this batch
    plan = api.Plan([api.desc_from_config(cfg)] * B, iters=cfg.iters)
    choice = plan.autotune(X)
    f = plan.empty_factors()
    out = {}

    def step_t():
        r = plan.fit(X, factors=f, trace=False)
        out["sg"] = plan.sinr(r["C"], r["G"], s2)

    ms = timed(step_t, steps)
    forms["fp32_autotuned"] = dict(fits_per_s=B / (ms / 1e3), ms_per_fit_batch=ms,
                                   max_sinr_err_db_vs_fp32=db_err(out["sg"], sg_fp32),
                                   choice={k: v for k, v in choice.items() if k != "probe_ms"})
    del plan, f
    # batched form: the whole FP32 fit + SINR captured once and replayed
    plan = api.Plan([api.desc_from_config(cfg)] * B, iters=cfg.iters)
    f = plan.empty_factors()
    sg_out = torch.empty_like(sg_fp32)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.fit(X, factors=f, trace=False)
        plan.sinr(f["C"], f["G"], s2, out=sg_out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.fit(X, factors=f, trace=False)
        plan.sinr(f["C"], f["G"], s2, out=sg_out)
    ms = timed(g.replay, steps)
    forms["graph_replay_fp32"] = dict(fits_per_s=B / (ms / 1e3), ms_per_fit_batch=ms,
                                      max_sinr_err_db_vs_fp32=db_err(sg_out, sg_fp32))
    del g, plan, f
    # differentiation form: SINR-aware refinement steps of (C, G) on the 8 x 128 x 1632
    # workload (64 channels, ranks (8, 24, 12), 4 streams, 10 dB)
    gcfg = synthgen.CONFIGS["grad"]
    dev = torch.device("cuda:0")
    xs = []
    for c in range(gcfg.n_channels):
        pp = synthgen.draw_paths(synthgen.channel_rng(gcfg.seed_index, c), gcfg.n_paths, gcfg.k_db)
        xs.append(synthgen.build_channel_torch(pp, gcfg.nr, gcfg.nt, gcfg.nsc, dev,
                                               dtype=torch.complex64).reshape(-1))
    Xg = torch.cat(xs)
    del xs
    plan = api.Plan([api.desc_from_config(gcfg)] * gcfg.n_channels, iters=gcfg.iters)
    gs2 = [float(v) for v in synthgen.snr_to_sigma2(gcfg.snr_db)]
    fg = plan.empty_factors()
    ms_fit = timed(lambda: plan.fit(Xg, factors=fg, trace=False), 2)
    forms["fit_8x128x1632"] = dict(
        workload="64 x (8 x 128 x 1632), 32 paths, groups of 12, ranks (8, 24, 12), 20 sweeps",
        fits_per_s=gcfg.n_channels / (ms_fit / 1e3), ms_per_fit_batch=ms_fit)
    r = plan.fit(Xg, trace=False)
    target = 10 * torch.log10(plan.sinr_full(Xg, gs2).clamp_min(1e-30))
    Ct = r["C"].clone().requires_grad_(True)
    Gt = r["G"].clone().requires_grad_(True)
    opt = torch.optim.Adam([Ct, Gt], lr=3e-3)
    losses = []

    def refine():
        y = api.SinrFn.apply(plan, Ct, Gt, gs2)
        live = target > -299.0
        loss = ((10 * torch.log10(y.clamp_min(1e-30)) - target)[live] ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        losses.append(loss.detach())

    ms = timed(refine, 50)
    forms["sinr_aware_refinement"] = dict(
        workload="64 x (8 x 128 x 1632), ranks (8, 24, 12), Ns 4, 10 dB, Adam lr 3e-3",
        steps_per_s=1e3 / ms, ms_per_step=ms, loss_first=float(losses[0]),
        loss_last=float(losses[-1]))
    # precision form on the 16 x 256 x 3276 workload (16 paths, ranks (12, 32, 12), Ns 8 at
    # 10 dB), 8 channels per batch: fit + SINR for FP32, the three 16-bit contraction forms,
    # the FP64 Gram eigensolve, and the 16-bit forms with the FP64 eigensolve; SINR error
    # against the plain FP32 output of the same batch
    wcfg = synthgen.CONFIGS["wide"]
    nw = 8
    xs = []
    for c in range(nw):
        pp = synthgen.draw_paths(synthgen.channel_rng(wcfg.seed_index, c), wcfg.n_paths, wcfg.k_db)
        xs.append(synthgen.build_channel_torch(pp, wcfg.nr, wcfg.nt, wcfg.nsc, dev,
                                               dtype=torch.complex64).reshape(-1))
    Xw = torch.cat(xs)
    del xs
    ws2 = [float(v) for v in synthgen.snr_to_sigma2(wcfg.snr_db)]
    wide = {}
    sg_ref = None
    for name, kw in (("fp32", {}), ("bf16", dict(ttm_prec="bf16")), ("fp16", dict(ttm_prec="fp16")),
                     ("split_bf16", dict(ttm_prec="split_bf16")), ("fp32_eig_fp64", dict(eig_fp64=True)),
                     ("bf16_eig_fp64", dict(ttm_prec="bf16", eig_fp64=True)),
                     ("fp16_eig_fp64", dict(ttm_prec="fp16", eig_fp64=True)),
                     ("split_bf16_eig_fp64", dict(ttm_prec="split_bf16", eig_fp64=True))):
        planw = api.Plan([api.desc_from_config(wcfg)] * nw, iters=wcfg.iters, **kw)
        fw = planw.empty_factors()
        outw = {}

        def step_w():
            r = planw.fit(Xw, factors=fw, trace=False)
            outw["sg"] = planw.sinr(r["C"], r["G"], ws2)
            outw["st"] = r["status"]

        ms_w = timed(step_w, 2)
        sgw = outw["sg"][:, :, :wcfg.ns].cpu().numpy()
        if sg_ref is None:
            sg_ref = sgw
        live = (sgw > 0) & (sg_ref > 0)
        wide[name] = dict(fits_per_s=nw / (ms_w / 1e3), ms_per_fit_batch=ms_w,
                          max_sinr_err_db_vs_fp32=float(np.abs(10 * np.log10(sgw[live])
                                                               - 10 * np.log10(sg_ref[live])).max()),
                          status_ok=bool((outw["st"] == 0).all()))
        del planw, fw
    forms["precision_16x256x3276"] = dict(
        workload="8 x (16 x 256 x 3276), 16 paths, K 3 dB, groups of 12, ranks (12, 32, 12), "
                 "20 sweeps, fit + SINR (Ns 8, 10 dB)", **wide)
    del Xw
    # batched form: 512 channels of uneven shapes (nr 4/8/16, nt 32..256, nsc 624..3276, groups
    # of 12 or 24, ranks up to (nr, nt / 4, 12)) in one plan, fit + SINR captured in one graph
    specs = synthgen.heterogeneous_batch(512)
    descs = [dict(nr=d["nr"], nt=d["nt"], nsc=d["nsc"], group_size=d["group_size"], m=d["m"],
                  n=d["n"], p=d["p"], ns=d["ns"]) for d in specs]
    Xb = torch.cat([synthgen.build_channel_torch(d["paths"], d["nr"], d["nt"], d["nsc"], dev,
                                                 dtype=torch.complex64).reshape(-1) for d in specs])
    del specs
    planb = api.Plan(descs, iters=20)
    fb = planb.empty_factors()
    bs2 = [float(v) for v in synthgen.snr_to_sigma2([10.0])]
    sgb = torch.empty((1, planb.totals.sc, planb.ns_max), dtype=torch.float32, device=dev)
    stb = {}

    def step_b():
        r = planb.fit(Xb, factors=fb, trace=False)
        planb.sinr(fb["C"], fb["G"], bs2, out=sgb)
        stb["st"] = r["status"]

    ms_eager = timed(step_b, 2)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step_b()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb):
        step_b()
    ms_graph = timed(gb.replay, 2)
    forms["batch_512_heterogeneous"] = dict(
        workload="512 channels, nr {4,8,16}, nt {32,64,128,256}, nsc {624,1632,3276}, 4..16 paths, "
                 "groups of 12/24, ranks up to (nr, nt/4, 12), 20 sweeps, fit + SINR (10 dB)",
        fits_per_s_graph=512 / (ms_graph / 1e3), ms_per_batch_graph=ms_graph,
        fits_per_s_eager=512 / (ms_eager / 1e3), ms_per_batch_eager=ms_eager,
        subcarriers=int(planb.totals.sc), x_bytes=int(Xb.numel() * 8),
        status_ok=bool((stb["st"] == 0).all()))
    del gb, planb, fb, Xb
    return forms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("rb273", "wide"), default="rb273",
                    help="rb273: 8x64x3276 channels (the headline); wide: 16x256x3276 channels")
    ap.add_argument("--batch", type=int, default=0,
                    help="channels per step (default 64 for rb273, 8 for wide)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3,
                    help="channels timed on the oracle with all BLAS threads")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision, graph-replay, refinement and batch forms")
    ap.add_argument("--steps-only", action="store_true",
                    help="only the warm-up, timed and profiled steps of the workload and one "
                         "single-stream fit (for profiler runs: the fit kernels' launches then have "
                         "two sizes, a part of the pipelined fit and the whole batch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three plain copies of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch

    import synthgen
    from paper_2401_09792_amd import api

    cfg = synthgen.CONFIGS[args.workload]
    wide = args.workload == "wide"
    dev = torch.device("cuda:0")
    B = args.batch or (8 if wide else 64)
    s2 = [float(v) for v in synthgen.snr_to_sigma2(cfg.snr_db)]
    n_snr = len(s2)

    # inputs: B seeded channels, built on the GPU from their drawn path parameters
    xs = []
    for c in range(B):
        pp = synthgen.draw_paths(synthgen.channel_rng(cfg.seed_index, c), cfg.n_paths, cfg.k_db)
        xs.append(synthgen.build_channel_torch(pp, cfg.nr, cfg.nt, cfg.nsc, dev,
                                               dtype=torch.complex64).reshape(-1))
    X = torch.cat(xs)
    del xs
    plan = api.Plan([api.desc_from_config(cfg)] * B, iters=cfg.iters)
    f = plan.empty_factors()
    gsinr = torch.full((n_snr, plan.totals.sc, plan.ns_max), 1.0e-3, dtype=torch.float32,
                       device=dev)
    torch.cuda.synchronize()

    def step():
        res = plan.fit(X, factors=f, trace=False)
        ht, _ = plan.reconstruct(res["A"], res["B"], res["C"], res["G"], ht=True, xhat=False)
        sg = plan.sinr(res["C"], res["G"], s2)
        gC, gG = plan.sinr_backward(res["C"], res["G"], s2, gsinr)
        return res, ht, sg

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # headline: the timed steps with the library's kernel timing off
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, ht, sg = step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps

    # a second pass of the same steps with every kernel bracketed by HIP events on its own
    # stream: live per-kernel durations for the rooflines
    kern = profile_steps(api, step, args.steps)
    # the T pass and the eigensolves also run once unsplit (one stream), so that their
    # durations are their own and not shared with concurrent parts
    # (also with --steps-only: the rooflines need the fit kernels' own durations)
    plan.set_tuning(bstep=0, tpass=0, split=0)
    kern_unsplit = profile_steps(api, lambda: plan.fit(X, factors=f, trace=False), 1)
    plan.set_tuning(bstep=0, tpass=0, split=2)
    torch.cuda.synchronize()

    fits_per_s = B * args.steps / (ms_total / 1e3)
    ng = -(-cfg.nsc // cfg.group_size)
    sinr_units = B * cfg.nsc * n_snr

    # dominant kernel with an algorithmic work model, and its roofline
    nr, nt, m, n, p, gs = cfg.nr, cfg.nt, cfg.m, cfg.n, cfg.p, cfg.group_size
    n_sweeps = cfg.iters
    sinr_flops = sinr_units * sinr_unit_flops(m, n, p, cfg.ns, n_snr)
    models = {
        # wide path, per launch over the B channels: the mode-2 Gram (one launch on the rows of
        # X for the initialisation, one per sweep on the W rows: the average over the
        # 1 + sweeps launches), T = H B, and the W rows of the B-step
        "k_gram_rows_st": B * CMAC * nt * (nt + 1) / 2
        * (cfg.nsc * nr + n_sweeps * ng * p * m) / (1 + n_sweeps),
        "k_rows_times_b": B * CMAC * cfg.nsc * nr * nt * n,
        "k_w_rows": B * CMAC * ng * (p * gs * nr * nt + p * m * nr * nt),
        # per launch: B channels x ng groups
        "k_fused_b_mfma": B * ng * CMAC * (gs * m * nr * nt + p * gs * m * nt
                                           + p * m * nt * nt / 2),
        "k_fused_b_mm": B * ng * CMAC * bstep_group_cmacs(nr, nt, gs, m, p),
        "k_sinr_lane": sinr_flops,
        "k_sinr_rows": sinr_flops,
        "k_sinr": sinr_flops,
        "k_gram_rows": B * gram_rows_flops(ng, p, m, nt),
    }
    bounds = {"k_fused_b_mfma": "mfma", "k_fused_b_mm": "mfma", "k_gram_rows": "mfma",
              "k_gram_rows_st": "mfma", "k_rows_times_b": "mfma", "k_w_rows": "mfma"}
    # the fit's pipelined parts overlap on four streams, so a kernel's own duration comes from
    # the single-stream pass of the same fit (every fit kernel there is one launch over the B
    # channels); the SINR, adjoint and reconstruction kernels run alone in either pass
    kfit = {k: v for k, v in kern.items()}
    kfit.update(kern_unsplit)
    ranked = sorted(((v["total_ms"], k) for k, v in kfit.items() if k in models), reverse=True)
    roof = None
    if ranked:
        dom = ranked[0][1]
        ach = models[dom] / (kfit[dom]["avg_us"] * 1e-6) / 1e12
        bound = bounds.get(dom, "alu")
        peak = PEAK_FP32_TFLOPS if bound == "mfma" else PEAK_VALU_FP32_TFLOPS
        roof = dict(kernel=dom, bound=bound, achieved=ach, peak=peak, unit="TFLOP/s",
                    frac=ach / peak, traffic=measured_traffic(dom, args.workload),
                    algorithmic_flops_per_launch=models[dom], avg_us=kfit[dom]["avg_us"],
                    timed_in="single-stream fit pass" if dom in kern_unsplit else "timed steps",
                    share_of_step=kfit[dom]["total_ms"] / ms_step)
    sinr_name = next((k for k in ("k_sinr_rows", "k_sinr_lane", "k_sinr") if k in kern), None)
    sinr_k = kern.get(sinr_name) if sinr_name else None
    sinr_rate = sinr_units / (sinr_k["total_ms"] * 1e-3) if sinr_k else None
    roof_sinr = None
    if sinr_k:
        t_s = sinr_k["total_ms"] * 1e-3
        sinr_bytes = sinr_units * sinr_unit_bytes(m, n, p, gs, n_snr, cfg.ns)
        roof_sinr = dict(kernel=sinr_name, bound="alu", achieved=sinr_flops / t_s / 1e12,
                         peak=PEAK_VALU_FP32_TFLOPS, unit="TFLOP/s",
                         frac=sinr_flops / t_s / 1e12 / PEAK_VALU_FP32_TFLOPS,
                         algorithmic_flops_per_launch=sinr_flops,
                         evals_per_launch=sinr_units, evals_per_s=sinr_rate,
                         hbm_gb_s=sinr_bytes / t_s / 1e9,
                         hbm_frac=sinr_bytes / t_s / 1e9 / PEAK_HBM_GBS,
                         traffic=measured_traffic(sinr_name, args.workload),
                         share_of_step=sinr_k["total_ms"] / ms_step)
    roof_rec = None
    if "k_reconstruct_ht" in kern:
        # Ht written, each group's core and the C rows read once
        rec_bytes = B * 8.0 * (cfg.nsc * m * n + ng * p * m * n + cfg.nsc * p)
        t_r = kern["k_reconstruct_ht"]["avg_us"] * 1e-6
        roof_rec = dict(kernel="k_reconstruct_ht", bound="hbm", achieved=rec_bytes / t_r / 1e9,
                        peak=PEAK_HBM_GBS, unit="GB/s", frac=rec_bytes / t_r / 1e9 / PEAK_HBM_GBS,
                        algorithmic_bytes_per_launch=rec_bytes,
                        traffic=measured_traffic("k_reconstruct_ht", args.workload))
    # the fit's other passes: the T pass on its work model (unsplit launch), the eigensolves
    # as latency (iterative; their flops are not counted)
    fit_parts = {}
    t_pass = kern_unsplit.get("k_fused_t_mfma")
    if t_pass:
        # T = H B, and Yh = A^H T unless m == nr (then the mode-3 Gram is taken of T and Yh is
        # formed on the last sweep only; its products are left out of the average)
        t_flops = B * ng * CMAC * (gs * nr * nt * n + (0 if m == nr else gs * m * nr * n))
        fit_parts["k_fused_t_mfma_unsplit"] = dict(
            avg_us=t_pass["avg_us"], algorithmic_flops_per_launch=t_flops,
            achieved_tflops=t_flops / (t_pass["avg_us"] * 1e-6) / 1e12,
            frac_mfma_fp32=t_flops / (t_pass["avg_us"] * 1e-6) / 1e12 / PEAK_FP32_TFLOPS)
    for nm in ("k_eigA", "k_eigA_rows", "k_eigB", "k_eigC", "k_eigC_rows", "k_fused_z",
               "k_reduce_S1", "k_reduce_S2_mfma"):
        if nm in kern_unsplit:
            fit_parts[nm + "_unsplit"] = dict(avg_us=kern_unsplit[nm]["avg_us"],
                                              launches_per_fit=kern_unsplit[nm]["launches"],
                                              ms_per_fit=kern_unsplit[nm]["total_ms"])
    fit_flops = B * CMAC * fit_cmacs(nr, nt, cfg.nsc, gs, m, n, p, cfg.iters)
    fit_parts["whole_step_sweep_mfma_frac"] = fit_flops / (ms_step * 1e-3) / 1e12 / PEAK_FP32_TFLOPS

    # single-channel latency and a 256-channel batch of the same step
    extras = not wide and not args.steps_only
    latency = single_channel_latency(api, synthgen, cfg, s2, dev, torch) if extras else None
    big = batch_throughput(api, synthgen, cfg, s2, dev, torch, 256) if extras else None

    # accuracy of this step's output on channel 0 against the oracle, and the CPU baseline
    cpu = None
    acc = {}
    if not args.no_cpu_baseline:
        import threadpoolctl

        from oracle import metrics, sinr as osinr, tucker

        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
        host = host_description()
        if wide:
            # a bounded sample: the first 540 subcarriers (45 groups) of channel 0, scaled to
            # channels of 3276 subcarriers
            nsub = 540
            rng = synthgen.channel_rng(cfg.seed_index, 0)
            Xs = synthgen.build_channel(synthgen.draw_paths(rng, cfg.n_paths, cfg.k_db),
                                        cfg.nr, cfg.nt, nsub)
            t = time.perf_counter()
            orc = tucker.fit(Xs, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.iters)
            Ht_o, _ = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"], cfg.group_size)
            osinr.sinr(Ht_o, s2, cfg.ns)
            cpu_s = time.perf_counter() - t
            cpu = dict(value=(nsub / cfg.nsc) / cpu_s, unit="fits/s", cores=threads, kind="oracle",
                       sample=f"first {nsub} of {cfg.nsc} subcarriers of one channel: fit + Ht + "
                              f"SINR (no adjoint), {cpu_s:.1f} s, scaled by {nsub}/{cfg.nsc}; "
                              "complex128 NumPy/LAPACK", host=host)
        else:
            # all BLAS threads on args.cpu_sample channels, then one thread on one channel; the
            # SINR part of each is also reported as evals/s
            def oracle_channels(nch):
                t_fit = t_sinr = 0.0
                first = None
                for c in range(nch):
                    Xc = synthgen.make_channel(cfg, c)
                    t = time.perf_counter()
                    orc = tucker.fit(Xc, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.iters)
                    Ht_o, _ = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"],
                                                 cfg.group_size)
                    t_fit += time.perf_counter() - t
                    t = time.perf_counter()
                    sg_o = osinr.sinr(Ht_o, s2, cfg.ns)
                    t_sinr += time.perf_counter() - t
                    if first is None:
                        first = (Xc, orc, sg_o)
                return t_fit, t_sinr, first

            nsamp = max(1, args.cpu_sample)
            t_fit, t_sinr, orc0 = oracle_channels(nsamp)
            with threadpoolctl.threadpool_limits(1):
                t_fit1, t_sinr1, _ = oracle_channels(1)
            evals = cfg.nsc * n_snr
            cpu = dict(value=nsamp / (t_fit + t_sinr), unit="fits/s", cores=threads, kind="oracle",
                       sample=f"{nsamp} channel(s) of the workload: fit + Ht + SINR at 4 SNRs "
                              f"(no adjoint), {t_fit + t_sinr:.1f} s, complex128 NumPy/LAPACK",
                       sinr_evals_per_s=nsamp * evals / t_sinr,
                       single_thread=dict(value=1.0 / (t_fit1 + t_sinr1), unit="fits/s", cores=1,
                                          sinr_evals_per_s=evals / t_sinr1,
                                          sample=f"1 channel, {t_fit1 + t_sinr1:.1f} s"),
                       host=host)
    if not args.no_cpu_baseline and not wide:
        from oracle import metrics

        Xc, orc, sg_o = orc0
        sg0 = sg[:, :cfg.nsc, :cfg.ns].cpu().numpy()
        err = metrics.db_error(sg0, sg_o)
        _, xh = plan.reconstruct(res["A"], res["B"], res["C"], res["G"], ht=False, xhat=True)
        xh0 = xh[:cfg.nsc * cfg.nr * cfg.nt].cpu().numpy().reshape(Xc.shape)
        acc = dict(max_sinr_err_db=float(err.max()), mean_sinr_err_db=float(err.mean()),
                   nmse_gpu=metrics.nmse(Xc, xh0))

    forms = None
    if not args.no_forms and not wide and not args.steps_only:
        forms = time_forms(api, synthgen, cfg, X, B, s2, ms_step, sg, torch, max(args.steps, 2))
        forms["compression_models"] = time_models(api, synthgen, torch, dev)
        forms["paper_submatrix_8x256x401"] = time_submatrix(api, synthgen, torch, dev)

    line = {
        "metric": "subcarrier SINR evals/sec + Tucker fits/sec at <=0.1 dB err vs FP64 oracle",
        "value": fits_per_s,
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": ("wide: 16x256x3276 channels, 16 paths, groups of 12, ranks "
                                "(12,32,12), 20 sweeps, Ns=8, SNR 10 dB") if wide else
                               ("rb273: 8x64x3276 channels, groups of 12, ranks (8,16,12), "
                                "20 sweeps, Ns=4, SNR -5/0/10/20 dB"),
                   "channels_per_step": B, "parallelism": "single GPU"},
        "sinr_evals_per_s": sinr_rate,
        "roofline": roof,
        "roofline_sinr": roof_sinr,
        "roofline_reconstruct": roof_rec,
        "fit_parts": fit_parts,
        "latency_1ch": latency,
        "batch_256": big,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "kernels": kern,
        "kernels_unsplit_fit": kern_unsplit,
        "forms": forms,
        "wall_s": wall,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
