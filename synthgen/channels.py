"""Seeded OFDM massive-MIMO channel generator (input synthesis only).

The paper measures on 3GPP TR 38.901 channels (Section 4, first paragraph), which are not
available here.  This generator stands in for them with a geometric multipath model of the
same structure as the paper's channel-submatrix equation: each subcarrier matrix is a sum
of one line-of-sight path and L-1 non-line-of-sight paths,

    H_k = sum_l alpha_l * exp(-j 2 pi k tau_l / Nsc) * a_r(theta_l) a_t(phi_l)^H,

with half-wavelength uniform linear arrays a_N(x)_i = exp(j pi i sin x), i = 0..N-1.
The LOS gain is sqrt(K/(K+1)) e^{j psi}; each NLOS gain is CN(0, 1/((K+1)(L-1))), so the
expected total path power is one and E|h_ij|^2 = 1.  Angles are U(-60 deg, 60 deg), delays
U(0, 16) samples.

Draw order per channel (fixed, so a seed always gives the same tensor): theta[L], phi[L],
tau[L], psi, then the NLOS real parts and imaginary parts.
Channel c of configuration k uses the child seed SeedSequence(240109792 + k, spawn_key=(c,)).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

BASE_SEED = 240109792


@dataclasses.dataclass(frozen=True)
class ChannelConfig:
    name: str
    nr: int
    nt: int
    nsc: int
    n_paths: int
    k_db: float
    group_size: int
    m: int
    n: int
    p: int
    iters: int
    ns: int
    snr_db: Sequence[float]
    n_channels: int = 1
    seed_index: int = 0


# Workload shapes (paper: Section 4 uses 3GPP channels; these are synthetic stand-ins).
CONFIGS: Dict[str, ChannelConfig] = {
    # small case, complex128 on the CPU, also run on the GPU in complex64
    "small": ChannelConfig("small", 4, 32, 64, 4, 10.0, 16, 4, 8, 4, 10, 2, (10.0,), 1, 0),
    # plain FP32 single-GPU case: 273 resource blocks x 12 subcarriers
    "rb273": ChannelConfig("rb273", 8, 64, 3276, 8, 6.0, 12, 8, 16, 12, 20, 4,
                           (-5.0, 0.0, 10.0, 20.0), 1, 1),
    # precision case: larger arrays, lossy in mode 1
    "wide": ChannelConfig("wide", 16, 256, 3276, 16, 3.0, 12, 12, 32, 12, 20, 8, (10.0,), 1, 2),
    # differentiation case: 64 channels, lossy in mode 2 (32 paths > n = 24)
    "grad": ChannelConfig("grad", 8, 128, 1632, 32, 3.0, 12, 8, 24, 12, 20, 4, (10.0,), 64, 4),
}


@dataclasses.dataclass
class PathParams:
    theta: np.ndarray  # receive angles [L], radians
    phi: np.ndarray    # transmit angles [L], radians
    tau: np.ndarray    # delays [L], samples
    alpha: np.ndarray  # complex gains [L]


def channel_rng(seed_index: int, channel: int) -> np.random.Generator:
    ss = np.random.SeedSequence(BASE_SEED + seed_index, spawn_key=(channel,))
    return np.random.default_rng(ss)


def draw_paths(rng: np.random.Generator, n_paths: int, k_db: float) -> PathParams:
    L = int(n_paths)
    lim = math.radians(60.0)
    theta = rng.uniform(-lim, lim, size=L)
    phi = rng.uniform(-lim, lim, size=L)
    tau = rng.uniform(0.0, 16.0, size=L)
    psi = rng.uniform(0.0, 2.0 * math.pi)
    kf = 10.0 ** (k_db / 10.0)
    alpha = np.zeros(L, dtype=np.complex128)
    alpha[0] = math.sqrt(kf / (kf + 1.0)) * np.exp(1j * psi)
    if L > 1:
        re = rng.standard_normal(L - 1)
        im = rng.standard_normal(L - 1)
        scale = math.sqrt(1.0 / ((kf + 1.0) * (L - 1)) / 2.0)
        alpha[1:] = scale * (re + 1j * im)
    return PathParams(theta, phi, tau, alpha)


def _steering(n: int, ang: np.ndarray) -> np.ndarray:
    idx = np.arange(n)[:, None]
    return np.exp(1j * math.pi * idx * np.sin(ang)[None, :])  # [n, L]


def build_channel(pp: PathParams, nr: int, nt: int, nsc: int) -> np.ndarray:
    """Channel tensor laid out [nsc][nr][nt], complex128."""
    ar = _steering(nr, pp.theta)                 # [nr, L]
    at = _steering(nt, pp.phi)                   # [nt, L]
    k = np.arange(nsc)[:, None]
    ph = np.exp(-2j * math.pi * k * pp.tau[None, :] / nsc) * pp.alpha[None, :]  # [nsc, L]
    # sum over paths of ph[k,l] * ar[:,l] * conj(at[:,l])^T
    return np.einsum("kl,il,jl->kij", ph, ar, at.conj(), optimize=True)


def build_channel_torch(pp: PathParams, nr: int, nt: int, nsc: int, device,
                        dtype=None):
    """Same tensor as build_channel, assembled with torch on `device` (fp64 then cast)."""
    import torch

    c128 = torch.complex128
    ar = torch.as_tensor(_steering(nr, pp.theta), dtype=c128, device=device)
    at = torch.as_tensor(_steering(nt, pp.phi), dtype=c128, device=device)
    k = torch.arange(nsc, dtype=torch.float64, device=device)[:, None]
    tau = torch.as_tensor(pp.tau, dtype=torch.float64, device=device)[None, :]
    alpha = torch.as_tensor(pp.alpha, dtype=c128, device=device)[None, :]
    ph = torch.exp(-2j * math.pi * k * tau / nsc) * alpha          # [nsc, L]
    left = ph[:, None, :] * ar[None, :, :]                          # [nsc, nr, L]
    x = torch.matmul(left, at.conj().transpose(0, 1).contiguous())  # [nsc, nr, nt]
    if dtype is not None:
        x = x.to(dtype)
    return x


def make_channel(cfg: ChannelConfig, channel: int = 0) -> np.ndarray:
    rng = channel_rng(cfg.seed_index, channel)
    pp = draw_paths(rng, cfg.n_paths, cfg.k_db)
    return build_channel(pp, cfg.nr, cfg.nt, cfg.nsc)


def random_unitary(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns (QR of a complex Gaussian)."""
    z = rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def planted_tucker(rng: np.random.Generator, nr: int, nt: int, nsc: int, gs: int,
                   m: int, n: int, p: int):
    """A channel tensor that is exactly representable at ranks (m, n, p) per group.

    Returns (X [nsc][nr][nt], A [nr][m], B [nt][n], C [nsc][p], G [groups][p][m][n]) with
    X_s = A (sum_q C[s,q] G_g[q]) B^H.  Used as input for exact-recovery tests.
    """
    A = random_unitary(rng, nr, m)
    B = random_unitary(rng, nt, n)
    n_groups = -(-nsc // gs)
    C = np.zeros((nsc, p), dtype=np.complex128)
    G = np.zeros((n_groups, p, m, n), dtype=np.complex128)
    X = np.zeros((nsc, nr, nt), dtype=np.complex128)
    for g in range(n_groups):
        s0 = g * gs
        sz = min(gs, nsc - s0)
        pg = min(p, sz)
        Cg = random_unitary(rng, sz, pg)
        C[s0:s0 + sz, :pg] = Cg
        core = rng.standard_normal((pg, m, n)) + 1j * rng.standard_normal((pg, m, n))
        # decaying core energy keeps the eigengaps well separated
        core *= (0.7 ** np.arange(pg))[:, None, None]
        G[g, :pg] = core
        for i in range(sz):
            Ht = np.tensordot(Cg[i], core, axes=(0, 0))
            X[s0 + i] = A @ Ht @ B.conj().T
    return X, A, B, C, G


def heterogeneous_batch(n_channels: int = 512, seed_index: int = 3) -> List[dict]:
    """Shapes and path parameters of a mixed batch of channels.

    Nr from {4, 8, 16}, Nt from {32, 64, 128, 256}, Nsc from {624, 1632, 3276}, L from
    U{4..16}, K-factor U(0, 10) dB, group size from {12, 24}; ranks m ~ U{Ns..Nr},
    n ~ U{Ns..Nt/4}, p ~ U{1..min(12, gs)}; Ns = min(Nr, 4).
    """
    out = []
    for c in range(n_channels):
        rng = channel_rng(seed_index, c)
        nr = int(rng.choice([4, 8, 16]))
        nt = int(rng.choice([32, 64, 128, 256]))
        nsc = int(rng.choice([624, 1632, 3276]))
        L = int(rng.integers(4, 17))
        kdb = float(rng.uniform(0.0, 10.0))
        gs = int(rng.choice([12, 24]))
        ns = min(nr, 4)
        m = int(rng.integers(ns, nr + 1))
        n = int(rng.integers(ns, nt // 4 + 1))
        p = int(rng.integers(1, min(12, gs) + 1))
        pp = draw_paths(rng, L, kdb)
        out.append(dict(nr=nr, nt=nt, nsc=nsc, n_paths=L, k_db=kdb, group_size=gs,
                        m=m, n=n, p=p, ns=ns, paths=pp))
    return out


def system_links(J: int, K: int) -> List[tuple]:
    """Links (u, k) of a system of J base stations with K UEs per cell, UE u = i K + j served by
    BS i, in the order the channels of a system plan are laid out (UE-major)."""
    return [(u, k) for u in range(J * K) for k in range(J)]


def make_system(J: int, K: int, nr: int, nt: int, nsc: int, n_paths: int, k_db: float,
                seed_index: int = 5) -> dict:
    """Channel tensors [nsc][nr][nt] of every link (u, k) of a J-cell system, each from its own
    seeded paths (child seed = the link's position in system_links)."""
    out = {}
    for idx, lk in enumerate(system_links(J, K)):
        pp = draw_paths(channel_rng(seed_index, idx), n_paths, k_db)
        out[lk] = build_channel(pp, nr, nt, nsc)
    return out


def draw_submatrix_paths(rng: np.random.Generator, n_clusters: int = 20, rays: int = 20,
                         k_db: float = 6.0, spread_deg: float = 2.0,
                         max_delay: float = 16.0) -> PathParams:
    """Rays of a clustered multipath channel, one channel submatrix per ray (the structure of
    the paper's channel-submatrix equation, Section 2.2, with P = n_clusters * rays + 1; the
    paper's 3GPP channels have P = 401, which the defaults give).  Stand-in for TR 38.901:
    cluster angles U(-60 deg, 60 deg), ray angles the cluster's plus N(0, spread_deg), cluster
    delays U(0, max_delay) samples with ray jitter U(0, 0.5), cluster powers proportional to
    exp(-delay / 4) summing to 1/(K+1), ray gains CN(0, cluster power / rays), and the LOS ray
    (gain sqrt(K/(K+1)) e^{j psi}, delay 0) last.  Ray l of cluster k sits at index k rays + l,
    so that groups of `rays` consecutive submatrices are the clusters.

    Draw order: cluster theta, phi, delay [n_clusters]; ray theta and phi offsets and delay
    jitter [n_clusters * rays]; psi, LOS theta, LOS phi; then the ray gains' real and
    imaginary parts."""
    nc, nrays = int(n_clusters), int(rays)
    lim = math.radians(60.0)
    sp = math.radians(spread_deg)
    ct = rng.uniform(-lim, lim, size=nc)
    cp = rng.uniform(-lim, lim, size=nc)
    cd = rng.uniform(0.0, max_delay, size=nc)
    dt = rng.standard_normal(nc * nrays) * sp
    dp = rng.standard_normal(nc * nrays) * sp
    dj = rng.uniform(0.0, 0.5, size=nc * nrays)
    psi = rng.uniform(0.0, 2.0 * math.pi)
    los_t = rng.uniform(-lim, lim)
    los_p = rng.uniform(-lim, lim)
    re = rng.standard_normal(nc * nrays)
    im = rng.standard_normal(nc * nrays)
    kf = 10.0 ** (k_db / 10.0)
    pw = np.exp(-cd / 4.0)
    pw = pw / pw.sum() / (kf + 1.0)
    ray_pw = np.repeat(pw / nrays, nrays)
    theta = np.concatenate([np.repeat(ct, nrays) + dt, [los_t]])
    phi = np.concatenate([np.repeat(cp, nrays) + dp, [los_p]])
    tau = np.concatenate([np.repeat(cd, nrays) + dj, [0.0]])
    alpha = np.concatenate([np.sqrt(ray_pw / 2.0) * (re + 1j * im),
                            [math.sqrt(kf / (kf + 1.0)) * np.exp(1j * psi)]])
    return PathParams(theta, phi, tau, alpha)


def build_submatrices(pp: PathParams, nr: int, nt: int) -> np.ndarray:
    """Channel submatrices at the reference time, one per ray: X_l = alpha_l a_r(theta_l)
    a_t(phi_l)^H, laid out [P][nr][nt] (mode 3 = submatrices), complex128."""
    ar = _steering(nr, pp.theta)
    at = _steering(nt, pp.phi)
    return np.einsum("l,il,jl->lij", pp.alpha, ar, at.conj(), optimize=True)


def submatrix_weights(pp: PathParams, n_pts: int, n_fft: int) -> np.ndarray:
    """Combining rows u_t[l] = exp(-j 2 pi t tau_l / n_fft) for the points t = 0..n_pts-1 of an
    n_fft-point OFDM grid, [n_pts][P]: combining the submatrices with them gives the channel
    at subcarrier t."""
    t = np.arange(int(n_pts))[:, None]
    return np.exp(-2j * math.pi * t * pp.tau[None, :] / float(n_fft))


def snr_to_sigma2(snr_db: Sequence[float]) -> np.ndarray:
    """Noise variance for unit average channel gain and unit power per stream."""
    return 10.0 ** (-np.asarray(snr_db, dtype=np.float64) / 10.0)
