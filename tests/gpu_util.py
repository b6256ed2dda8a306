"""Helpers for the GPU parity tests: packing oracle arrays into the library's buffers."""

import sys

import numpy as np
import torch

import synthgen
from oracle import tucker


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev_c64(a: np.ndarray) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.complex64).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def desc(nr, nt, nsc, gs, m, n, p, ns):
    return dict(nr=nr, nt=nt, nsc=nsc, group_size=gs, m=m, n=n, p=p, ns=ns)


def unpack(plan, c: int, buf: np.ndarray, what: str) -> np.ndarray:
    """Channel c's block of a packed buffer, reshaped to the documented layout."""
    d = plan.descs[c]
    o = plan.offsets(c)
    ng = -(-d["nsc"] // d["group_size"])
    shapes = dict(x=(d["nsc"], d["nr"], d["nt"]), a=(d["nr"], d["m"]), b=(d["nt"], d["n"]),
                  c=(d["nsc"], d["p"]), g=(ng, d["p"], d["m"], d["n"]),
                  ht=(d["nsc"], d["m"], d["n"]))
    shp = shapes[what]
    start = getattr(o, what)
    return buf[start:start + int(np.prod(shp))].reshape(shp)


def db(x):
    return 10.0 * np.log10(x)


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
