import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly when it is not built."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2401_09792_amd import api

    api.load()  # raises if the shared library is missing
    return api


@pytest.fixture(scope="session")
def rb273_oracle():
    """The 8 x 64 x 3276 channel (273 groups of 12, ranks (8, 16, 12), 20 sweeps) and the
    FP64 oracle's fit, reconstruction and compressed SINR at its four SNRs."""
    import synthgen
    from oracle import sinr as osinr, tucker

    cfg = synthgen.CONFIGS["rb273"]
    X = synthgen.make_channel(cfg, 0)
    orc = tucker.fit(X, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.iters)
    Ht, Xh = tucker.reconstruct(orc["A"], orc["B"], orc["C"], orc["G"], cfg.group_size)
    s2 = synthgen.snr_to_sigma2(cfg.snr_db)
    return dict(cfg=cfg, X=X, orc=orc, Xh=Xh, sinr=osinr.sinr(Ht, s2, cfg.ns), s2=s2)
