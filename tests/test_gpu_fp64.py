"""The FP64 device path (c128 plans): the SINR chain of Section 3.3 and its adjoint in double
precision on the GPU, checked against the FP64 oracle and by central finite differences
(torch.autograd.gradcheck) on the 2 x 8 x 12 slice of the differentiation workload
(one group of 12 subcarriers, ranks (2, 4, 3), Ns = 2).

The FP64 path also calibrates the bar of the FP32 adjoint: the FP32 kernels see C and G
rounded to FP32 and round inside the chain at the same relative level, so their error is
measured against the change of the exact (FP64) gradient under relative input perturbations
of one FP32 unit roundoff (the gradient's sensitivity), not against a fixed fraction.
"""

import numpy as np
import pytest
import torch

from oracle import grad as ograd
from tests.gpu_util import announce, crandn, desc, dev_c64, host, unpack
from tests.test_gpu_backward import _compressed

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # FP32 unit roundoff


def dev_c128(a: np.ndarray) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.complex128).cuda()


def _f32(v):
    # the noise variances cross the ABI as float32; the oracle takes the same values
    return [float(np.float32(x)) for x in v]


SHAPES = [
    # nsc, gs, m, n, p, ns
    (12, 12, 2, 4, 3, 2),      # the 2 x 8 x 12 slice
    (40, 12, 8, 16, 12, 4),
    (30, 16, 4, 8, 4, 3),      # short last group
    (26, 13, 10, 20, 4, 4),    # m > 8
    (22, 11, 12, 40, 3, 4),    # n > 32
]


@pytest.mark.parametrize("shape", SHAPES)
def test_c128_sinr_and_adjoint_match_oracle(gpu_lib, shape):
    nsc, gs, m, n, p, ns = shape
    announce(f"c128 sinr + adjoint {shape}")
    rng, C, G = _compressed(7, nsc, gs, m, n, p)
    s2 = _f32([0.05, 0.5])
    plan = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns)], iters=1, dtype="c128")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = host(plan.sinr(dev_c128(C), dev_c128(G), s2, status=st))
    assert y.dtype == np.float64
    ref = ograd.sinr_compressed_t(torch.as_tensor(C), torch.as_tensor(G), gs, s2, ns).numpy()
    rel = np.abs(y[..., :ns] - ref).max() / np.abs(ref).max()
    g_up = rng.standard_normal((2, nsc, ns))
    gs_full = np.zeros((2, nsc, plan.ns_max))
    gs_full[..., :ns] = g_up
    gC, gG = plan.sinr_backward(dev_c128(C), dev_c128(G), s2, torch.as_tensor(gs_full).cuda())
    gC_o, gG_o = ograd.sinr_grad(C, G, gs, s2, ns, g_up)
    eC = np.abs(unpack(plan, 0, host(gC), "c") - gC_o).max() / np.abs(gC_o).max()
    eG = np.abs(unpack(plan, 0, host(gG), "g") - gG_o).max() / np.abs(gG_o).max()
    print(f"[c128] {shape}: SINR {rel:.2e}, dl/dC {eC:.2e}, dl/dG {eG:.2e} (relative to max)",
          flush=True)
    assert int(st.item()) == 0
    assert rel <= 1e-10, rel
    assert eC <= 1e-9 and eG <= 1e-9, (eC, eG)


def test_c128_sinr_full_matches_oracle(gpu_lib):
    announce("c128 full-channel sinr")
    rng = np.random.default_rng(17)
    X = crandn(rng, 20, 6, 40)
    s2 = _f32([0.1, 1.0])
    plan = gpu_lib.Plan([desc(6, 40, 20, 10, 4, 8, 4, 3)], iters=1, dtype="c128")
    y = host(plan.sinr_full(dev_c128(X), s2))[..., :3]
    ref = ograd.sinr_chain_t(torch.as_tensor(X), s2, 3).numpy()
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_gradcheck_fp64_slice(gpu_lib):
    # central finite differences of the GPU's FP64 forward against its FP64 adjoint, through
    # the autograd function, on one group of 12 subcarriers of a 2 x 8 array at ranks (2, 4, 3)
    announce("gradcheck 2x8x12 slice, c128")
    _, C, G = _compressed(21, 12, 12, 2, 4, 3)
    plan = gpu_lib.Plan([desc(2, 8, 12, 12, 2, 4, 3, 2)], iters=1, dtype="c128")
    Ct = dev_c128(C).requires_grad_(True)
    Gt = dev_c128(G).requires_grad_(True)
    s2 = _f32([0.1])  # 10 dB

    def f(c, g):
        return gpu_lib.SinrFn.apply(plan, c, g, s2)

    assert torch.autograd.gradcheck(f, (Ct, Gt), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("shape", [(40, 12, 8, 16, 12, 4), (30, 16, 4, 8, 4, 3),
                                   (26, 13, 10, 20, 4, 4)])
def test_fp32_adjoint_within_its_sensitivity(gpu_lib, shape):
    # The FP32 adjoint against the exact (FP64 GPU) gradient, with a bar set by the gradient's
    # measured sensitivity: the largest change of the FP64 gradient over three relative input
    # perturbations of size u = 2^-24.  A factor of 64 covers the depth of the chain (Gram,
    # Jacobi sweeps, Cholesky, two solves, the adjoint stages), each rounding at level u.
    nsc, gs, m, n, p, ns = shape
    announce(f"fp32 adjoint vs sensitivity {shape}")
    rng, C, G = _compressed(23, nsc, gs, m, n, p)
    s2 = _f32([0.05, 0.5])
    g_up = rng.standard_normal((2, nsc, ns))
    p64 = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns)], iters=1, dtype="c128")
    p32 = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns)], iters=1)
    g64 = torch.zeros((2, nsc, p64.ns_max), dtype=torch.float64)
    g64[..., :ns] = torch.as_tensor(g_up)

    def grad64(Cv, Gv):
        gC, gG = p64.sinr_backward(dev_c128(Cv), dev_c128(Gv), s2, g64.cuda())
        return unpack(p64, 0, host(gC), "c"), unpack(p64, 0, host(gG), "g")

    ref_C, ref_G = grad64(C, G)
    sens_C = sens_G = 0.0
    for k in range(3):
        pr = np.random.default_rng(100 + k)
        Cp = C * (1 + U32 * crandn(pr, *C.shape) / np.sqrt(2))
        Gp = G * (1 + U32 * crandn(pr, *G.shape) / np.sqrt(2))
        Cp[C == 0] = 0
        Gp[G == 0] = 0
        a, b = grad64(Cp, Gp)
        sens_C = max(sens_C, np.abs(a - ref_C).max() / np.abs(ref_C).max())
        sens_G = max(sens_G, np.abs(b - ref_G).max() / np.abs(ref_G).max())
    gC, gG = p32.sinr_backward(dev_c64(C), dev_c64(G), s2, g64.float().cuda())
    eC = np.abs(unpack(p32, 0, host(gC), "c") - ref_C).max() / np.abs(ref_C).max()
    eG = np.abs(unpack(p32, 0, host(gG), "g") - ref_G).max() / np.abs(ref_G).max()
    print(f"[fp32 adjoint] {shape}: error dl/dC {eC:.2e} dl/dG {eG:.2e}; sensitivity "
          f"dl/dC {sens_C:.2e} dl/dG {sens_G:.2e} (relative to max)", flush=True)
    assert eC <= 64 * max(sens_C, U32), (eC, sens_C)
    assert eG <= 64 * max(sens_G, U32), (eG, sens_G)
