"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random numbers and assembles channel tensors from them.  It
contains none of the compression or SINR arithmetic: the oracle and the HIP library each
implement that on their own.
"""

from .channels import (  # noqa: F401
    ChannelConfig,
    PathParams,
    CONFIGS,
    draw_paths,
    channel_rng,
    build_channel,
    build_channel_torch,
    make_channel,
    random_unitary,
    planted_tucker,
    heterogeneous_batch,
    snr_to_sigma2,
    system_links,
    make_system,
    draw_submatrix_paths,
    build_submatrices,
    submatrix_weights,
)
