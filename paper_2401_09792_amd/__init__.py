"""MI355X-native groupwise Tucker compression of OFDM massive-MIMO channels and
compressed-domain SINR (HIP kernels behind the C ABI of include/gtucker.h)."""

from . import _binding  # noqa: F401


def load():
    """Loads libgtucker.so (raises if it is not built)."""
    return _binding.load()
