"""MI355X (gfx950) implementation of the split-step method (SSM) for
McKean-Vlasov SDEs, arXiv:2105.09688: the per-time-step update of an
N-particle interacting system as hand-written HIP kernels behind a C ABI
(include/ssm.h).  The shared library is loaded on first use and its absence is
an error: there is no fallback path."""
from ._lib import SSMError, load  # noqa: F401

__all__ = ["SSM", "SSMError", "load", "workloads"]


def __getattr__(name):
    if name in ("SSM", "pair_sum", "implicit_solve", "brownian", "philox_blocks"):
        from . import ssm as _ssm
        return getattr(_ssm, name)
    raise AttributeError(name)
