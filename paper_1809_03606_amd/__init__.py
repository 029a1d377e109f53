"""Batched successive-cancellation stack decoding of polar codes on MI355X (gfx950).

The decoder is the HIP library ``libpolarscs.so`` (C-ABI in ``include/polarscs.h``);
``binding`` marshals arguments to it, ``channel`` generates seeded BPSK/AWGN inputs.
Importing the package loads nothing; the first library call does.
"""
from . import binding, channel  # noqa: F401

__all__ = ["binding", "channel"]
