"""MI355X (gfx950) U(1)-symmetric MPS gate engine.

The gate path (Theta formation by charge-sector products, block-diagonal
gate, per-sector Jacobi SVD, global truncation, update) runs in the HIP
kernels of ``libu1mps.so`` behind the C ABI of ``include/u1mps.h``;
``binding`` is its ctypes wrapper.
"""
from .binding import MPS, MPSError, TorchDevice, apply_batch, lib  # noqa: F401
