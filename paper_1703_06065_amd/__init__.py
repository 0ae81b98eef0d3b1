"""Block CUR hot path on AMD Instinct MI355X (gfx950).

The computation lives in the HIP library ``libbcur.so`` (sources in
``csrc/``, C ABI in ``include/bcur.h``); ``binding`` is its ctypes wrapper.
"""
from .binding import BcurError, Context, Server, load_library  # noqa: F401

__all__ = ["Context", "Server", "BcurError", "load_library"]
