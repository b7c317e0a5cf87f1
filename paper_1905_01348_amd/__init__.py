"""libfock: MI355X-native Fock exchange (V_X) and ACE operators.

The compute path is the HIP library libfock.so (C ABI in include/fock.h);
this package is its ctypes binding plus the build script.
"""
from .fock import (  # noqa: F401
    PREC,
    Ace,
    Context,
    FockError,
    Server,
    debug_host_pair,
    load,
    make_cell,
    make_kernel,
)
