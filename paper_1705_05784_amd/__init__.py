"""MI355X-native F-AMS pressure solver (hand-written HIP behind a C ABI).

`paper_1705_05784_amd.fams` is the ctypes binding of libfams.so;
`paper_1705_05784_amd.build` compiles it for gfx950.
"""
from . import fams  # noqa: F401
