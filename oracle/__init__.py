"""CPU FP64 oracle (test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  The library never imports it, and it
imports nothing from the library.
"""

from .xpcs_oracle import *  # noqa: F401,F403
from . import xpcs_oracle  # noqa: F401
