"""ProbeWalk on MI355X (gfx950): HIP kernels behind a C ABI.

The product is ``libprobewalk.so`` (``csrc/``, declared in
``include/probewalk.h``); ``binding`` is its ctypes binding. Importing this
package does not load the library; ``binding.lib()`` does, and raises if the
library has not been built.
"""

from . import binding  # noqa: F401
from .budgets import BUDGETS, budget_policy  # noqa: F401
