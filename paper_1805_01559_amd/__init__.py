"""MI355X-native entropy-regularised OT device association.

The solver is the HIP library ``libot_assoc.so`` (C ABI in include/ot_assoc.h);
``ot_assoc`` is its ctypes binding. Importing this package does not load the
library; the first call does, and raises if it has not been built.
"""

from . import ot_assoc  # noqa: F401
