"""MI355X-native IB-aware steady SIMPLE solver (HFDIB-RANS hot path).

The compute path is the HIP library ``libhfdib.so`` (include/hfdib.h); this
package only binds it.  See ``binding.Solver``.
"""

from .binding import (  # noqa: F401
    Solver,
    Batch,
    HfdibError,
    make_desc_config,
    default_config,
    lib,
    EXPORTED,
    LIB_PATH,
)
