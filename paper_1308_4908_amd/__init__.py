"""MI355X (gfx950) multi-sensor HDR reconstruction by local polynomial
approximation with ICI window selection (Kronander et al., arXiv 1308.4908).

The work runs in liblpa.so (HIP kernels behind a C ABI, include/lpa.h); this
package only marshals arguments (see ``lpa``).  Importing it does not load the
library; the first call does, and fails loudly if it is not built.
"""
from . import lpa  # noqa: F401
from .lpa import Context, LpaError, Rig  # noqa: F401
