"""MI355X (gfx950) total convolution by the reduced-Wigner l-recursion.

The computation lives in libtotalconv.so (HIP kernels behind the C ABI of
include/totalconv.h); this package is its Python face:

* ``wigner_d_rings``, ``totalconv_fwd``, ``totalconv_adj`` (on colatitudes) and their
  ``_x`` twins (on ring cosines): thin ctypes wrappers with the C entry points' names
  (``_binding``);
* ``TotalConv`` / ``totalconv`` (``TotalConvX`` on ring cosines): a
  ``torch.autograd.Function`` whose backward is the hand-written adjoint kernel;
* ``synthetic``: seeded input generators (rings, skies, beams).

Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
from . import synthetic  # noqa: F401
from ._binding import (  # noqa: F401
    TC_OP_ADJ, TC_OP_FWD, TC_OP_WIGNER, TotalConvError, lib, rings_from_beta, totalconv_adj, totalconv_adj_x,
    totalconv_fwd, totalconv_fwd_x, wigner_d_rings, wigner_d_rings_x, workspace_bytes, workspace_bytes_x,
)


def __getattr__(name):
    if name in ("TotalConv", "totalconv", "TotalConvX", "TotalConvPol", "TotalConvPolX"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
