"""B-TriRT lattice Boltzmann melting on MI355X (gfx950).

The hot path of Zhao, Wu, Chai & Shi (arXiv 1909.13086): a fused
collide-and-stream step of the block triple-relaxation-time update (Sec. 2,
Eq. (2)) for the total-enthalpy and Boussinesq flow populations of a D2Q9
lattice, in a cavity heated locally from below (Sec. 3.2).  The compute runs in
the hand-written HIP library ``liblbm.so`` behind the C ABI of include/lbm.h;
this package is its thin Python binding.  PyTorch is used only for device
memory and streams.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import LbmError, lib, make_case  # noqa: F401
from .context import Context  # noqa: F401
