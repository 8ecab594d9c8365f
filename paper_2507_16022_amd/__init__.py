"""MI355X (gfx950) hot path of sampler-free GW inference by matrix products
(arXiv:2507.16022): the distance- and phase-marginalised likelihood of every
(bank waveform, extrinsic sample) pair and the evidence, behind the C ABI of
include/dotpe.h.  `dotpe` is the Python binding."""
from . import dotpe  # noqa: F401
