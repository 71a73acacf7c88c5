"""FP64 CPU oracle of the Evoformer block.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Shares no code with
the HIP implementation."""
from . import evoformer, sizes  # noqa: F401
