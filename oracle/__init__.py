"""FP64 CPU oracle of the FireANTs dense matching step.

Test infrastructure only: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  See ``fireants64`` (the
registration), ``inverse64`` (the post hoc inverse of a warp) and
``symmetric64`` (the symmetric registration).
"""
from .fireants64 import *  # noqa: F401,F403
from .fireants64 import __all__  # noqa: F401
