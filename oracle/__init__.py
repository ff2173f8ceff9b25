"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from .tlrmdd import *  # noqa: F401,F403
from . import tlrmdd  # noqa: F401
