"""FP64 CPU oracle (test infrastructure only): see oracle.oracle."""
from .oracle import *  # noqa: F401,F403
from .oracle import Op, build, FLOPS_HOP, FLOPS_WILSON, FLOPS_DWF  # noqa: F401
from . import eo  # noqa: F401,E402
from . import mobius  # noqa: F401,E402
from . import hmc  # noqa: F401,E402
from . import mg  # noqa: F401,E402
