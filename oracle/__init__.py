"""CPU oracle of the PPL hot path (test infrastructure only; see ppl_oracle.py)."""
from .ppl_oracle import *  # noqa: F401,F403
from . import mlp_oracle  # noqa: F401,E402
from . import precision_oracle  # noqa: F401,E402
