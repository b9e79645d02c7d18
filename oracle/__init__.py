"""CPU oracle for Gaussian-mixture interpolation -- test infrastructure only.

Only the test-suite, the package's smoke check and the benchmark's CPU-baseline
leg import this package.  The product path never does.
"""
from .gmm_oracle import *  # noqa: F401,F403
from .gmm_oracle import default_workers  # noqa: F401
from . import gmm_variants  # noqa: F401,E402
