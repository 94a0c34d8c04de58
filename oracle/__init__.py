"""FP64 CPU oracle -- test infrastructure only (tests, smoke check, bench CPU baseline).

The product path never imports this package.
"""
from .chanflow_oracle import *  # noqa: F401,F403
from .chanflow_oracle import __all__  # noqa: F401
