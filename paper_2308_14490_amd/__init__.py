"""MI355X-native AZ least-squares solver for periodized Gaussian RBF
approximation and collocation (Zhou & Huybrechs).

The computation lives in ``libazrbf.so`` (HIP, gfx950); ``azrbf`` is its thin
Python binding and ``problems`` builds plans from workload descriptions.
"""
from . import azrbf  # noqa: F401
