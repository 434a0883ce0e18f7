"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package generates *inputs only*: point clouds on analytic surfaces,
parameter blobs, regression targets and partition sizes.  It holds none of
the method's arithmetic (no kNN, no message passing, no loss); both the oracle
and the GPU library take what it produces as given.

All randomness is drawn from ``numpy.random.Generator(PCG64(seed))``.
"""
from .geometry import sphere, bumpy_ellipsoid, car_body
from .configs import CONFIGS, Config, make_inputs, partition_sizes, init_params

__all__ = ["sphere", "bumpy_ellipsoid", "car_body", "CONFIGS", "Config",
           "make_inputs", "partition_sizes", "init_params"]
