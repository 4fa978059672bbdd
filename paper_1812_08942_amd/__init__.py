"""MI355X (gfx950) implementation of the spectrum-preserving node
aggregation of Zhao, Wang & Feng, arXiv 1812.08942 (Phase A, Sec. 3.2),
behind the C ABI of include/graphreduce.h."""
from . import graphreduce  # noqa: F401
from .graphreduce import DeviceGraph, gr_reduce  # noqa: F401
