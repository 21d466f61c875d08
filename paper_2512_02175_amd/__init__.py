"""MI355X (gfx950) timestep-splitting Euler-Maruyama particle step on metric
graphs (Dwaraknath & Ying, "Sampling on Metric Graphs").

The compute lives in libmetricgraph.so (HIP, C ABI in include/metricgraph.h);
``binding`` exposes it to Python under the same names.
"""
from . import binding  # noqa: F401
from .binding import *  # noqa: F401,F403
