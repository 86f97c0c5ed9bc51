"""Seeded synthetic inputs for the EBSD template-matching hot path.

These generators stand in for the paper's data (a DynamicS master pattern,
silicon and alpha-iron maps, MTEX orientation libraries), none of which is
available.  They produce inputs only: a master pattern on an
equirectangular grid, orientation sets, and simulated experimental patterns.
Both the FP64 oracle and the HIP path consume these arrays; neither imports
anything else from the other, and nothing here implements a step of the
method (no gridded-master interpolation, filtering, correlation or
refinement).  Experimental patterns are rendered by evaluating the analytic
band model along each pixel ray (the forward model of the experiment),
which is a different route from the method's bicubic lookup of the gridded
master.
"""

from .master import band_master, band_intensity  # noqa: F401
from .orient import random_quats, fz_reduce, random_fz_quats, perturb_quats, voronoi_map  # noqa: F401
from .simulate import simulate_patterns  # noqa: F401
from . import configs  # noqa: F401
