"""FP64 CPU oracle for refined template matching (Foden, Collins, Wilkinson &
Britton, "Indexing Electron Backscatter Diffraction Patterns with a Refined
Template Matching Approach", arXiv 1807.11313).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct definition that the HIP path is checked against.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path (``paper_1807_11313_amd``)
never does, and the two share no code.  Inputs come from ``fixtures``
(seeded generators that hold none of the method's arithmetic).

Modules, each citing the paper passage it follows:

* ``rotations``  quaternions, the 24 cubic operators, disorientation
  (section "SO(3) Spacing", the disorientation equation).
* ``geometry``   detector geometry, gnomonic template projection with bicubic
  interpolation of the master pattern (section "SO(3) Library Generation";
  the pattern-centre footnote of section "Fast Fourier Transform").
* ``spectra``    contrast normalisation, windowing, unitary 2-D DFT
  (Equation 4), band-pass filtering, energies.
* ``xcf``        cross-correlation map (Equations 2, 3 and the spatial
  definition of r_fg), normalisation by the autocorrelations, integer
  peak, library argmax, upsampled sub-pixel peak (Equation 5).
* ``refine``     orientation refinement: x/y from the shift (Equation 7,
  shift over detector distance), z from the log-polar transform, iterated
  (section "Orientation and Pattern Centre Refinement").
* ``pipeline``   ``index_patterns`` and ``refine_orientations``, the two
  calls of the C-ABI, composed from the steps above.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""

from . import rotations, geometry, spectra, xcf, refine, pipeline  # noqa: F401
from .params import Params  # noqa: F401
