"""Method parameters of the oracle (test infrastructure only).

The paper leaves the window, the band-pass filter, the upsampling factor and
the log-polar grid unspecified (section "Fast Fourier Transform": filters,
windowing and peak upsampling follow the HR-EBSD work it cites; section
"Orientation and Pattern Centre Refinement": log-polar transform, about two
iterations).  The defaults below are the readings used throughout:

* window: separable Hann, w_i = sin^2(pi (i + 1/2) / N);
* band-pass H(rho) = (1 - exp(-rho^2 / 2 s_hp^2)) exp(-rho^2 / 2 s_lp^2),
  cut to zero beyond rho_max; s_hp = 2 cycles/image, s_lp = N/8,
  rho_max = 3N/8 (so the spectrum is exactly zero outside a disc);
* sub-pixel upsampling factor kappa = 100 over a +-0.75 px box;
* log-polar grid N_rho = N/2 log-spaced radii in [2, N/2 - 2] px and
  N_eta = 2N angles about the screen centre;
* two refinement iterations, no early exit.
"""

from dataclasses import dataclass
import math


@dataclass
class Params:
    window: bool = True
    sigma_hp: float = 2.0          # cycles / image
    sigma_lp_frac: float = 0.125   # sigma_lp = frac * N
    rho_max_frac: float = 0.375    # rho_max = frac * N
    max_shift: int = -1            # -1: every cyclic shift is searched
    upsample: int = 100            # kappa
    n_iter: int = 2
    n_rho: int = 0                 # 0: N/2
    n_eta: int = 0                 # 0: 2N

    def sigma_lp(self, n):
        return self.sigma_lp_frac * n

    def rho_max(self, n):
        return self.rho_max_frac * n

    def band(self, n):
        """Half-width B of the square that holds the non-zero spectrum."""
        return int(math.floor(self.rho_max(n) + 1e-9))

    def nrho(self, n):
        return self.n_rho if self.n_rho > 0 else n // 2

    def neta(self, n):
        return self.n_eta if self.n_eta > 0 else 2 * n
