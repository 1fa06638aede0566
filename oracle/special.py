"""Modified Bessel functions of the second kind, K_n, used as black boxes.

The equation of state (eq. relativistic-eos), the normalisations of Sec. III.A
and the constants of Appendix A are written with K_1, K_2, K_3.  The oracle
calls scipy (float64, exponentially scaled to avoid underflow) on the lattice
and mpmath for init-time constants; neither is the GPU library's own code.
"""
import numpy as np
from mpmath import mp
from scipy.special import kve


def k_ratio_np(nu_num, nu_den, z):
    """K_{nu_num}(z)/K_{nu_den}(z) in float64 (scaled Bessel functions)."""
    z = np.asarray(z, dtype=np.float64)
    return kve(nu_num, z) / kve(nu_den, z)


def besselk_mp(n, x):
    return mp.besselk(n, x)
