"""Physical constants for the oracle (CODATA 2018 SI definitions).

The paper fixes no numerical values for its constants (Sec. "Intensities and
partition function", after Eq. 2, defines c2 = hc/k_B); the reading taken here is
the exact 2019 SI values of h, c and k_B and the CODATA 2018 atomic mass constant.
"""
import math

H_PLANCK = 6.62607015e-34        # J s (exact)
C_LIGHT_SI = 299792458.0         # m/s (exact)
K_BOLTZMANN = 1.380649e-23       # J/K (exact)
AMU_KG = 1.66053906660e-27       # kg (CODATA 2018)
C_LIGHT_CGS = C_LIGHT_SI * 100.0 # cm/s
C2 = H_PLANCK * C_LIGHT_SI / K_BOLTZMANN * 100.0   # second radiation constant, cm K
LN2 = math.log(2.0)
T0_REF = 296.0                   # K, reference temperature of gamma_ref
P0_REF = 1.0                     # bar, reference pressure of gamma_ref

__all__ = ["H_PLANCK", "C_LIGHT_SI", "K_BOLTZMANN", "AMU_KG", "C_LIGHT_CGS", "C2",
           "LN2", "T0_REF", "P0_REF"]
