"""Physical constants (SI) used to synthesise inputs.

Exact SI definitions where they exist; the electron mass is CODATA 2018.  The
solar rotation rate is the one the paper uses for its wind model (Sect. 2.1:
one turn in 30 days); wind speed and field strength are those of the analytic
Parker spiral that stands in for the paper's MHD wind.
"""
import math

C_LIGHT = 299_792_458.0            # m/s (exact)
E_CHARGE = 1.602176634e-19         # C (exact)
M_ELECTRON = 9.1093837015e-31      # kg (CODATA 2018)
AU = 1.495978707e11                # m (exact, IAU 2012)
DAY = 86_400.0                     # s
OMEGA_SUN = 2.0 * math.pi / (30.0 * DAY)   # rad/s, Sect. 2.1
V_WIND = 4.0e5                     # m/s, radial wind of the Parker field
B0_1AU = 5.0e-9                    # T, radial field at 1 AU
KEV = 1.0e3 * E_CHARGE             # J
