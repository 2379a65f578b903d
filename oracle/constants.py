"""Vacuum constants of the oracle (SI).  TEST INFRASTRUCTURE ONLY (see oracle.py).

c is exact by the definition of the metre; mu0 takes its classical value
4 pi 1e-7 H/m; eps0 = 1 / (mu0 c^2).  The paper writes its examples in units
with eps = mu = 1 (Section 4.1); these are the values of the SI runs.
"""
import math

C0 = 299792458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
