"""Seeded synthetic inputs shared by the oracle and the HIP path.

Holds only input preparation: counter-based random numbers, geometries, the
synthetic H / V / three-center tensor, the mean-field eigenpairs and the
imaginary-time grids with their fitted transform weights.  None of the GW
method's arithmetic lives here.
"""
from . import philox, system, grids, configs  # noqa: F401
