"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

Holds workload descriptions (geometry, nuclei, orbital counts, pulse shape)
and seeded generators of orbital values and CI vectors.  It contains none
of the method's arithmetic: no quadrature, operator, solve or propagation.
"""
from .inputs import *  # noqa: F401,F403
