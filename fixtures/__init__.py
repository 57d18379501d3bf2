"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds workload parameter records and input generators only; none of the
method's arithmetic lives here.
"""
from .configs import Workload, c1, c2, c3, c4, c4_union, c5, ALL, SERVE_SHAPES, SERVE_SHOTS, serve_steps  # noqa: F401
from .inputs import medium, wavepackets, trials, reflectivity, normal_field, tiny, bandlimited_data  # noqa: F401
from .rng import Stream, splitmix64  # noqa: F401
