"""FP64 CPU oracle of the matrix-probing hot path.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  Shares no code with the
HIP path; only the seeded input generators in ``fixtures`` feed both.
"""
from .wave import Problem, ricker, laplacian, cfl_limit, FD8  # noqa: F401
