"""MI355X-native normal operator of the acoustic wave equation and its probed inverse.

Operators (Demanet et al., matrix probing of the wave-equation Hessian):
``Problem.apply_F`` (demigration), ``Problem.apply_Fadj`` (migration),
``Problem.apply_H`` (normal operator F*F), ``probe_fit`` (least-squares fit of
the inverse-Hessian symbol coefficients), ``apply_Hinv`` (fast application of
the fitted series), ``Problem.model`` (nonlinear modelling).  Around them:
``inversion`` (steepest descent, preconditioned CG, Kn fits, Gauss-Newton),
``curvelets`` (curvelet-space trial functions and the ray-traced illumination mask),
``study`` (the generalization study), ``autograd`` and ``serve``.  All compute runs in
the HIP kernels of libmatprobe.so.
"""
from .problem import Problem, Basis, probe_fit, apply_Hinv  # noqa: F401
from ._lib import MatprobeError, lib  # noqa: F401
