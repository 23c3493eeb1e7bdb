"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only *generates inputs*: scanner geometry descriptions, ellipse and
ellipsoid phantoms, an attenuation map, noisy Poisson sinograms made from
closed-form line integrals of those continuous phantoms, and subset index
sequences.  It holds none of the reconstruction method's arithmetic (no system
matrix, no projection with it, no EM ratio, no update), so neither side of a
parity test can borrow a step of the method from here.

The paper's own data (a BrainWeb brain slice and an XCAT torso) are not
available; these seeded phantoms stand in for them with the sizes, count
levels and background fractions of the workloads described in the docs.
"""

from .phantoms import (  # noqa: F401
    Geometry,
    Problem,
    make_problem,
    make_multislice_problem,
    make_order,
    scanner_requests,
    serving_requests,
    CONFIG_SMALL,
    CONFIG_HEADLINE,
    CONFIG_MULTISLICE,
)
