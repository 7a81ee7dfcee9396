"""Seeded synthetic LDU pressure systems on hexahedral boxes.

This package only *defines inputs*: face addressing, coefficients, boundary
terms and right-hand sides.  It holds none of the solver's arithmetic and is
imported by both the oracle's tests and the GPU path's tests and benchmark.
"""
from .boxes import (  # noqa: F401
    LduCase,
    box_faces,
    box_case,
    assemble_diag,
    relabel,
    rcm_order,
    random_order,
    config_case,
    c3_assembly_inputs,
    CONFIG_NAMES,
)
