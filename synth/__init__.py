"""Seeded synthetic inputs (meshes, per-cell fields, right-hand sides).

This package holds none of the corrector method's arithmetic: it only places
points, triangulates them and samples input fields, so that the CPU oracle
and the GPU library can be fed identical inputs.
"""
