"""FP64 CPU oracle for the fractal sphere tracer -- test infrastructure only.

Nothing in the GPU library imports this package.
"""
