"""FP64 oracle: learned per-light transmittance field (placeholder until built).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
