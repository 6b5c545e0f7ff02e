"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package holds none of the method's arithmetic: only the transfer
functions (beams and priors), inverse-noise maps and problem sizes that stand
in for the paper's Planck workloads, which are not available.
"""
