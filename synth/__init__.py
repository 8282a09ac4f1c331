"""Seeded synthetic inputs shared by the HIP path's tests and the FP64 oracle.

This package holds configuration records and input generators only
(phase screens, frozen-flow sequences, the DM modal basis).  It contains
none of the pyramid sensor's arithmetic: no Fourier optics, no mask, no
slopes, no reconstructor.
"""
