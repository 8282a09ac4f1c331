"""FP64 CPU oracle of the modulated pyramid wavefront sensor path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import,
call, link or execute this package; only the tests, the smoke check and
the CPU-baseline leg of the benchmark do.  It shares no code with the HIP
path: it takes the literal route (2-D FFT of the full N x N field per
modulation point, the 2-D pyramid mask, 2-D inverse FFT) and uses no
separable factorisation, no pruning and no precomputed tables.

Citations name the paper's sections: the sensor chain pyramid -> detector
-> slope computer -> modal reconstructor -> integrator is the processing
chain of the SCAO example (Sec. 4, main file, Tab. 2), with the
parameters of its "pyramid", "slopec", "modalrec" and "control" blocks
(Sec. 4, Tab. 1).  The paper prints no equations; the Fourier-optics
model implemented here is the textbook modulated pyramid, with every
convention the paper leaves open fixed as documented in each function.
"""
from .pwfs import (pupil_amplitude, valid_subapertures, modulation_offsets,
                   pyramid_mask, intensity, pupil_images, slopes, Oracle,
                   overlap_matrix, rebin, acquire_valid, field_stop_mask, sensor_mask)

__all__ = ["pupil_amplitude", "valid_subapertures", "modulation_offsets",
           "pyramid_mask", "intensity", "pupil_images", "slopes", "Oracle",
           "overlap_matrix", "rebin", "acquire_valid", "field_stop_mask", "sensor_mask"]
