"""MI355X-native modulated pyramid wavefront sensor (HIP kernels behind a C ABI).

The library libpwfs.so (built in-tree by build.py) holds every step of the
sensor path; this package only marshals arguments to it.  Loading fails
loudly when the library is missing or no device is present: there is no
CPU implementation behind these names.
"""
from ._lib import (PwfsError, Plan, PsfCamera, ShPlan, recon_apply, library_path, load_library,
                   STATUS_NAMES, config_struct)

__all__ = ["PwfsError", "Plan", "PsfCamera", "ShPlan", "recon_apply", "library_path", "load_library",
           "STATUS_NAMES", "config_struct"]
