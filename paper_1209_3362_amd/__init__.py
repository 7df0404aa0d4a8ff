"""MI355X (gfx950) structure function D(q, tau) of dynamic near-field scattering.

The compute path is the HIP library libnfs.so (C ABI in include/nfs.h);
this package only marshals arguments to it. Build it with
`python -m paper_1209_3362_amd.build`. Importing the binding does not need a
GPU; every compute call does, and fails loudly when the library is missing.
"""
from .nfs import (Plan, NfsError, load_library, library_path, status_name,
                  workspace_size, structure_function, Batch, batch_capacities, STATUS,
                  probe_bandwidth, structure_function_noalloc)

__all__ = ["Plan", "NfsError", "load_library", "library_path", "status_name",
           "workspace_size", "structure_function", "Batch", "batch_capacities", "STATUS",
           "probe_bandwidth", "structure_function_noalloc"]
