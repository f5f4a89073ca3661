"""MI355X-native MDLG: Lennard-Jones MD coarse-grained on the fly into the
Molecular-Dynamics lattice gas of Parsa & Wagner.

The computation lives in ``libmdlg.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/mdlg.h``); this package only marshals arguments.
"""
from .native import (MdlgError, System, autotune, describe, library_path, load,  # noqa: F401
                     make_config, workspace_bytes)
