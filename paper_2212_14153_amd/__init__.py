"""MI355X-native time step of the fluid-particle-dynamics fiber method (arXiv:2212.14153).

The compute path is the HIP library ``libfpdlbm.so`` (C ABI in ``include/fpdlbm.h``);
this package holds its sources (``csrc/``), the build script and a thin ctypes binding.
"""
from ._lib import (  # noqa: F401
    FPD_BF16DEV, FPD_F16DEV, FPD_F32, FPD_F64, FPD_FLAG_CLAMP_PHI, FPD_FLAG_NO_GRAPH,
    FPD_FLAG_TIME_KERNELS, FPD_INIT_LINEAR_COUETTE, FPD_INIT_REST, Batch, FpdError,
    LaunchConfig, Simulation, check, fpd_copy_probe, fpd_params, fpd_params_default,
    fpd_params_from_physical, fpd_population_bytes, lib, params_from_mapping,
    simulation_from_workload,
)
