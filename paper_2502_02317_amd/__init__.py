"""MI355X-native hot path of the PEPS branch-and-bound search for low-energy
states of generalized Potts/Ising models (SpinGlassPEPS, arXiv 2502.02317).

The computation lives in ``libspg.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/spg.h``); ``spg`` is its thin ctypes binding."""
from .spg import (SpgError, build_peps, boundary_mps, marginals, branch_and_bound,  # noqa: F401
                  env_info, env_export, env_import, load, pack_oracle_mps, unpack_mps, EXPORTS,
                  LIB_PATH, profile_enable, profile_reset, profile_query, KERNEL_CLASSES)
