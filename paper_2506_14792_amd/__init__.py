"""MI355X-native spectral IMEX timestep and discrete adjoint (Python binding of libsps.so).

The compute path is the HIP library; this package only marshals arguments.  Importing it
does not load the library; the first call does, and fails loudly if it is missing.
"""
from .sps import (ClosureNet, Couette, Kolmogorov, PoiseuilleStability, Problem, RbcBatch, ShBatch, SpsError, lib,
                  poiseuille_host_band, rbc_host_bands,
                  use_torch_allocator, RBC2D, KS1D, SH2D, RK222, SBDF2,
                  SBDF3, SBDF4, RK443, CKPT_UNIFORM, CKPT_BINOMIAL, CKPT_TWO_LEVEL,
                  checkpoint_schedule, checkpoint_schedule_costs)  # noqa: F401
