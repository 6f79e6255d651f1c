"""MI355X (gfx950) implementation of the GL-ECSIM particle pass with the
comoving-frame current and the limited Lax-Friedrichs field diffusion of
Chen, Zhou & Toth (arXiv 2506.11320).  The compute path is the HIP library
libglecsim.so; ``glecsim`` is its thin Python binding."""
from .glecsim import (GE_A_BULK, GE_A_LIGHT, GE_BC_INFLOW, GE_BC_PERIODIC, GE_BC_WALL, GE_FP32, GE_FP64, GE_HARVEST_KRYLOV, GE_HARVEST_SOLUTION,  # noqa: F401
                      GE_LAG_EN, GE_PC_CNN, GE_PC_JACOBI, GE_PC_NONE, GE_PICARD1, GlecsimError,
                      Simulation, load_library)
