"""MI355X space-time sparse-grid solver for the linear wave equation.

HIP/gfx950 implementation of the combination technique of Ferrari, Moiola,
Perinati, Perugia ("A space-time sparse-grid method for the wave equation"):
one coercive space-time Galerkin solve per combination index on the two
diagonals jx + jt = L and L-1, prolonged to the finest grid and combined with
+/-1 (eq. 19), plus its adjoint.  The C ABI is declared in include/sgwave.h;
this package only marshals torch tensors into it.
"""

from .binding import (SparseGridWave, SparseGridBatch, SGWaveFunction, SGError, sgwave,  # noqa: F401
                      host_pencil, host_pencil_2d, host_time_fdm, host_taps, host_time_level,
                      host_time_chunks, lib,
                      tuning_status,
                      LIB_PATH)
