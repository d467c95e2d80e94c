"""Space-time Petrov-Galerkin heat solver for MI355X (gfx950).

Solves Kx U Mt^T + Mx U Dt^T = F1 F2^T -- the matrix form of the space-time
Petrov-Galerkin discretisation of the heat equation -- by Galerkin projection
onto an extended Krylov space, returning low-rank factors U ~= V Y.  All
computation runs in the HIP library ``libsts.so`` behind the C ABI of
``include/sts.h``; ``binding`` is its ctypes marshalling layer.
"""
from .binding import (  # noqa: F401
    EXPORTED, STS_FE_P1_1D, STS_FE_P1_2D, STS_FE_Q1_3D_7PT, STS_OP_K, STS_OP_M, Pool, Problem,
    Server, adaptive_shift, footprint, shifted_solve,
    STSError, apply_op, basis_update, cg, default_opts, gram, load, m_orthonormalize, make_space,
    mass_solve, mg_vcycle, pcg_mg, pcg_mg_mixed, pcg_mg_refined, release_cached_memory, sym_eig,
    time_matrices, time_sweep, tridiag_solve,
)
