"""CPU oracle for the extrapolated GBS macro step (Ellison & Fornberg,
"A parallel-in-time approach for wave-type PDEs").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 (and exact
rational) reference written from the paper.  Only ``tests/``, the smoke check
and the ``cpu_baseline`` leg of the benchmark may import it.  The GPU library
never calls into it and shares no code with it.

Modules
-------
weights    -- order-constraint (Vandermonde) weights, square and dep/free split
stability  -- per-sequence stability polynomials P_N, R = sum c_i P_i, exact ISB
optimize   -- App. B imaginary-axis optimiser (bisection over a convex minimax LP)
operators  -- periodic centred finite-difference RHS operators (FD4, FD8)
gbs        -- the literal GBS macro step (FE, leap-frog, averaging, combine)
spectral   -- closed-form fully discrete propagator for constant coefficients
adjoint    -- the discrete adjoint of the macro step and the receiver misfit
"""
