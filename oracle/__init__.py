"""FP64 CPU oracle for correlated-sampling phaseless AFQMC.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and
its Python binding) may import, call, link or execute anything here; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.  The
oracle shares no code with the HIP path: it reads its inputs from ``synth``
(seeded input generation only) and implements everything else itself, in
plain numpy/scipy float64, step by step in the paper's order.

Modules
-------
afqmc   the walker step: force bias (Eq. 8-9), HS propagator between one-body
        halves (Eq. 3, 4, 11), overlap ratio and phaseless weight (Sec. II.A
        and the hybrid weight of Sec. II.D), mixed local energy (Eq. 7, 10),
        modified Gram-Schmidt (Sec. II.D), correlated pairs (Sec. II.B);
        free-projection modes.
tangent forward-mode dE/dlambda of the mixed energy for h -> h + lambda V
        through a window of steps (the reference for the reverse-mode adjoint).
philox  Philox4x32-10 counter-based generator plus Box-Muller normals.
fci     dense determinant-space Hamiltonian for tiny systems (test pins).

Parity pins: see tests/test_oracle_*.py.  The phase-projection rule
max(0, cos(dtheta)) is a definition taken from Sec. II.A and is pinned only
by its own statement ("parity unpinned" beyond that definition); everything
else is pinned by dense FCI, closed forms or invariants.
"""
