"""Plain FP64 CPU oracle for the aTTN ground-state hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it, and it shares no code with the library: it reads the same
seeded problem arrays (from ``problems``) and computes everything itself with
NumPy / SciPy in float64.

Modules and the parts of the paper they follow:

* ``ed``     -- exact diagonalisation of the lattice Hamiltonian (sum of local
                terms, paper Sec. 3.3) and full-state helpers: the aTTN state
                D(u)|psi_TTN> (eq. 1) as a 2^N vector.
* ``tree``   -- binary tree tensor network structure (Sec. 3.1).
* ``terms``  -- disentangler layer contracted into every term, h' = U^T h U
                (Sec. 4.3, algorithm "Contract disentangler layer"; the state is
                D|psi_TTN>, so the rotated Hamiltonian is D^T H D and every term
                becomes U^T h U -- the paper also writes D H D^dagger, which spans
                the same variational class), and operator-Schmidt splits.
* ``davidson`` -- an eigensolver form that is not from the paper: the H_eff
                diagonal, Davidson's method with Jacobi or learned pointwise
                corrections, the exact Jacobi-Davidson correction, the MLP
                model, its gradient and Adam updates (published methods cited
                in the module).
* ``ttn``    -- isometric TTN, effective operators kept term by term
                (Sec. 3.3.2), the generalised matvec (Sec. 4.4.2), Lanczos,
                QR isometrisation (Sec. 3.1) and the sweep (Sec. 4).

Pins: every function is checked in ``tests/test_oracle_*.py`` against exact
diagonalisation, closed forms, brute-force dense effective Hamiltonians and
invariants, never against itself.
"""
