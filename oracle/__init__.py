"""FP64 CPU oracle for the energy-stable Allen–Cahn/Cahn–Hilliard scheme (2.20).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything here; only tests, the smoke
check and the benchmark's CPU-baseline leg do.  The oracle shares no code with
the HIP path.

Contents (each function cites the passage of the paper it follows):

* scheme      — the discrete operators, the truncated-series discrete variational
                derivative G^S (Lemma 2.2, eq. D2-1), the residual of scheme
                (2.20), the discrete energy (eqs. relations/freeenergy) and mass.
* scalar      — an independent cell-by-cell residual written with explicit loops,
                for tiny grids and sampled cells.
* jacobian    — the analytic Jacobian of the residual as a sparse matrix,
                composed from the same difference operators.
* newton      — inexact-Newton step solve (Section 3.1) with a sparse direct
                linear solve and a backtracking line search.
* controller  — adaptive time stepping (eq. sencondt with the sqrt(2) retry and
                eta doubling of Section 3.2).
* schwarz     — overlapping decomposition, subdomain matrices A_k = R J R^T,
                textbook ILU(0) and the additive Schwarz family (eq. invM and the
                restricted variants) for preconditioner parity.
* adjoint     — discrete adjoint of the time-step map (transpose solves).

Parity status per function is listed in each module header.
"""
