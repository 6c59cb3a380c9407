"""Plain complex128 CPU oracle for the two-site MPS time-evolution update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP product
path (``paper_1703_00387_amd``) never imports it, and it never imports the
product path: the two share nothing except the seeded parameter generators in
``workloads``.

Everything here is written for readability against the paper (Jaschke, Wall,
Carr, "Open source Matrix Product States", arXiv:1703.00387): NumPy/SciPy in
complex128, LAPACK for SVD/eigh, no blocking or fusion.

Modules
-------
models      local operators, bond Hamiltonians, MPOs, dense H (Sec. Hamiltonians)
mps         Vidal/Hastings-form MPS, bond update with truncation, TEBD2/TEBD4,
            Sornborger-Stewart sweep, observables (Secs. Basic concepts,
            Sornborger-Stewart decomposition)
ed          state-vector references: exact propagation, exact Trotter circuit,
            reduced density matrices and the paper's error measures
freefermion single-particle propagation of the XX chain (exact and Trotterized)
krylov      Lanczos exponential (Sec. Krylov time evolution, App. Krylov)
tdvp        environments, structured H_eff apply, two-site TDVP (Sec. TDVP)
ktebd       Krylov TEBD: the Sornborger-Stewart sweep with the Lanczos
            exponential of every bond term (App. Details of the Krylov method)
timedep     time-dependent Hamiltonians: commutator-free Magnus expansions
            (midpoint rule, fourth-order two-exponential scheme) over Trotter steps
u1          U(1)-symmetric truncated SVD: blockwise SVDs, global count rule
            (App. Convenient features); TEBD of charge-carrying chains
grad        reverse-mode gradient of TEBD2 with truncated-SVD backward, the
            exact-diagonalisation adjoint gradient, finite differences
"""
