"""FP64 CPU oracle for the mirror-symmetric Poisson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the test suite, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with
the GPU library: it is a plain, slow, FP64 restatement of the paper
(arXiv 2407.05930, "A multigrid reduction framework for domains with
symmetries") written with NumPy/SciPy primitives.

Modules
  splitmix   the counter-based hash used for all pseudo-random choices
  symmetry   Sec. 2: base blocks H_j, the change of basis Q_s, the decoupled
             subsystems (eqs. (2.4)-(2.14)) and Alg. 1
  amg        Sec. 3.2: strength, Alg. 2 populated coarsening, the reduction
             prolongation (eq. (3.13)), the block-FSAI top smoother
             (eq. (3.14)), the reduced operator (eq. (3.15)), standard AMG
             levels below it and the V-cycle of Alg. 3
  krylov     per-column PCG for the decoupled systems of Alg. 1
  lrc        Sec. 2.1/2.2: low-rank corrections (LRCFSAI(k), LRCAMG(k)),
             eigenpairs by Lanczos
  adjoint    gradient of 0.5||p - p*||^2 through the solve
  copies     Sec. 3 / 3.2 in the original basis: AMGR for a domain made of
             copies (interface of the copies, replicated Alg. 2 split)
  amgs       Sec. 3.1: the Schur-complement AMG (eqs. (3.2)-(3.12)) on the
             decoupled subsystems

Pins: each function is checked in ``tests/test_oracle_*.py`` against closed
forms, invariants, brute force or textbook routines.  Functions without
such a pin say "parity unpinned" in their docstring.
"""
