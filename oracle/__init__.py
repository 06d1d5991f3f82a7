"""CPU oracle for exact-reduction pipelined BiCGStab -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct implementations of what the GPU path computes,
written from the paper (Havdiak, Aliaga, Iakymchuk, "Robustness and Accuracy in
Pipelined Bi-Conjugate Gradient Stabilized Method"):

* ``exact``   exact dot products rounded once (Section 2, the ExBLAS paragraph);
              tier 1, Python integers.
* ``spmv``    sequential CSR row sums (the A.x of Algorithms 1 and 2).
* ``solvers`` BiCGStab (Algorithm 1), p-BiCGStab (Algorithm 2) in FP64 with exact
              dots, the FP32-inner / FP64-refinement driver and right
              preconditioning.
* ``rational`` the same two algorithms over ``fractions.Fraction``.
* ``ctier``   tier 2: the same exact dot / SpMV / solvers in plain C + OpenMP
              (``oracle/c/oracle.c``), bit-identical to tier 1, used where the
              Python tier is too slow and as the timed CPU baseline.
* ``spai``    learned sparse-approximate-inverse pieces (features, MLP, loss,
              gradients, Adam, bf16 inference emulation) in float64/float32.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and never imports
it; the only common dependency is the seeded input generator ``synthgen``.
"""
