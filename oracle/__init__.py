"""FP64 CPU oracle for entropic W1 on non-uniform meshes (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import, call, link or execute anything in this package. The product path
(the HIP library and its Python binding) never touches it and fails loudly when
its own extension is missing.

Contents
  dense         NumPy definitions: the kernel matrix, the dense log-domain
                kernel-vector product, dense Sinkhorn with Algorithm 1's loop
                semantics (1D) and Algorithm 2's (2D), the transport cost.
  closed_form   closed-form 1D W1 (integral of |F_mu - F_nu|), brute-force LP,
                monotone coupling, Shannon entropy.
  clib          plain-C versions (built with gcc): dense products and costs
                for larger sizes, the dividing index and vector representation
                of Theorems 2.1/2.2 with instrumented operation counts, and
                Algorithms 1 and 2 with the eq. (p-DP)/(q-DP) recurrences in
                log form.

Shares no code with the HIP path; both sides only consume the seeded arrays
from ``paper_2605_26659_amd.workloads``.
"""
