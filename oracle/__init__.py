"""Plain FP64 CPU oracle for the parallel infinite-size DMRG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its Python
binding and driver) may import, call, link or execute anything in this
package; only the test suite, the smoke check and the CPU-baseline leg of the
benchmark do.  The oracle shares no code with the GPU path: its only
dependency inside this repository is ``workloads`` (seeded inputs, no method
arithmetic).

It follows H. Ueda, "Infinite-Size Density Matrix Renormalization Group with
Parallel Hida's Algorithm" (arXiv 1606.06790) step by step:

* ``mpo``      finite-state MPO of the Heisenberg models (Sec. 2, Eq. (1); Sec. 3, Eq. (7))
* ``ed``       sparse exact diagonalisation of open segments (the untruncated pin)
* ``dense``    the hot-path steps on full tensors, no symmetry blocks (Sec. 4: the
               paper's own runs use no quantum-number blocks)
* ``u1``       the same steps inside U(1) S^z blocks
* ``lanczos``  Lanczos with full re-orthogonalisation (Step 3)
* ``layout``   the canonical flat storage order shared with the C-ABI (a
               specification, implemented here independently)
* ``idmrg``    the parallel iDMRG driver (Steps 1, 2', 3', 4, 5', 6)

Every floating-point operation is IEEE double precision.
"""
