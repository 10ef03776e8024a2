"""FP64 CPU oracle for the randomized sketching hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the C-ABI library and its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is written from the paper (S. Wang, "A Practical Guide to
Randomized Matrix Computations with MATLAB Implementations", arXiv:1505.07570)
as plain, slow, obviously-correct numpy in float64:

* ``rng``      - the counter-based random-number contract (Philox4x32-10,
                 published by Salmon et al., SC'11) and the derived signs,
                 bucket hashes, Feistel-permuted sample indices and Gaussians.
* ``sketch``   - the three sketching operators of Sec. 3.2 with the sketch
                 matrix S formed explicitly and C = S^T A as a dense product.
* ``rsvd``     - the prototype randomized k-SVD (Alg. 5.2) with the
                 subspace-iteration step of Alg. 5.1.
* ``lsr``      - sketch-and-solve least squares (eq. 4.2, Sec. 4.2) and the
                 exact solution of Sec. 4.1.
* ``nystrom``  - the RBF kernel (Sec. 6.1.1) and the Nystrom method (Sec. 6.4).
* ``mixed``    - BF16 / FP8 rounding and the per-column-scaled quantized
                 products of the mixed-precision subspace iteration.
* ``spsd``     - leverage scores and leverage-score sampling (Sec. 3.3.2), the
                 faster SPSD sketching of Alg. 6.1 (Sec. 6.3) and the faster
                 CUR decomposition (Sec. 6.6.3).

Inputs reach the oracle as the exact bits the GPU path sees (float32 data is
promoted exactly to float64).  Shared with the GPU path: nothing but the
seeded input generators in ``synth`` (which hold none of the method's
arithmetic) and the written RNG contract, which both sides implement
independently.
"""

from . import rng, sketch, rsvd, lsr, nystrom, mixed, spsd  # noqa: F401
