"""Plain FP64 CPU oracle for the mode-k tensor-vector contraction (TVC) and the
higher-order power method (HOPM) of Martinez-Ferrer, Yzelman and Beltran,
"Distributed and heterogeneous tensor-vector contraction algorithms for high
performance computing" (FGCS 2025, arXiv 2501.03121).

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product path (the HIP
library and its Python binding) never imports, links or calls anything here, and
nothing here imports the product.  The two sides share only seeded input
generators, which hold none of the method's arithmetic.

Modules
  tvc    -- the k-mode contraction from its definition (Sec. 3), brute force,
            sampled single outputs for very large tensors.
  hopm   -- canonical Gauss-Seidel HOPM (Sec. 3), Algorithm 1 (dHOPM_3) at one
            process as a schedule model, and the streamed-memory model Eq. (3).
  quant  -- bit-level storage formats: bf16 (round-to-nearest-even and
            truncation), IEEE binary16, OCP FP8 E4M3 with per-slab scales.
  grad   -- adjoints of the contraction and a hand-written reverse pass through
            unrolled HOPM sweeps.

Every function computes in float64 from the exact upcast of its inputs.
"""
from . import tvc, hopm, quant, grad  # noqa: F401
