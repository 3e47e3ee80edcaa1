"""FP64 CPU oracle for the perspective texture optimisation hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg import it.
It shares no code with the GPU path (no kernels, headers, helpers or tables);
the only common inputs are the seeded arrays of the synthetic generator.

Everything here is plain numpy in float64, written from the paper
(Bashir & Ghouri, "Perspective Texture Synthesis Based on Improved Energy
Optimization"): the texture energy and its robust form (Eqs. 4-8), the
EM-like alternation of a search phase and an optimisation phase, the sparse
grid at w/4, the 2x2 patch update, PCA before a k-means search tree
(Methodology, sections 2.1 and 2.2), and coarse-to-fine synthesis.  Where the
method reaches a result with a plain definition (exhaustive nearest
neighbour, weighted least squares), the oracle computes that definition;
where it approximates (PCA, the tree, BF16 distances, a learned proposal), the
oracle takes the approximation's steps in order.

Modules:
  vectors  - neighbourhood vectors and the two window grids
  exact    - exhaustive nearest neighbourhood search (Eq. 4's z_p)
  pca      - PCA basis and projection
  tree     - hierarchical k-means search tree, descent and leaf search
  irls     - robust energy, IRLS weights (Eqs. 5-8)
  mstep    - 2x2 patch blend (the optimisation phase)
  solve    - alternation, pyramid, upsampling, multiscale solve
  bf16     - BF16 distance form with top-k re-rank
  mlp      - leaf-proposal MLP forward/backward/Adam
  parity   - judging helpers for comparisons with the GPU library
"""
from . import vectors, exact, pca, tree, irls, mstep, solve, bf16, mlp, parity  # noqa: F401
