"""Plain FP64 CPU oracle for the adaptively conditioned first-order conic solver.

TEST INFRASTRUCTURE ONLY.  This package is the parity authority for the GPU
solver.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does, and it shares no code
with the HIP library (the two meet only on the seeded inputs).

It follows the paper "Rapid Convergence of First-Order Numerical Algorithms
via Adaptive Conditioning" (Adil, Tavakkol, Madani, arXiv 2103.00736):

* `cones`    - proj_C and abs_C of Definition 1 for products of Lorentz cones
               (orthant coordinates are Lorentz cones of size one, Sec. II).
* `subspace` - the reflection abs through range((A O)^T) and the
               pseudo-inverse (A O)^dagger used in Algorithms 1 and 2.
* `alg2`     - Algorithm 2 step by step (Algorithm 1 is the case where the
               conditioning set is empty), with the conditioning of steps 5-14.
* `kkt`      - the primal/dual residuals, duality gap and cone distances
               used as stopping rule.
* `dr`       - textbook Douglas-Rachford splitting of Sec. III-A.1, used only
               as an independent pin of Algorithm 1.

Everything is float64 NumPy/SciPy.  Readings taken where the paper is silent
or garbled are listed in each function's docstring.
"""
