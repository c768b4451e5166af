"""CPU oracle for the 4-point homography hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations written from the
paper (Cai et al., "Fast and Interpretable 2D Homography Decomposition:
Similarity-Kernel-Similarity and Affine-Core-Affine Transformations",
arXiv 2402.18008). Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package. The HIP library never calls into it and
shares no code with it.

Modules
  homography  DLT (plain definition, exact and FP64), ACA (structured product
              form, literal matrix form, corrected polynomial form), SKS,
              rectangle ACA (Algorithm 1), affine ACA, degeneracy flag,
              power-of-two scaling, comparison metric
  flops       a counting number type (Livermore convention) for FLOP pins
  sampling    Philox4x32-10 and Floyd subset sampling
  ransac      hypothesise-and-verify reference and brute force
  warp        4-point-offset -> homography -> bilinear warp -> L1 reference in
              torch float64 (autograd through DLT) plus finite differences

Every function is pinned by a ``-m "not gpu"`` test against exact arithmetic,
invariants, special cases, brute force or a library routine. The sampler's
mapping from Philox words to point indices is this implementation's own
choice: it is pinned by the published Philox known-answer vectors, brute force
over every Floyd outcome for small N, and distinctness and uniformity, and has
no external reference beyond those.
"""
