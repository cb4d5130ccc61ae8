"""FP64 CPU oracle for the blockBP surface-code decoder (Kaufmann & Arad, arXiv 2402.04834).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct NumPy re-statement of what the
decoder computes. It is imported only by `tests/`, by `__graft_entry__.smoke()` and by the `cpu_baseline`
leg of `bench.py`; the GPU product path never imports, links or calls it, and it shares no code with the
HIP library (not even geometry helpers).

Modules
  lattice  -- surface-code geometry, the Pauli f_s that produces a syndrome, the four logical cosets
              (Sec. II.B; Alg. 1 first two steps)
  network  -- the coset tensor network T_s(L) of size (2d-1) x (2d-1), bond dimension 2 (Sec. III.A,
              Fig. 1) and its exact contraction by column transfer
  mps      -- matrix-product-state tools: canonical forms, QR + truncated-SVD compression, overlaps,
              direct sums (the boundary-MPS machinery of Sec. III.A)
  blockbp  -- block partition, MPS-message belief propagation with the two-colour schedule, damping and
              convergence distance, the Bethe estimate of Lemma 3.1, and the decision rule (Sec. III.C-E,
              Alg. 1 and its remarks)
  bmps     -- boundary-MPS contraction of a whole coset network with bond dimension chi: the single-block
              limit of blockBP and the paper's chi = 16 accuracy reference (Sec. III.A, III.D, IV)

Every floating-point quantity is float64. Shapes carry an arbitrary leading batch ("...") so that many
syndromes and cosets are processed by one NumPy call; no blocking, fusion or reordering beyond what the
paper states is applied.
"""
