"""FP64 CPU oracle for the narrow capture / narrow escape solver (Kaye & Greengard).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously correct
restatement of the paper's method, used to check the GPU library. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
it. The library never imports it and shares no code, tables or constants
with it; the two meet only through the seeded inputs of `layouts`.

Modules
  greens      sphere Neumann Green's functions (Section 2.1)
  zernike     scaled Zernike basis, sampling nodes, discrete transform P (Section 4)
  onepatch    one-patch modal integral equation solver -> B, fine grid, weights, I
              (Sections 5 and 9)
  idcomp      interpolative decomposition of the outgoing field -> T, skeleton
              (Section 7.1)
  system      frames, dense compressed / uncompressed system, GMRES, scalars
              (Sections 3, 6, 8)
  tables      per-(problem, eps) precompute driver and on-disk cache
  csum        plain C all-pairs Green's sum used for the larger dense matvecs
  mlp         FP64 reference MLP (forward, backward) for the learned warm start

Parity-unpinned functions are listed in each module header.
"""
