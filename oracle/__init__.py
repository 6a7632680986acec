"""Plain FP64 CPU oracle of the CSS density-matrix path. TEST INFRASTRUCTURE.

This package is the slow, obviously correct reference that the GPU library is
checked against. Only the test suite, smoke() in __graft_entry__.py and the
CPU-baseline leg of the benchmark may import or run it; the product
path (the HIP library and its Python binding) never does, and shares no code
with it. It is written from the paper (arXiv 2605.20918): every function cites
the equation or passage it follows and states the readings taken where the
paper is silent.

Modules:
  pattern   conflict graph of the colouring = sparsity pattern of P
  coloring  greedy Welsh-Powell multicolouring
  probes    +-1 CSS probe vectors, SplitMix64 signs, Q_1 and B_0
  lanczos   block Lanczos (Golub-Underwood) and the block-tridiagonal H^K
  subspace  Fermi function, exact diagonalisation, contraction F
  density   reconstruction X, extraction of P, trace, band energy, pipeline

Parity status: every function is pinned by the CPU tests (closed forms,
special cases that reduce to dense diagonalisation, Krylov polynomial
exactness, published SplitMix64 outputs, brute force on tiny inputs).
"""
