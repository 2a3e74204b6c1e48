"""FP64 CPU oracle of the hybrid compressor's per-histogram hot path (test infrastructure).

This package is test infrastructure.  Only the test suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the HIP library and imports nothing from it.  Everything is plain NumPy in
FP64 (plus `math.fsum` for correctly rounded moment sums), written from the paper:

  grid      velocity grid, cell volumes, moment basis             (Section II, Eq. 1-4)
  moments   true moments b = A f and the four QoIs                (Eq. 1-4)
  ae        dense / tied-linear autoencoder forward+backward, MSE, Adam, z-score
                                                                  (Section III Stage 2-3, Eq. 5;
                                                                   Section IV-C)
  conv      convolutional autoencoder for 39 x 39 grids, BF16 form (Section III Stage 2)
  pq        per-dimension product-quantizer fit (1-D k-means) and encode
                                                                  (Section III Stage 3, IV-E)
  coder     multilevel residual coder with its bound search       (Section III Stage 4)
  newton    Lagrange / Newton projection restoring the moments    (Section III Stage 5, Eq. 6)
  pipeline  compress / decompress of a batch                      (Section III, Fig. 1)
  metrics   NRMSE and compression ratio                           (Eq. 7, Section IV-A)

Parity status: the moment, autoencoder, quantizer, coder and projection functions are
pinned by closed forms, library routines, brute force and invariants in the CPU tests.
Where the paper defers to works that are not available (the exact Stage-5 objective, the
MGARD coefficients, the PQ initialisation), the oracle follows a stated reading; its
agreement with the paper's own outputs is unpinned.
"""
from . import grid, moments, ae, conv, pq, coder, newton, pipeline, metrics  # noqa: F401
