"""Seeded synthetic inputs for matrix-power views.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
holds only input generation (random matrices, update factors, update streams,
graph adjacency matrices); none of the view-maintenance arithmetic lives here.

Workload recipe (the paper's experiments use dense random matrices that are
"preconditioned" for stability and a stream of rank-1 updates, Sec. 7
"Workload"):

* A: i.i.d. N(0, 1/n) entries, rescaled so that its spectral norm is 0.9.
* Update factors U, V (n x r): i.i.d. N(0, sigma) with standard deviation
  sigma = 1e-2 / sqrt(n), so each rank-1 term u v^T has norm about 1e-4.
* Row updates (u = e_i) with Zipf-distributed row frequencies, as in the
  batch-update experiment (Sec. 7, Table 6).
* General form T_{i+1} = A T_i + B: T_0 ~ N(0, 1), B ~ N(0, 0.01) (n x p),
  and the gradient-descent regression of Sec. 7 (A = I - eta X^T X,
  B = eta X^T Y, new training rows as rank-1 changes of A).

Every generator draws from numpy's PCG64 seeded through a SeedSequence whose
spawn key names the stream (config id, view id, purpose), so the same
(seed, key) always gives the same values on every machine.
"""

from .gen import (  # noqa: F401
    rng,
    spectral_norm_estimate,
    gaussian_matrix,
    update_factors,
    row_updates,
    zipf_rows,
    random_dag,
    integer_matrix,
    round_to,
    general_operands,
    regression_problem,
    regression_rows,
    KEY_A,
    KEY_UPDATES,
)
