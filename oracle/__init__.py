"""FP64 CPU oracle for incremental matrix-power views.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path;
both sides take their inputs from the separate `synth` generators.

Every function cites the passage of the LINVIEW paper (Nikolic, ElSeidy,
Koch, "LINVIEW: Incremental View Maintenance for Complex Analytical
Queries", arXiv 1403.6968) that it follows.  All arithmetic is float64.

Pins (what fixes each function other than itself) are in
`tests/test_oracle_pins.py` (powers), `test_oracle_sums.py`,
`test_oracle_general.py` (general form: exponential, skip-s and linear
models), `test_oracle_models.py` and `test_oracle_ols.py`; every function
here is pinned, none is "parity unpinned".
"""

from .linview_oracle import (  # noqa: F401
    levels,
    reeval,
    incr_factors,
    incr_update,
    apply_updates,
    power_rows,
    power_cols,
    brute_power,
    chain_residuals,
    maxrel,
    deltarel,
    OpCounter,
)
from .sums_oracle import (  # noqa: F401
    reeval_sums,
    incr_sums_factors,
    incr_update_sums,
)
from .general_oracle import (  # noqa: F401
    iterate_general,
    reeval_general,
    incr_update_general,
    incr_general_factors,
    incr_update_general_factored,
    skip_indices,
    reeval_general_skip,
    incr_general_factors_skip,
    incr_update_general_factored_skip,
    reeval_general_lin,
    incr_update_general_hybrid_lin,
    incr_update_general_factored_lin,
)
from .models_oracle import (  # noqa: F401
    model_steps,
    stored_powers,
    reeval_model,
    incr_model_factors,
    incr_update_model,
    paper_cost,
)
from .ols_oracle import (  # noqa: F401
    reeval_ols,
    ols_delta_z,
    sherman_morrison,
    incr_update_ols,
)
