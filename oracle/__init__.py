"""CPU binary64 oracle of the single-pass online randomized ID.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the HIP
library in ``paper_2405_16076_amd`` and imports nothing from it; the two meet
only through the seeded input generators in ``synth``.
"""
from .philox import philox4x32, philox4x32_scalar, decision_uniform, seed_key, PRUNE_DRAW  # noqa: F401
from .omega import (omega_block, omega_bound, omega_entry_scalar, omega_table, quantize_fp8_blocks,  # noqa: F401
                    quantize_fp8_omega, round_to_bf16, round_to_e4m3)
from .rid import (Config, OnlineRID, UpdateRecord, basis_gram, coeff_alg4, fill_factor,  # noqa: F401
                  nahutchpp, pinv, ridge_lambda, ridge_scores, select_slots, sketch_columns)
from .exact import exact_error, exact_ls  # noqa: F401
