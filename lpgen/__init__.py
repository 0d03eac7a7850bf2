"""Seeded synthetic LP workloads (inputs only; no solver arithmetic)."""
from .generators import (BASE_SEED, LP, Certificate, WORKLOADS, batched_lp, bernoulli_lp,
                         make, mixed_bounds_lp, ot_lp, pack_block_diagonal, qap_lp,
                         tiny_boxed_lp, transport_lp, zipf_lp)

__all__ = ["BASE_SEED", "LP", "Certificate", "WORKLOADS", "batched_lp", "bernoulli_lp", "make",
           "mixed_bounds_lp", "ot_lp", "pack_block_diagonal", "qap_lp", "tiny_boxed_lp",
           "transport_lp", "zipf_lp"]
