"""Seeded synthetic inputs for the Newton-step KKT solve.

This package only draws sparsity patterns and random values. It holds none
of the method's arithmetic (no assembly, no factorisation, no solve), so the
oracle under ``oracle/`` and the HIP library can both be fed from it without
sharing any numerical code.

Every draw goes through ``rng_for(config, instance, value_set)``, a NumPy
``SeedSequence([240315913, config, instance, value_set])``, so each instance
and each value set is reproducible on its own.
"""
from .nmpc import (  # noqa: F401
    SEED_ROOT, Pattern, Values, rng_for, log_uniform,
    nmpc_pattern, nmpc_values, distillation_pattern, distillation_values,
    dyadic_nmpc_values, batch_shapes, serving_shapes, poisson_arrivals, hub_pattern, hub_values,
    general_pattern, general_values,
    workload, small_config, paper_config, hykkt_config,
)
