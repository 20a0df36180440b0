"""Seeded synthetic workloads (input recipes only).

This package draws the random inputs that the tests and the benchmark feed to
both the oracle and the HIP library: true galaxy properties, pixel noise,
stamp sizes, request arrival times.  It holds none of the inference method's
arithmetic (no rendering, likelihood, shear response or sampler), so a bug in
either implementation cannot be hidden by code the two share.
"""
from .gen import (CONFIGS, Truth, draw_truth, draw_noise, draw_requests, stamp_size_rule,
                  SIZE_CLASSES, data_seed, chain_seed)

__all__ = ["CONFIGS", "Truth", "draw_truth", "draw_noise", "draw_requests", "stamp_size_rule",
           "SIZE_CLASSES", "data_seed", "chain_seed"]
