"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package draws and stores inputs only: it holds none of the method's
arithmetic (no loss, regulariser, prox, dual or solver code), so the oracle
and the HIP path can both consume its bytes without sharing any computation.
"""
from .synthetic import (Instance, make_instance, make_nodes, round_bf16, bf16_to_f32,  # noqa: F401
                        CONFIGS, config_instance)
