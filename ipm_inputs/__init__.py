"""Seeded synthetic IPM-shaped linear systems (inputs only; no solver arithmetic)."""
from .gen import (System, streams, contiguous_blocks, a_pattern, log_uniform, normal_equations,
                  ada_system, c1, c2, c3, bbd_system, IPMSequence, c5_requests, c5_system,
                  poisson_arrivals, cache_dir)
