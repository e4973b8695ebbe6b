"""Seeded synthetic rulesets and traffic for the first-match classifier.

This package only draws random inputs.  It holds none of the classifier's
arithmetic and is shared, unchanged, by the CPU oracle's tests and by the GPU
path's tests and benchmark, so both sides always see identical arrays.
"""

from .gen import (  # noqa: F401
    SEEDS,
    Packets,
    Ruleset,
    concat_rulesets,
    make_packets,
    make_rules,
    workload,
    multichain_workload,
    serving_chains,
    serving_arrivals,
)
