"""Seeded synthetic discrete Bayesian-network data.

This package only draws inputs: a random DAG, cardinalities, Dirichlet CPTs and
forward-sampled rows stored as uint8 columns (one contiguous row per variable,
the transposed storage of the paper's Section IV-C).  It holds none of the
structure-learning arithmetic (no counting, no statistics, no PC-stable logic),
so both the CPU oracle and the GPU path can take their inputs from it.
"""

from .generate import (  # noqa: F401
    CONFIGS,
    Dataset,
    forward_sample,
    make_config,
    make_dataset,
    random_dag,
)
