"""Seeded synthetic workloads for the LP/QP problem form (min 1/2 x'Qx + c'x,
l_c <= Ax <= u_c, l_v <= x <= u_v).

This module only builds problem data. It holds none of the solver's arithmetic
and is shared by the CPU oracle, the tests and the benchmark. Every generator
takes an integer seed and draws from numpy's PCG64.
"""

from .lp import (  # noqa: F401
    LP,
    SharedBatch,
    csr_from_dense,
    dense_from_csr,
    planted_sparse_lp,
    large_zipf_lp,
    dense_planted_lp,
    dense_knapsack_lp,
    grid_incidence,
    grid_mincost_batch,
    shortest_path_learning,
    ragged_planted_batch,
    tiny_boxed_lp,
    infeasible_lp,
    infeasible_qp,
    mixed_qp_batch,
    contradict_row,
    portfolio_qp_batch,
    portfolio_instance,
    zipf_pmf,
    random_qp,
    seed_for,
)
