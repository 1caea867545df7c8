"""Seeded synthetic workloads shared by the oracle and the GPU path.

This package holds only input generation: grids, layered or nodal media,
receiver layouts, prior boxes and prior draws.  It contains none of the
method's arithmetic (no stencil, no source discretisation, no Hessian, no
quadrature), so that the independent oracle and the HIP path can both be fed
the very same inputs without sharing any of the code under test.
"""
from .workloads import (  # noqa: F401
    Grid, Medium, Workload, prior_box, draw_uniform, equispaced_receivers,
    candidate_receivers, random_receivers, homogeneous_medium, layered_medium,
    random_layers_medium, nodal_perturbed_medium, cfl_dt, config, CONFIG_NAMES,
    PARAM_NAMES, serving_stream, poisson_arrivals, loh_medium, loh_prior, loh_prior_mean_paper,
    loh_receivers, loh_scenarios, loh_candidates, loh_workload, loh_nested_setup,
    loh_nested_draws, LOH_NESTED_ACTIVE, c4_largest_query, serving_head_of_line,
    serving_queries,
)
