"""Seeded synthetic inputs, shared by the oracle and by the GPU path.

This package holds random structure only: graphs as CSR arrays and dense random
blocks.  It contains none of the walk-Laplacian arithmetic (no walk counts, no
generating functions, no Krylov steps, no estimators), so the oracle and the
HIP library can both consume its outputs without sharing any code with each
other.
"""

from .graphs import (  # noqa: F401
    csr_from_edges,
    erdos_renyi_gnm,
    barabasi_albert,
    road_grid,
    stochastic_block_model,
    configuration_model_powerlaw,
    rmat,
    cycle_graph,
    circulant_graph,
    complete_graph,
    hypercube_graph,
    star_graph,
    toy_g58,
    csr_from_dense,
    batch_specs,
    training_specs,
    graph_from_spec,
    rmat_device,
)
from .blocks import gaussian_block, rademacher_block, spike_block, sparse_initial_block, glorot_params  # noqa: F401
