"""Seeded synthetic graph workloads (inputs only).

This package draws the graphs the clustering pipeline is run on: stochastic
block models with planted communities, Chung-Lu graphs with power-law expected
degrees and planted blocks, disconnected regular blocks, and batches of SBMs.
It holds none of the clustering method's arithmetic (no Laplacian, filter,
sampling, k-means or interpolation); both the CPU oracle and the GPU library
receive the CSR arrays it writes as plain inputs.
"""
from .graphs import (  # noqa: F401
    Graph,
    eps_critical,
    sbm,
    sbm_config,
    chung_lu_blocks,
    disconnected_regular,
    sbm_batch,
    sbm_batch_specs,
    csr_from_edges,
)
