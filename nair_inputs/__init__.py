"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This package holds only input construction: an upwind discontinuous-Galerkin
discretisation of steady transport (the model problem of the paper's numerical
results section, equation "transport") on quadrilateral meshes, and the named
workload configurations.  It contains none of the solver's arithmetic, and
imports neither the oracle nor the HIP library.
"""
from .dg_quad import dg_quad, DGSystem, topo_sort_blocks, gauss_lobatto_nodes, sigma_q_model
from .configs import CONFIGS, make_config, config_names, BATCH_CONFIGS, make_batch, concat_systems, angle_system

__all__ = ["dg_quad", "DGSystem", "topo_sort_blocks", "gauss_lobatto_nodes", "sigma_q_model",
           "CONFIGS", "make_config", "config_names", "BATCH_CONFIGS", "make_batch",
           "concat_systems", "angle_system"]
