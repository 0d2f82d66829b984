"""Seeded synthetic inputs shared by the library's tests, the benchmark and the
CPU oracle.

This module generates operator data only (gauge-link phases, diffusion face
coefficients, graph matrices, problem sizes) and the workload parameter sets.
It holds none of the trace-estimation arithmetic: neither the oracle nor the
library is imported here, and both receive these arrays as plain inputs.
"""
from .generate import (gauge_field, varcoef_faces, batch_problem_sizes,  # noqa: F401
                       WORKLOADS, workload, wilson_mass, nn_init_weights,  # noqa: F401
                       varcoef_levels, graph_laplacian,  # noqa: F401
                       laplace_matrix, bilinear_prolongations)
