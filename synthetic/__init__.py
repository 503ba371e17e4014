"""Seeded synthetic inputs for the InFo-ESRF perturbation update.

This package only *draws* inputs: forecast ensembles, truths, observation
operators, observation noise, localization stencils and random sketches.  It
holds none of the filter's arithmetic (no covariance apply, no solve, no
quadrature), so both the HIP path and the CPU oracle may take their inputs
from it without sharing any of the method.

Workloads (the paper's experiments are synthetic too; these stand in for
them, see the Gaussian forecast model of Sec. 4 and the multi-layer
Lorenz-96 system of Sec. 5):

* ``gaussian_problem``: 1-D periodic grid, members and truth drawn from
  N(0, C) with a Gaussian-shaped circulant C, Gaspari--Cohn localization,
  point observations of every ``obs_stride``-th grid point.
* ``lorenz_problem``: multi-layer Lorenz-96 ensemble (Sec. 5, eq. 5.1).
* ``experiment1_problem`` / ``experiment2_problem``: the paper's own settings
  of Sec. 4 (weighted-channel observations of a Gaussian prior) and Sec. 5
  (vertical channels of the 32 x 40 coupled Lorenz-96 atmosphere).
"""
from .gaussian import (  # noqa: F401
    Problem,
    config_seed,
    gaspari_cohn,
    gc_table_1d,
    gc_table_2d,
    gaussian_problem,
    point_obs_csr,
    config1,
    config2,
    config4_instances,
    sketch_matrix,
)
from .lorenz import lorenz_problem, l96_tendency, l96_rk4_step  # noqa: F401
from .paper import (  # noqa: F401
    chordal,
    experiment1_prior_row,
    experiment1_problem,
    experiment2_forcing,
    experiment2_noise,
    experiment2_problem,
)
