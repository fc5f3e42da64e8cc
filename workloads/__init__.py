"""Seeded synthetic series and run parameters for the RQA workloads.

This module only *generates inputs*: scalar time series (computed in FP64 and
cast once to FP32) and the parameter sets that go with them.  It contains none
of the recurrence arithmetic, so both the CPU oracle and the HIP path can be
fed from it without sharing any of the method's code.

Workloads (sizes and distributions follow the RQA experiments: long series of
up to about a million points, fixed radius, minimum line lengths of 2):

* ``logistic``   N=2,000 logistic map r=3.9 (m=2, tau=1, L2, eps=0.1)
* ``ar1_season`` N=100,000 AR(1) phi=0.95 plus a period-365 sinusoid and
  Gaussian noise sigma=0.3, z-normalised (m=3, tau=6, L2, eps=0.5)
* ``lorenz``     N=1,048,576 Lorenz-63 x-coordinate, RK4 dt=0.01
  (m=3, tau=10, L-infinity, eps = fl32(0.05 * std))
* ``windows``    N=500,000 uniform noise, 400 windows of 1,000..20,000 points
  (m=5, tau=2, L1, eps=0.3)
* ``served``     Poisson request stream of independent seeded series
* ``sine``       sin(linspace(0, 1000 pi, 1000001)) (m=2, tau=2, L2, eps=1.0),
  the synthetic runtime series of the paper's Sect. 8.2
"""
from .series import (  # noqa: F401
    NORM_L1, NORM_L2, NORM_LINF, Params,
    logistic_series, ar1_seasonal_series, lorenz_x_series, uniform_series,
    sine_series, corner_lines, workload, windows_plan, served_requests, served_request,
    n_vectors,
)
