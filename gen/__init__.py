"""Seeded synthetic inputs shaped like the paper's separation workloads.

This package samples data from the generative model of the Bayesian N-FHMM
(Section 2.2) and from the source-model shapes of the experiments
(Section 5).  It holds none of the inference arithmetic; both the FP64
oracle and the HIP path read the same arrays from here.
"""
from .problems import CONFIGS, make_nhmm_problem, make_problem, make_tiny, problem_dims  # noqa: F401
