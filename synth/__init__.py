"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Pure input generation (random numbers, processes, window geometry and
surrogate permutations); no transfer-entropy arithmetic lives here.
"""
from .configs import (Workload, ar_robustness, ar_scenarios, generic, history, job_workload, linear_pair, make_perms, meg_like,
                      nonlinear_ensemble, served_jobs, uneven_surrogates)

__all__ = ["Workload", "ar_robustness", "ar_scenarios", "generic", "history", "job_workload", "linear_pair", "make_perms", "meg_like",
           "nonlinear_ensemble", "served_jobs", "uneven_surrogates"]
