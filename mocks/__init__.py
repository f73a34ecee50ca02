"""Seeded synthetic catalogues for tests and benchmarks.

This module generates inputs only: lognormal galaxy boxes with a linear Kaiser
displacement, survey-like masked catalogues with randoms, and the named
workloads. It holds none of the estimator's arithmetic and is the only code the
oracle's callers and the HIP path's callers share.
"""
from .lognormal import (power_law_pk, gaussian_field, lognormal_box, survey_catalogue,
                        workload, survey_workload, WORKLOADS, to_soa)

__all__ = ["power_law_pk", "gaussian_field", "lognormal_box", "survey_catalogue",
           "workload", "survey_workload", "WORKLOADS", "to_soa"]
