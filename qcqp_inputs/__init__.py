"""Seeded synthetic QCQP instances shared by the tests, the oracle harness and the benchmark.

This module only draws random numbers and assembles problem data; it holds none of the
solver's arithmetic.  Every instance is a convex QCQP in the form of eq. (QCQP), §2.1:

    min_{x in X} 1/2 x'Q_0 x + q_0'x + c_0   s.t.  1/2 x'Q_i x + q_i'x + c_i <= 0 (i=1..m),  Ax = b,

with X = [lb, ub] a box, or (kml_minmax) the saddle problem min_x max_{lambda in simplex, v} of the
same coupling.  Arrays follow one convention everywhere:

    Q  : (m+1, n, n) float64, Q[0] is the objective (or (m, n, n) with has_q0=False)
    q  : (m+1, n), c : (m+1,), lb/ub : (n,), A : (p, n), b : (p,)
"""
from .gen import (Instance, random_qcqp, random_qcqp_torch, random_qcqp_exact, stack_sha256,
                  paper_random_qcqp, random_conic_qcqp, kml_qcqp, kml_minmax, round_instance,
                  config_seed, serving_trace)

__all__ = ["Instance", "random_qcqp", "random_qcqp_torch", "random_qcqp_exact", "stack_sha256",
           "paper_random_qcqp", "random_conic_qcqp",
           "kml_qcqp", "kml_minmax",
           "round_instance", "config_seed", "serving_trace"]
