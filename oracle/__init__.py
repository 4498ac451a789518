"""Plain FP64 CPU oracle for restarted Halpern PDHG on linear programs.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP solver is checked against.  Only the test suite, the
package-level smoke check and the benchmark's CPU-baseline leg may import it;
the solver library never does, and it shares no code with the HIP path (the
two meet only in the seeded instance generators of `lpgen`).

Contents
  core   -- diagonal scaling, power iteration, the PDHG operator T, the
            M-norm, the Halpern / reflected Halpern step and the restarted
            solver loop (Algorithms 1 and 2, adaptive restart rule).
  kkt    -- relative KKT error of a primal-dual pair and the Farkas-ray
            checks for primal and dual infeasibility.
  brute  -- brute-force vertex enumeration for tiny bounded LPs.
  rng    -- the SplitMix64 counter-based generator used for the power
            iteration's start vector.
"""
from .core import (Options, Result, ScaledLP, scale, power_iteration, pdhg_T, m_norm,
                   halpern_point, solve, to_csr, STATUS_NAMES)
from .kkt import rel_kkt, primal_ray_check, dual_ray_check
from .brute import vertex_enumeration
from .rng import splitmix64, uniform_pm1

__all__ = ["Options", "Result", "ScaledLP", "scale", "power_iteration", "pdhg_T", "m_norm",
           "halpern_point", "solve", "to_csr", "STATUS_NAMES", "rel_kkt", "primal_ray_check",
           "dual_ray_check", "vertex_enumeration", "splitmix64", "uniform_pm1"]
