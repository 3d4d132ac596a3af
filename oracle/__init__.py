"""CPU oracle for the EMT nodal-analysis time loop (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
"""
from .oracle import (run, run_batch, adjoint, loss_complex, assemble, companions,
                     lu_solve, build, max_threads, steady_state)

__all__ = ["run", "run_batch", "adjoint", "loss_complex", "assemble", "companions",
           "lu_solve", "build", "max_threads", "steady_state"]
