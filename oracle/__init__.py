"""FP64 CPU oracle of the guiding-centre electron method (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It loads ``liboracle.so`` (plain C, built by ``oracle/build.py``)
and marshals numpy arrays; all arithmetic happens in the C code.
"""
from .oracle import (  # noqa: F401
    PARTICLE_DTYPE, ACTIVE, EXITED, FINISHED, NONFINITE, BOOTSTRAP, PENDING,
    Field, philox, u01, field_eval, field_eval_extra, parker_closed_form, rhs, pc_predict, pc_correct,
    make_ens_table, inject, advance, advance_traj, moments, moments_size, MomentSpec, max_threads,
    lib,
)
