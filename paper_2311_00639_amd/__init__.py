"""Python binding of libsyk (argument marshalling only).

Every step of the path runs in the HIP library ``libsyk.so`` built from ``csrc/``;
this module only converts arguments (torch tensors are passed by device pointer,
streams by their HIP handle) and raises on non-OK status codes.  There is no
Python or CPU fallback: if the library is missing, importing the binding raises.

Names follow the C ABI in ``include/syk.h``: create_hamiltonian, apply_H,
haar_state, apply_majorana, krylov_expm, otoc, workspace_bytes, tridiag_expm, and the
request engine (Engine: syk_engine_create / submit / poll / cancel / get_stats / destroy),
the disorder average otoc_ensemble and the finite-size-scaling analysis crossing_time and
lyapunov_fit.
"""
from ._lib import (  # noqa: F401
    C64,
    C128,
    EXACT_K,
    BERNOULLI,
    ECANCELLED,
    EAGAIN,
    FIT_GLOBAL,
    FIT_SLOPE,
    Engine,
    BLOCK_U,
    BLOCK_D,
    FULL,
    SykError,
    Hamiltonian,
    Operator,
    KrylovOpts,
    apply_H,
    apply_majorana,
    autotune,
    create_hamiltonian,
    crossing_time,
    green,
    haar_state,
    haar_state_noalloc,
    kernel_revision,
    krylov_expm,
    library_path,
    lyapunov_fit,
    otoc,
    otoc_batch,
    otoc_ensemble,
    plan_blocks,
    plan_describe,
    release_workspace,
    select_variant,
    tridiag_expm,
    workspace_bytes,
)
