"""FP64 CPU oracle of the deposition-stroke renderer -- test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never loads it and the
two share no code; see ``tbr_oracle.cpp`` for what each function follows in
the paper (TBR, arxiv 2609.08722: Sec. 3 chain and compositing, Sec. 4
operator, Sec. 5 relaxation and gradient).

Parity status: every function here is pinned by the CPU tests under
``tests/test_oracle_*.py`` (closed forms, invariants and brute force); none is
"parity unpinned".
"""

from .binding import (  # noqa: F401
    build,
    chart,
    compensate,
    hard_points,
    lib_path,
    map_jacobian,
    num_threads,
    phi,
    phi_drops,
    psi,
    psi_drops,
    render,
    backward,
    set_num_threads,
)
