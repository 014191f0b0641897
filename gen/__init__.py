"""Seeded synthetic least-squares workloads.

This module only draws inputs: sparse A (CSR), right-hand side b and the
vector x_true used to build b. It holds none of the method's arithmetic and
is the one piece of code that both the CPU oracle and the GPU path consume.
"""

from .workloads import (  # noqa: F401
    Problem,
    tiny_c1,
    grid_c2,
    sparse_dense_c3,
    random_sparse,
    paper_shape,
    PAPER_SHAPES,
    by_name,
    served_request,
    served_stream,
)
