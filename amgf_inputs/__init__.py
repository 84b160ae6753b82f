"""Seeded synthetic inputs for the AMGF solve: two stacked elastic cubes in contact.

This package builds the *problem* (stiffness K, gap Jacobian J, barrier diagonal D,
right-hand side b, node coordinates and boundary masks).  It holds none of the
preconditioner's arithmetic: the Schur operator, the hierarchy and every solve step
live in the GPU library and, independently, in the CPU oracle.  Both of them take
their inputs from here.
"""
from .twoblock import (  # noqa: F401
    TwoBlockProblem,
    make_two_block,
    q1_element_matrices,
    ip_sequence_D,
    CONFIGS,
    make_config,
    renumber_nodes,
)
from .block_on_block import make_block_on_block  # noqa: F401
from .contact_qp import bound_barrier, contact_load_and_gap, lumped_masses  # noqa: F401
from . import learning  # noqa: F401
