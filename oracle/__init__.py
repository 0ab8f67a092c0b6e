"""FP64 CPU oracle for ABIP (Lin, Ma, Ye, Zhang: "An ADMM-Based Interior-Point
Method for Large-Scale Linear Programming", arXiv:1805.12344).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow, NumPy/SciPy implementation written from the paper:
``oracle.abip`` holds the method (HSD embedding, Algorithms 1 and 2, the
stopping rules, over-relaxation and the restart rules), ``oracle.reference``
holds the independent references used to pin it (central point by Newton's
method, dense KKT adjoint, basis-solution derivatives, vertex enumeration),
``oracle.precision`` the FP32-data model of the linear step used to check the
GPU's FP32 bulk phase element by element.
Functions without an independent pin say "parity unpinned" in their docstring.
"""
from .abip import (  # noqa: F401
    Settings, State, Problem, hsd_constants, assemble_Q, apply_Q, DenseIQSolver,
    SchurIQSolver, CGIQSolver, barrier_prox, initial_state, admm_iteration, inner_residual,
    termination, restart, solve, alg1_iteration, alg1_initial, bb_estimate, bb_rule, bb_select,
    SOLVED, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, MAX_ITERS, MU_STOP,
)
from .precision import Fp32DataSchurSolver  # noqa: F401
from .reference import (  # noqa: F401
    central_point, kkt_adjoint, contract_adjoint, basis_gradients, vertex_enumeration,
    kkt_relative,
)
