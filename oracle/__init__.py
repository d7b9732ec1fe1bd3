"""CPU oracle of the sub-grid-bathymetry DG shallow-water method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library.
"""
from .swdg import (  # noqa: F401
    Mesh, Params, Oracle, tableau, gll_rule, eq_rule, gl_rule, step_coupled,
    lagrange_values, lagrange_derivs, basis_nodes, rule_for, tensor_basis,
)
