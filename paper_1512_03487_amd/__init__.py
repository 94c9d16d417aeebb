"""MI355X-native Wilson / domain-wall hopping operator, mixed-precision CG and adjoint kernels.

The compute path is the HIP library libgrid_mi.so (C ABI in include/grid_mi.h); this package is
its thin torch binding. ``fields`` draws seeded synthetic inputs.
"""
from . import fields  # noqa: F401
from .api import (F16Spinor, cg, cg_workspace_bytes, coarse_stencil, convert_links, convert_spinor,  # noqa: F401
                  dhop, dhop_backward, dhop_cb, dwf, dwf_mdag_m, gauge_force, hmc_energy, link_exp, m5inv,
                  md_leapfrog, mg_basis, mg_coarse_op, mg_pcg, mg_prolong, mg_restrict, mg_solve, mg_workspace_bytes,
                  mobius, pseudofermion_action, solve_eo, solve_eo_workspace_bytes, version, wilson)
from .autograd import DhopFn, PseudofermionActionFn  # noqa: F401
from . import hmc  # noqa: F401,E402

__all__ = ["fields", "F16Spinor", "dhop", "wilson", "dwf", "dwf_mdag_m", "cg", "cg_workspace_bytes",
           "dhop_backward", "dhop_cb", "m5inv", "mobius", "gauge_force", "link_exp", "md_leapfrog", "hmc_energy",
           "solve_eo", "solve_eo_workspace_bytes", "coarse_stencil", "mg_basis", "mg_coarse_op", "mg_restrict",
           "mg_pcg", "mg_prolong", "mg_solve", "mg_workspace_bytes", "convert_spinor", "convert_links", "version",
           "DhopFn", "PseudofermionActionFn", "pseudofermion_action"]
