"""MI355X-native lattice-Boltzmann plasma-wakefield step (Parise et al., arXiv:2201.05473).

The compute path is the HIP library liblbmpwfa.so (built by ``build.py``) behind the C ABI of
``include/lbmpwfa.h``; ``binding`` marshals arguments to it with ctypes and uses torch only for
device memory and streams.
"""
from .binding import (LBM_EHIP, LBM_EINVAL, LBM_ENOMEM, LBM_ESTATE, LBM_EUNSTABLE, LBM_F16,
                      LBM_F16N,
                      LBM_F32, LBM_F64, LBM_OK, Lattice, LbmError, lbm_checkpoint_bytes, lbm_counters, lbm_destroy,
                      lbm_diagnostics, lbm_fields, lbm_get_state, lbm_init, lbm_last_error,
                      lbm_load, lbm_moments, lbm_save, lbm_set_state, lbm_step, lbm_workspace_bytes, load_library,
                      lbm_adjoint, lbm_adjoint_revolve, lbm_adjoint_revolve_workspace_bytes, lbm_bubble_length,
                      lbm_get_bunch, lbm_set_bunch,
                      lbm_adjoint_workspace_bytes, lbm_vjp_init, lbm_vjp_step, lbm_vjp_workspace_bytes)
from .autograd import LbmWake, wake_objective

__all__ = [
    "LBM_OK", "LBM_EINVAL", "LBM_ENOMEM", "LBM_EHIP", "LBM_EUNSTABLE", "LBM_ESTATE", "LBM_F16", "LBM_F16N", "LBM_F32", "LBM_F64", "Lattice", "LbmError", "load_library",
    "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_moments", "lbm_fields", "lbm_get_state",
    "lbm_set_state", "lbm_diagnostics", "lbm_checkpoint_bytes", "lbm_save", "lbm_load", "lbm_adjoint", "lbm_adjoint_workspace_bytes",
    "lbm_adjoint_revolve", "lbm_adjoint_revolve_workspace_bytes", "lbm_bubble_length", "lbm_set_bunch",
    "lbm_get_bunch",
    "lbm_vjp_step", "lbm_vjp_init", "lbm_vjp_workspace_bytes", "LbmWake", "wake_objective", "lbm_counters", "lbm_destroy", "lbm_last_error",
]
