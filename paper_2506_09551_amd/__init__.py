"""MI355X multi-shifted BiCG for resonant (Kramers-Heisenberg) spectra.

The compute path lives in the HIP library ``libmsb.so`` (C ABI in
``include/msb.h``); this package only marshals arguments to it.
"""
from ._capi import (  # noqa: F401
    MSB_C128, MSB_C64, MSB_OK, MSB_EINVAL, MSB_ENOMEM, MSB_EHIP, MSB_BREAKDOWN,
    MSB_NOT_CONVERGED, MSB_FLOOR, STATUS, MsbError, LibStream, make_system, exported_symbols, lib,
    msb_create, msb_destroy, msb_release_workspace, msb_dim, msb_sector_info, msb_device_ok, msb_apply, msb_apply_block, msb_apply_noalloc, msb_apply_timed,
    msb_number_op, msb_dipole, msb_ground_state, msb_solve, msb_solve_reseed, msb_combine, msb_spectrum, msb_spectrum_cf, msb_autotune,
    msb_set_shape, msb_mlp_num_params, msb_mlp_create, msb_mlp_destroy, msb_mlp_set_params,
    msb_mlp_get_params, msb_mlp_grad, msb_mlp_train, msb_mlp_predict, msb_mlp_fallback,
)
