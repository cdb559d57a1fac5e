"""MI355X-native multislice ptychography forward model and gradient.

The computation lives in the HIP library ``libadorym.so`` (C ABI in
``include/adorym.h``); this package is its Python binding.
"""
from .api import Context, Geometry, Job, Plan, split_positions, supports_n  # noqa: F401
from .autograd import (MultisliceLoss, multislice_loss, multislice_loss_defocus, multislice_loss_gaps,  # noqa: F401
                       multislice_loss_modes, multislice_loss_nearfield, object_prior)
