"""MI355X-native structure-preserving reduction of Yee FDTD equations.

The numerical work runs in ``_lib/libyeerom.so`` (HIP, gfx950), declared in
``include/yeerom.h``; ``yeerom`` is its argument-marshalling binding.
"""
from .yeerom import (YR_F32, YR_F64, Operator, Ports, Rom, YeeromError, fdtd_step,  # noqa: F401
                     lib, mor_reduce, rom_lift, rom_perturb, rom_step, rom_step_noalloc,
                     schur_apply)
