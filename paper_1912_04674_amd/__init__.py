"""MI355X-native cylindrical envelope PIC (arXiv:1912.04674): HIP kernels for
gfx950 behind the C ABI of include/envpic.h, with a thin ctypes binding."""
from .envpic import (CHI, FP32_BULK, FP64, J, MOMENTUM, POSITION, EnvpicError, Params, Sim,
                     batch_step, footprint, lib, make_params, params_default, stream_copy)

__all__ = ["CHI", "FP32_BULK", "FP64", "J", "MOMENTUM", "POSITION", "EnvpicError", "Params", "Sim",
           "batch_step", "footprint", "lib", "make_params", "params_default", "stream_copy"]
