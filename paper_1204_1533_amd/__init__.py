"""MI355X line-DG hot path: HIP kernels for gfx950 behind the C ABI of include/ldg.h."""
from .ldg import (Context, Net, LDGError, load_library, exported_symbols,  # noqa: F401
                  LDG_POISSON, LDG_EULER, LDG_NS, LDG_F64, LDG_F32, LDG_BF16)
