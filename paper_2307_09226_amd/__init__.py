"""MI355X (gfx950) synthesis of FMCW TDM-MIMO beat cubes where every rendered
pixel is a point scatterer.

Submodules:
  scenes  seeded synthetic inputs (radar parameter sets, rendered pixels)
  rs      ctypes binding of librs.so, the C ABI declared in include/rs.h
  build   hipcc build of librs.so

`rs` is imported on first use so that the input generator works without the
built library; importing `rs` itself raises when librs.so is missing.
"""
import importlib

__all__ = ["scenes", "rs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
