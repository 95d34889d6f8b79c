"""MI355X (gfx950) RGB + depth sensor renderer (the rendering hot path of
the Habitat simulator, arXiv:1904.01201).

The work happens in libhabmi.so (HIP kernels and a C++ runtime behind the C
ABI of include/hab.h); this package is its ctypes binding.  Importing the
package does not load the library; the first Context does, and raises if
it has not been built.
"""
from .binding import (HabError, OUT_RGB, OUT_DEPTH, OUT_TRI, OUT_SEMANTIC, HAB_NO_HIT, HAB_OK,
                      HAB_ERR_INVALID_ARG, HAB_ERR_OUT_OF_MEMORY, HAB_ERR_RANGE,
                      HAB_ERR_DEVICE, HAB_ERR_NOT_READY, HAB_ERR_CAPACITY, HAB_ERR_CANCELLED,
                      HAB_ERR_TIMEOUT, load, lib_path)
from .renderer import Context, NavHandle, SceneHandle, Server, Stepper

__all__ = ["Context", "NavHandle", "SceneHandle", "Server", "Stepper", "HabError", "OUT_RGB", "OUT_DEPTH", "OUT_TRI",
           "OUT_SEMANTIC",           "HAB_NO_HIT", "HAB_OK", "HAB_ERR_INVALID_ARG", "HAB_ERR_OUT_OF_MEMORY",
           "HAB_ERR_RANGE", "HAB_ERR_DEVICE", "HAB_ERR_NOT_READY", "HAB_ERR_CAPACITY",
           "HAB_ERR_CANCELLED", "HAB_ERR_TIMEOUT", "load",
           "lib_path"]
