"""ctypes signatures of the optional libmd entry points (autotuner, graphs,
surrogate), kept apart from the core ones in md.py."""
import ctypes

_VP = ctypes.c_void_p


def signatures():
    return {}
