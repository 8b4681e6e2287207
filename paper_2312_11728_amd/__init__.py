"""MI355X-native Kalman-filter track-fit hot path (HIP kernels behind a C
interface, include/kf.h).  ``kf`` is the ctypes binding; importing it loads
libkf.so and fails if the library is not built."""
import importlib

__all__ = ["kf"]


def __getattr__(name):
    if name == "kf":
        return importlib.import_module(".kf", __name__)
    raise AttributeError(name)
