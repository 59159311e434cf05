"""Device buffers for the binding, allocated through the same HIP runtime the
library links (so a process never loads two HIP runtimes).

DeviceArray exposes ``data_ptr()`` and ``is_cuda`` like a torch tensor, so it
can be passed wherever the binding accepts a device array.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref

import numpy as np

_hip = None

# Arrays still alive are freed by an exit handler of this module: Python runs
# its atexit handlers before the C library's exit handlers, among them the HIP
# runtime's own teardown, after which a hipFree from a finaliser (__del__ during
# interpreter shutdown) touches a runtime that no longer exists and aborts the
# process.
_live: "weakref.WeakSet[DeviceArray]" = weakref.WeakSet()


@atexit.register
def _free_all():
    for a in list(_live):
        try:
            a.free()
        except Exception:
            pass


def hip():
    global _hip
    if _hip is None:
        from . import lib

        lib()  # load libfiedler.so first: it pins the HIP runtime
        H = C.CDLL("libamdhip64.so.7")
        H.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        H.hipFree.argtypes = [C.c_void_p]
        H.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        H.hipDeviceSynchronize.argtypes = []
        for f in (H.hipMalloc, H.hipFree, H.hipMemcpy, H.hipDeviceSynchronize):
            f.restype = C.c_int
        _hip = H
    return _hip


_H2D, _D2H = 1, 2


class DeviceArray:
    """A device copy of a 1-D numpy array (or an uninitialised one)."""

    is_cuda = True

    def __init__(self, src=None, dtype=None, count=None):
        if src is not None:
            src = np.ascontiguousarray(src)
            self.dtype, self.count = src.dtype, src.shape[0]
        else:
            self.dtype, self.count = np.dtype(dtype), int(count)
        self.nbytes = max(1, self.count * self.dtype.itemsize)
        p = C.c_void_p()
        st = hip().hipMalloc(C.byref(p), self.nbytes)
        if st != 0:
            raise MemoryError(f"hipMalloc failed ({st})")
        self._p = p
        _live.add(self)
        self.shape = (self.count,)
        if src is not None and self.count:
            self._check(hip().hipMemcpy(self._p, src.ctypes.data, src.nbytes, _H2D))

    @staticmethod
    def _check(st):
        if st != 0:
            raise RuntimeError(f"HIP error {st}")

    def data_ptr(self) -> int:
        return self._p.value

    def numpy(self) -> np.ndarray:
        out = np.empty(self.count, self.dtype)
        if self.count:
            self._check(hip().hipMemcpy(out.ctypes.data, self._p, out.nbytes, _D2H))
        return out

    def free(self):
        if self._p:
            hip().hipFree(self._p)
            self._p = None

    def __del__(self):
        # During interpreter shutdown the exit handler above has already freed
        # every live array; never call into HIP from a late finaliser.
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass
