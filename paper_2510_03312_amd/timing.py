"""Per-stage GPU timing with HIP events recorded by the library itself.

``StageTimer`` creates 2 * UBS_N_STAGES HIP events per slot and hands their
handles to a frame (``ubs_frame.stage_events``); the library records one
before and one after each stage's kernels on the call's stream.  Reading the
elapsed times needs the events to have completed (synchronise first).
"""
from __future__ import annotations

import ctypes
from typing import Dict, List

from . import _lib

_hip = None


def hip() -> ctypes.CDLL:
    global _hip
    if _hip is None:
        h = ctypes.CDLL("libamdhip64.so")
        h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        h.hipEventCreate.restype = ctypes.c_int
        h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        h.hipEventDestroy.restype = ctypes.c_int
        h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                          ctypes.c_void_p]
        h.hipEventElapsedTime.restype = ctypes.c_int
        h.hipEventQuery.argtypes = [ctypes.c_void_p]
        h.hipEventQuery.restype = ctypes.c_int
        h.hipGetLastError.argtypes = []
        h.hipGetLastError.restype = ctypes.c_int
        _hip = h
    return _hip


class StageTimer:
    """``slots`` independent sets of stage events (one set per timed step)."""

    def __init__(self, slots: int):
        self.slots = slots
        n = 2 * _lib.N_STAGES
        self.arrays: List[ctypes.Array] = []
        for _ in range(slots):
            arr = (ctypes.c_void_p * n)()
            for k in range(n):
                ev = ctypes.c_void_p()
                if hip().hipEventCreate(ctypes.byref(ev)) != 0:
                    raise RuntimeError("hipEventCreate failed")
                arr[k] = ev
            self.arrays.append(arr)
        self.used = [set() for _ in range(slots)]

    def slot(self, slot: int):
        """The ``ubs_frame.stage_events`` pointer of one slot."""
        return ctypes.cast(self.arrays[slot], ctypes.POINTER(ctypes.c_void_p))

    def attach(self, frame_c, slot: int) -> None:
        frame_c.stage_events = self.slot(slot)

    @staticmethod
    def detach(frame_c) -> None:
        frame_c.stage_events = None

    def elapsed_ms(self, slot: int) -> Dict[str, float]:
        """Stage durations of one slot (only stages that ran: the events of a
        stage that did not run were never recorded, and asking for their
        elapsed time fails; that error is cleared so that it does not
        surface at the next HIP call)."""
        out = {}
        arr = self.arrays[slot]
        for s, name in enumerate(_lib.STAGES):
            a, b = arr[2 * s], arr[2 * s + 1]
            if hip().hipEventQuery(a) != 0 or hip().hipEventQuery(b) != 0:
                hip().hipGetLastError()
                continue
            ms = ctypes.c_float()
            if hip().hipEventElapsedTime(ctypes.byref(ms), a, b) == 0:
                out[name] = float(ms.value)
            else:
                hip().hipGetLastError()
        return out

    def close(self) -> None:
        for arr in self.arrays:
            for k in range(len(arr)):
                if arr[k]:
                    hip().hipEventDestroy(arr[k])
                    arr[k] = None
        self.arrays = []
