"""ctypes binding of the device brick generator (csrc/gwgen.hip -> libgwgen.so).

Generates the same bricks as ``System.bricks`` directly in device memory
(for workloads whose tensor is too large to draw on the host).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libgwgen.so")
        if not os.path.exists(path):
            raise RuntimeError("libgwgen.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(path)
        L.gwgen_bricks.restype = ctypes.c_int
        L.gwgen_bricks.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.gwgen_normal.restype = ctypes.c_int
        L.gwgen_normal.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p]
        _LIB = L
    return _LIB


def bricks_on_device(system, trip, device="cuda", out=None):
    """Torch float64 tensor [n_trip, bs] of the bricks of ``trip`` on the device."""
    import torch
    from .system import STREAM_T, stream_id
    trip_d = torch.as_tensor(np.ascontiguousarray(trip, dtype=np.int32), device=device)
    dist_d = torch.as_tensor(np.ascontiguousarray(system.dist), device=device)
    if out is None:
        out = torch.empty((len(trip), system.brick_size()), dtype=torch.float64, device=device)
    st = torch.cuda.current_stream().cuda_stream
    rc = lib().gwgen_bricks(system.seed, stream_id(STREAM_T, system.sys_id), len(trip),
                            trip_d.data_ptr(), dist_d.data_ptr(), system.n_atoms,
                            system.n_ao_atom, system.n_ri_atom, system.n_ri, system.k_t,
                            out.data_ptr(), st)
    if rc != 0:
        raise RuntimeError(f"gwgen_bricks failed: hip error {rc}")
    return out


def normal_on_device(seed, stream, idx, device="cuda"):
    import torch
    idx_d = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.uint64).view(np.int64), device=device)
    out = torch.empty(len(idx), dtype=torch.float64, device=device)
    rc = lib().gwgen_normal(seed, stream, idx_d.data_ptr(), len(idx), out.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise RuntimeError(f"gwgen_normal failed: hip error {rc}")
    return out
