"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU oracle (dp_oracle.c).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. The product path (the HIP library behind ``include/dpk.h``) never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dp_oracle.c")
_LIB = os.path.join(_HERE, "libdp_oracle.so")
_lock = threading.Lock()
_lib = None

MAXT = 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("ntypes", C.c_int), ("sel", C.c_int * MAXT), ("rcut", C.c_double),
                ("rcut_smth", C.c_double), ("emb", C.c_int * 3), ("axis", C.c_int),
                ("fit", C.c_int * 3), ("type_one_side", C.c_int), ("descriptor", C.c_int),
                ("params", C.POINTER(C.c_double))]

DESCRIPTORS = {"se_e2_a": 0, "se_e2_r": 1, "se_e3": 2}


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = C.CDLL(build())
            dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
            mp = C.POINTER(_Model)
            lib.orc_switch.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
            lib.orc_param_count.argtypes = [mp]
            lib.orc_param_count.restype = C.c_long
            lib.orc_embed_eval.argtypes = [mp, C.c_int, C.c_double, dp, dp, dp]
            lib.orc_fit_eval.argtypes = [mp, C.c_int, dp, dp]
            lib.orc_fit_eval.restype = C.c_double
            lib.orc_table_build.argtypes = [mp, C.c_double, C.c_int, dp]
            lib.orc_table_eval.argtypes = [mp, dp, C.c_double, C.c_int, C.c_int, C.c_double, dp, dp]
            lib.orc_nlist.argtypes = [mp, C.c_long, dp, ip, dp, C.c_int, ip, dp, lp]
            lib.orc_compute.argtypes = [mp, C.c_long, dp, ip, dp, C.c_int, dp, C.c_double, C.c_int,
                                        dp, dp, dp, dp, lp, lp, ip, dp, dp]
            lib.orc_compute_ghost.argtypes = [mp, C.c_long, C.c_long, dp, ip, dp, dp, dp, dp]
            lib.orc_num_threads.restype = C.c_int
            lib.orc_set_num_threads.argtypes = [C.c_int]
            lib.orc_set_num_threads.restype = None
            _lib = lib
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int))


class Oracle:
    """Binds a model description (dict) and its flat FP64 parameter blob."""

    def __init__(self, model: dict, params: np.ndarray):
        self.lib = _load()
        self.model = dict(model)
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        m = _Model()
        m.ntypes = model["ntypes"]
        for t, s in enumerate(model["sel"]):
            m.sel[t] = s
        m.rcut, m.rcut_smth = model["rcut"], model["rcut_smth"]
        for k in range(3):
            m.emb[k] = model["emb"][k]
            m.fit[k] = model["fit"][k]
        m.axis = model["axis"]
        m.type_one_side = int(model["type_one_side"])
        m.descriptor = DESCRIPTORS[model.get("descriptor", "se_e2_a")]
        m.params = _dp(self.params)
        self._m = m
        n = self.lib.orc_param_count(C.byref(m))
        if n != self.params.size:
            raise ValueError(f"parameter blob has {self.params.size} values, model needs {n}")
        self.nc = sum(model["sel"])
        self.M = model["emb"][-1]

    # -- pieces -------------------------------------------------------------------------
    def switch(self, r: float):
        s, ds = C.c_double(), C.c_double()
        self.lib.orc_switch(float(r), self.model["rcut_smth"], self.model["rcut"],
                            C.byref(s), C.byref(ds))
        return s.value, ds.value

    def embed(self, net: int, x: float):
        y, dy, d2y = (np.empty(self.M) for _ in range(3))
        self.lib.orc_embed_eval(C.byref(self._m), net, float(x), _dp(y), _dp(dy), _dp(d2y))
        return y, dy, d2y

    def fit(self, t: int, d: np.ndarray):
        d = np.ascontiguousarray(d, dtype=np.float64)
        grad = np.empty_like(d)
        e = self.lib.orc_fit_eval(C.byref(self._m), t, _dp(d), _dp(grad))
        return e, grad

    def table(self, dx: float, nint: int) -> np.ndarray:
        nt = self.model["ntypes"]
        nets = nt if self.model["type_one_side"] else nt * nt
        coef = np.empty((nets, nint, self.M, 6))
        self.lib.orc_table_build(C.byref(self._m), dx, nint, _dp(coef))
        return coef

    def table_eval(self, coef: np.ndarray, dx: float, net: int, x: float):
        y, dy = np.empty(self.M), np.empty(self.M)
        oor = self.lib.orc_table_eval(C.byref(self._m), _dp(coef), dx, coef.shape[1], net, float(x),
                                      _dp(y), _dp(dy))
        return y, dy, bool(oor)

    def nlist(self, coord, atype, box, method: int = 1):
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        n = coord.shape[0]
        nl = np.empty((n, self.nc), dtype=np.int32)
        rij = np.empty((n, self.nc, 3))
        nd = C.c_long()
        rc = self.lib.orc_nlist(C.byref(self._m), n, _dp(coord), _ip(atype), _dp(box), method,
                                _ip(nl), _dp(rij), C.byref(nd))
        if rc:
            raise ValueError(f"orc_nlist failed with code {rc}")
        return nl, rij, nd.value

    # -- whole model ------------------------------------------------------------------------
    def compute(self, coord, atype, box, method: int = 1, table=None, dx: float = 0.0,
                dumps: bool = False):
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        n = coord.shape[0]
        e = C.c_double()
        f = np.empty((n, 3))
        v = np.empty(9)
        ei = np.empty(n)
        nd, noor = C.c_long(), C.c_long()
        nl = np.empty((n, self.nc), dtype=np.int32) if dumps else None
        T = np.empty((n, self.M, 4)) if dumps else None
        dT = np.empty((n, self.M, 4)) if dumps else None
        tab = None if table is None else np.ascontiguousarray(table, dtype=np.float64)
        nint = 0 if table is None else tab.shape[1]
        rc = self.lib.orc_compute(C.byref(self._m), n, _dp(coord), _ip(atype), _dp(box), method,
                                  _dp(tab), float(dx), nint, C.byref(e), _dp(f), _dp(v), _dp(ei),
                                  C.byref(nd), C.byref(noor), _ip(nl), _dp(T), _dp(dT))
        if rc:
            raise ValueError(f"orc_compute failed with code {rc}")
        out = dict(energy=e.value, force=f, virial=v.reshape(3, 3), atom_energy=ei,
                   ndrop=nd.value, table_oor=noor.value)
        if dumps:
            out.update(nlist=nl, T=T, dT=dT)
        return out

    def compute_ghost(self, coord, atype, nlocal: int):
        """One domain: atoms [0, nlocal) owned, the rest ghosts (open geometry, no cell)."""
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n = coord.shape[0]
        e = C.c_double()
        f = np.empty((n, 3))
        v = np.empty(9)
        ei = np.empty(nlocal)
        rc = self.lib.orc_compute_ghost(C.byref(self._m), nlocal, n - nlocal, _dp(coord), _ip(atype), C.byref(e),
                                        _dp(f), _dp(v), _dp(ei))
        if rc:
            raise ValueError(f"orc_compute_ghost failed with code {rc}")
        return dict(energy=e.value, force=f, virial=v.reshape(3, 3), atom_energy=ei)

    def energy(self, coord, atype, box, method: int = 1, table=None, dx: float = 0.0):
        return self.compute(coord, atype, box, method, table, dx)["energy"]

    def threads(self) -> int:
        return self.lib.orc_num_threads()

    def set_threads(self, n: int):
        self.lib.orc_set_num_threads(int(n))
