"""ctypes binding of libdpk.so (C ABI in include/dpk.h): argument marshalling only.

Every step of the evaluation runs in the HIP library; there is no Python or CPU fallback. Loading
fails loudly when the library has not been built (``python -m paper_2304_09409_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpk.so")

DPK_OK, DPK_E_INVALID_ARG, DPK_E_TYPE_RANGE, DPK_E_BOX = 0, -1, -2, -3
DPK_E_NBR_OVERFLOW, DPK_E_BUDGET, DPK_E_OOM, DPK_E_DEVICE, DPK_E_UNIMPLEMENTED = -4, -5, -6, -7, -8
DPK_E_TIMEOUT, DPK_E_CANCELLED = -9, -10
PRECISIONS = {"fp64": 0, "mixed": 1, "bf16": 2, "fp32": 3}
MAX_TYPES = 8


class DpkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpk error {code}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("ntypes", C.c_int32), ("sel", C.c_int32 * MAX_TYPES), ("rcut", C.c_double),
                ("rcut_smth", C.c_double), ("emb", C.c_int32 * 3), ("axis", C.c_int32),
                ("fit", C.c_int32 * 3), ("type_one_side", C.c_int32), ("descriptor", C.c_int32)]

DESCRIPTORS = {"se_e2_a": 0, "se_e2_r": 1, "se_e3": 2}


class _Stats(C.Structure):
    _fields_ = [("nbr_dropped", C.c_int64), ("table_out_of_range", C.c_int64),
                ("max_candidates", C.c_int64), ("workspace_bytes", C.c_int64)]


_lib = None


def lib():
    """Load libdpk.so (once)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime and links it by an unversioned name; load it first so
        # that libdpk.so binds to the same runtime (one HIP runtime per process: torch's device
        # pointers and streams are then valid for the library, and torch can still initialise).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_09409_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.dpk_last_error.restype = C.c_char_p
        L.dpk_model_param_count.argtypes = [C.POINTER(_Desc)]
        L.dpk_model_param_count.restype = C.c_int64
        L.dpk_model_create.argtypes = [C.POINTER(_Desc), dp, C.c_int64, C.POINTER(vp)]
        L.dpk_model_tabulate.argtypes = [vp, C.c_double, C.c_double]
        L.dpk_model_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.dpk_model_save.argtypes = [vp, C.c_char_p]
        L.dpk_model_describe.argtypes = [vp, C.POINTER(_Desc), dp, dp, dp]
        L.dpk_compute_device_dbox.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.dpk_compute_ghost.argtypes = [vp, C.c_int64, C.c_int64, dp, ip, ip, ip, dp, dp, dp, dp]
        L.dpk_model_free.argtypes = [vp]
        L.dpk_model_free.restype = None
        L.dpk_ctx_create.argtypes = [vp, C.c_int, C.c_int, C.c_size_t, C.c_int, C.POINTER(vp)]
        L.dpk_ctx_free.argtypes = [vp]
        L.dpk_ctx_free.restype = None
        L.dpk_ctx_workspace_bytes.argtypes = [vp, C.c_int64]
        L.dpk_ctx_workspace_bytes.restype = C.c_int64
        L.dpk_compute.argtypes = [vp, C.c_int64, dp, ip, dp, dp, dp, dp, dp]
        L.dpk_compute_device.argtypes = [vp, C.c_int64, vp, vp, dp, vp, vp, vp, vp, vp]
        L.dpk_compute_device_noalloc.argtypes = [vp, C.c_int64, vp, vp, dp, vp, vp, vp, vp, vp]
        L.dpk_ctx_check.argtypes = [vp]
        L.dpk_ctx_set_candidate_capacity.argtypes = [vp, C.c_int]
        L.dpk_ctx_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.dpk_ctx_profile.argtypes = [vp, C.c_int]
        L.dpk_ctx_profile_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.dpk_debug_nlist.argtypes = [vp, ip]
        L.dpk_debug_descriptor.argtypes = [vp, dp, dp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != DPK_OK:
        raise DpkError(rc, lib().dpk_last_error().decode())


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def make_desc(model: dict) -> _Desc:
    d = _Desc()
    d.ntypes = model["ntypes"]
    for t, s in enumerate(model["sel"]):
        d.sel[t] = s
    d.rcut, d.rcut_smth = model["rcut"], model["rcut_smth"]
    for k in range(3):
        d.emb[k] = model["emb"][k]
        d.fit[k] = model["fit"][k]
    d.axis = model["axis"]
    d.type_one_side = int(model["type_one_side"])
    d.descriptor = DESCRIPTORS[model.get("descriptor", "se_e2_a")]
    return d


def param_count(model: dict) -> int:
    d = make_desc(model)
    return int(lib().dpk_model_param_count(C.byref(d)))


def _desc_dict(d: _Desc) -> dict:
    out = dict(ntypes=d.ntypes, sel=[d.sel[t] for t in range(d.ntypes)], rcut=d.rcut, rcut_smth=d.rcut_smth,
               emb=list(d.emb), axis=d.axis, fit=list(d.fit), type_one_side=bool(d.type_one_side))
    if d.descriptor:
        out["descriptor"] = {v: k for k, v in DESCRIPTORS.items()}[d.descriptor]
    return out


class Model:
    """An immutable model (description + FP64 parameter blob) of one of the descriptor kinds."""

    def __init__(self, model: dict, params: np.ndarray, _handle=None):
        if _handle is None:
            self._desc = make_desc(model)
            p = np.ascontiguousarray(params, dtype=np.float64)
            h = C.c_void_p()
            _check(lib().dpk_model_create(C.byref(self._desc), _dp(p), p.size, C.byref(h)))
        else:
            h = _handle
        self.handle = h
        self.desc_dict = dict(model)
        self.nc = int(sum(model["sel"]))
        self.ntypes = int(model["ntypes"])

    @classmethod
    def load(cls, path: str) -> "Model":
        """A model from a file written by save() (dpk_model_load)."""
        h = C.c_void_p()
        _check(lib().dpk_model_load(os.fsencode(path), C.byref(h)))
        d = _Desc()
        _check(lib().dpk_model_describe(h, C.byref(d), None, None, None))
        return cls(_desc_dict(d), None, _handle=h)

    def save(self, path: str):
        _check(lib().dpk_model_save(self.handle, os.fsencode(path)))

    def describe(self):
        """(description dict, FP64 parameters, table stride, table range)."""
        d = _Desc()
        st, xm = C.c_double(), C.c_double()
        _check(lib().dpk_model_describe(self.handle, C.byref(d), None, C.byref(st), C.byref(xm)))
        p = np.empty(lib().dpk_model_param_count(C.byref(d)))
        _check(lib().dpk_model_describe(self.handle, C.byref(d), _dp(p), None, None))
        return _desc_dict(d), p, st.value, xm.value

    def tabulate(self, stride: float, x_max: float):
        _check(lib().dpk_model_tabulate(self.handle, stride, x_max))
        return self

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpk_model_free(self.handle)
            self.handle = None


class Context:
    """Device context: one GPU, one precision, a workspace."""

    def __init__(self, model: Model, device: int = 0, precision: str = "fp64", budget_bytes: int = 0,
                 strict_sel: bool = False):
        self.model = model
        self.precision = precision
        h = C.c_void_p()
        _check(lib().dpk_ctx_create(model.handle, device, PRECISIONS[precision], budget_bytes,
                                    int(strict_sel), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpk_ctx_free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def workspace_bytes(self, natoms: int) -> int:
        return int(lib().dpk_ctx_workspace_bytes(self.handle, natoms))

    def compute(self, coord, atype, box=None, atom_energy: bool = False) -> dict:
        """Host arrays in, host arrays out (synchronous)."""
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n = coord.shape[0]
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        e = C.c_double()
        f = np.empty((n, 3))
        v = np.empty(9)
        ae = np.empty(n) if atom_energy else None
        _check(lib().dpk_compute(self.handle, n, _dp(coord), _ip(atype), _dp(box), C.byref(e), _dp(f), _dp(v),
                                 _dp(ae)))
        out = dict(energy=e.value, force=f, virial=v.reshape(3, 3))
        if atom_energy:
            out["atom_energy"] = ae
        return out

    def compute_ghost(self, coord, atype, nlocal: int, ext=None, atom_energy: bool = False) -> dict:
        """One domain: atoms [0, nlocal) owned, the rest ghosts (dpk_compute_ghost). ext: None (the
        library's own search) or (ext_start [nlocal + 1], ext_list) candidate lists."""
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n = coord.shape[0]
        st = li = None
        if ext is not None:
            st = np.ascontiguousarray(ext[0], dtype=np.int32)
            li = np.ascontiguousarray(ext[1], dtype=np.int32)
        e = C.c_double()
        f = np.empty((n, 3))
        v = np.empty(9)
        ae = np.empty(nlocal) if atom_energy else None
        _check(lib().dpk_compute_ghost(self.handle, nlocal, n - nlocal, _dp(coord), _ip(atype), _ip(st), _ip(li),
                                       C.byref(e), _dp(f), _dp(v), _dp(ae)))
        out = dict(energy=e.value, force=f, virial=v.reshape(3, 3))
        if atom_energy:
            out["atom_energy"] = ae
        return out

    def compute_device(self, coord, atype, box, energy, force, virial, atom_energy=None, stream=None,
                       noalloc: bool = False):
        """torch tensors on the GPU (float64 coord [N,3], int32 atype [N]; outputs float64 energy [1],
        force [N,3], virial [9] or [3,3]); box a host array or None. Asynchronous on `stream`
        (default: torch's current stream). noalloc: the allocation-free entry point (periodic box,
        workspace in the device's shared fixed region)."""
        import torch
        n = coord.shape[0]
        for t, dt in ((coord, torch.float64), (atype, torch.int32), (energy, torch.float64),
                      (force, torch.float64), (virial, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError("compute_device needs contiguous GPU tensors of the documented dtypes")
        if stream is None:
            stream = torch.cuda.current_stream(coord.device)
        hbox = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        fn = lib().dpk_compute_device_noalloc if noalloc else lib().dpk_compute_device
        _check(fn(self.handle, n, coord.data_ptr(), atype.data_ptr(), _dp(hbox),
                                        energy.data_ptr(), force.data_ptr(), virial.data_ptr(),
                                        None if atom_energy is None else atom_energy.data_ptr(),
                                        stream.cuda_stream))

    def check(self):
        _check(lib().dpk_ctx_check(self.handle))

    def set_candidate_capacity(self, entries: int):
        """Candidate-buffer entries per atom for the following frames (0 = from the density)."""
        _check(lib().dpk_ctx_set_candidate_capacity(self.handle, int(entries)))

    def compute_device_checked(self, coord, atype, box, energy, force, virial, atom_energy=None, stream=None):
        """compute_device, then wait for the frame and report its device-side errors; a frame that
        overflowed the candidate buffer sized from its mean density runs once more with the
        largest buffer (as the host-buffer entry point does)."""
        self.compute_device(coord, atype, box, energy, force, virial, atom_energy, stream)
        try:
            self.check()
        except DpkError as e:
            if e.code != DPK_E_NBR_OVERFLOW:
                raise
            self.set_candidate_capacity(1024)
            try:
                self.compute_device(coord, atype, box, energy, force, virial, atom_energy, stream)
                self.check()
            finally:
                self.set_candidate_capacity(0)

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().dpk_ctx_stats(self.handle, C.byref(s)))
        return dict(nbr_dropped=s.nbr_dropped, table_out_of_range=s.table_out_of_range,
                    max_candidates=s.max_candidates, workspace_bytes=s.workspace_bytes)

    STAGES = ("prep", "nlist", "embed_fwd", "fit", "embed_bwd", "final")

    def profile(self, enable: bool = True):
        _check(lib().dpk_ctx_profile(self.handle, int(enable)))

    def profile_read(self) -> tuple[dict, int]:
        ms = np.zeros(len(self.STAGES))
        nf = C.c_int64()
        _check(lib().dpk_ctx_profile_read(self.handle, _dp(ms), C.byref(nf)))
        return dict(zip(self.STAGES, ms.tolist())), nf.value

    def debug_nlist(self, natoms: int) -> np.ndarray:
        out = np.empty((natoms, self.model.nc), dtype=np.int32)
        _check(lib().dpk_debug_nlist(self.handle, _ip(out)))
        return out

    def debug_descriptor(self, natoms: int):
        T = np.empty((natoms, 100, 4))
        dT = np.empty((natoms, 100, 4))
        _check(lib().dpk_debug_descriptor(self.handle, _dp(T), _dp(dT)))
        return T, dT


# ------------------------------------------------------------------------------------------
# Model deviation
# ------------------------------------------------------------------------------------------
class _DeviStats(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("f_max", "f_avg", "f_min", "v_max", "v_avg", "v_min")]


class _LossSpec(C.Structure):
    _fields_ = [("energy", C.POINTER(C.c_double)), ("force", C.POINTER(C.c_double)),
                ("virial", C.POINTER(C.c_double)), ("atom_pref", C.POINTER(C.c_double)),
                ("pe", C.c_double), ("pf", C.c_double), ("pv", C.c_double)]


def _train_sigs(L):
    if getattr(L, "_train_sigs", False):
        return
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.dpk_trainer_create.argtypes = [vp, C.c_int, C.POINTER(vp)]
    L.dpk_trainer_free.argtypes = [vp]
    L.dpk_trainer_free.restype = None
    L.dpk_trainer_accumulate.argtypes = [vp, C.c_int64, dp, C.POINTER(C.c_int32), dp, C.POINTER(_LossSpec),
                                         C.c_double, dp, dp, dp, dp]
    for f in ("dpk_trainer_gradient", "dpk_trainer_params"):
        getattr(L, f).argtypes = [vp, dp]
    L.dpk_trainer_set_params.argtypes = [vp, dp]
    L.dpk_trainer_zero_grad.argtypes = [vp]
    L.dpk_trainer_adam_step.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
    L.dpk_learning_rate.argtypes = [C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_int64]
    L.dpk_learning_rate.restype = C.c_double
    L.dpk_loss_prefactor.argtypes = [C.c_double] * 4
    L.dpk_loss_prefactor.restype = C.c_double
    L._train_sigs = True


def learning_rate(lr0: float, lr_stop: float, step: int, stop_steps: int, decay_steps: int) -> float:
    L = lib()
    _train_sigs(L)
    return L.dpk_learning_rate(lr0, lr_stop, step, stop_steps, decay_steps)


def loss_prefactor(p_start: float, p_limit: float, lr: float, lr0: float) -> float:
    L = lib()
    _train_sigs(L)
    return L.dpk_loss_prefactor(p_start, p_limit, lr, lr0)


class Trainer:
    """Loss and parameter gradient of frames, Adam steps (dpk_trainer_*), FP64 on one device."""

    def __init__(self, model: Model, device: int = 0):
        L = lib()
        _train_sigs(L)
        h = C.c_void_p()
        _check(L.dpk_trainer_create(model.handle, device, C.byref(h)))
        self.handle = h
        self.nparams = param_count(model.describe()[0])

    def accumulate(self, coord, atype, box=None, energy=None, force=None, virial=None, pe=0.0, pf=0.0, pv=0.0,
                   atom_pref=None, weight: float = 1.0) -> dict:
        """One frame: its prediction and loss; weight * dL/dtheta is added to the gradient."""
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n = coord.shape[0]
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        keep = []

        def arr(x, shape=None):
            if x is None:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(shape) if shape else
                                     np.asarray(x, dtype=np.float64))
            keep.append(a)
            return _dp(a)

        spec = _LossSpec(arr(None if energy is None else [energy]), arr(force, (n, 3)), arr(virial, (9,)),
                         arr(atom_pref, (n,)), float(pe), float(pf), float(pv))
        loss, e = np.empty(4), C.c_double()
        f, v = np.empty((n, 3)), np.empty(9)
        _check(lib().dpk_trainer_accumulate(self.handle, n, _dp(coord), _ip(atype), _dp(box), C.byref(spec),
                                            float(weight), _dp(loss), C.byref(e), _dp(f), _dp(v)))
        return {"loss": loss[0], "L_E": loss[1], "L_F": loss[2], "L_Xi": loss[3], "energy": e.value, "force": f,
                "virial": v.reshape(3, 3)}

    def gradient(self) -> np.ndarray:
        g = np.empty(self.nparams)
        _check(lib().dpk_trainer_gradient(self.handle, _dp(g)))
        return g

    def zero_grad(self):
        _check(lib().dpk_trainer_zero_grad(self.handle))

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(lib().dpk_trainer_adam_step(self.handle, lr, beta1, beta2, eps))

    def params(self) -> np.ndarray:
        p = np.empty(self.nparams)
        _check(lib().dpk_trainer_params(self.handle, _dp(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        assert p.size == self.nparams
        _check(lib().dpk_trainer_set_params(self.handle, _dp(p)))

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpk_trainer_free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Deviation:
    """An ensemble of models of one description on one device (dpk_devi_*)."""

    def __init__(self, models, device: int = 0, precision: str = "fp64"):
        L = lib()
        if not getattr(L, "_devi_sigs", False):
            L.dpk_devi_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
            L.dpk_devi_free.argtypes = [C.c_void_p]
            L.dpk_devi_free.restype = None
            dp = C.POINTER(C.c_double)
            L.dpk_devi_compute.argtypes = [C.c_void_p, C.c_int64, dp, C.POINTER(C.c_int32), dp, C.c_double,
                                           dp, dp, dp, dp, dp, C.POINTER(_DeviStats)]
            L._devi_sigs = True
        self.models = list(models)
        arr = (C.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        h = C.c_void_p()
        _check(L.dpk_devi_create(arr, len(self.models), device, PRECISIONS[precision], C.byref(h)))
        self.handle = h

    def compute(self, coord, atype, box=None, nu=None) -> dict:
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n, nm = coord.shape[0], len(self.models)
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        e, f, v = np.empty(nm), np.empty((nm, n, 3)), np.empty((nm, 9))
        ef, evv = np.empty(n), np.empty(9)
        st = _DeviStats()
        _check(lib().dpk_devi_compute(self.handle, n, _dp(coord), _ip(atype), _dp(box),
                                      -1.0 if nu is None else float(nu), _dp(e), _dp(f), _dp(v), _dp(ef),
                                      _dp(evv), C.byref(st)))
        return {"energy": e, "force": f, "virial": v.reshape(nm, 3, 3), "eps_f": ef, "eps_v": evv.reshape(3, 3),
                "stats": {k: getattr(st, k) for k, _ in _DeviStats._fields_}}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpk_devi_free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


# ------------------------------------------------------------------------------------------
# Serving
# ------------------------------------------------------------------------------------------
class _Frame(C.Structure):
    _fields_ = [("natoms", C.c_int64), ("coord", C.POINTER(C.c_double)), ("atype", C.POINTER(C.c_int32)),
                ("box", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)),
                ("force", C.POINTER(C.c_double)), ("virial", C.POINTER(C.c_double)),
                ("atom_energy", C.POINTER(C.c_double)), ("simulation", C.c_int64)]


class _Counters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("peak_bytes", C.c_int64), ("budget_waits", C.c_int64), ("slot_reuse", C.c_int64),
                ("launches", C.c_int64)]


def _server_sigs(L):
    if getattr(L, "_server_sigs", False):
        return
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.dpk_server_create.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_size_t, C.POINTER(vp)]
    L.dpk_server_submit.argtypes = [vp, C.POINTER(_Frame), C.POINTER(C.c_uint64)]
    L.dpk_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int)]
    L.dpk_server_wait.argtypes = [vp, C.c_uint64]
    L.dpk_server_wait_for.argtypes = [vp, C.c_uint64, C.c_int64]
    L.dpk_server_cancel.argtypes = [vp, C.c_uint64]
    L.dpk_server_times.argtypes = [vp, C.c_uint64, i64p]
    L.dpk_server_release.argtypes = [vp, C.c_uint64]
    L.dpk_server_stats.argtypes = [vp, C.POINTER(_Counters)]
    L.dpk_server_free.argtypes = [vp]
    L.dpk_server_free.restype = None
    L.dpk_admit_plan.argtypes = [C.c_int, i32p, i64p, i64p, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L._server_sigs = True


def admit_plan(busy, slot_bytes, slot_sim, need, simulation=-1, budget=0, model_bytes=0):
    """The server's admission rule (pure host function): returns (code, slot, release_idle)."""
    L = lib()
    _server_sigs(L)
    b = np.ascontiguousarray(busy, dtype=np.int32)
    sb = np.ascontiguousarray(slot_bytes, dtype=np.int64)
    ss = np.ascontiguousarray(slot_sim, dtype=np.int64)
    slot, rel = C.c_int32(), C.c_int32()
    rc = L.dpk_admit_plan(len(b), b.ctypes.data_as(C.POINTER(C.c_int32)), sb.ctypes.data_as(C.POINTER(C.c_int64)),
                          ss.ctypes.data_as(C.POINTER(C.c_int64)), need, simulation, budget, model_bytes,
                          C.byref(slot), C.byref(rel))
    return rc, slot.value, bool(rel.value)


class Ticket:
    """A submitted frame. The server holds the frame's host buffers until the frame has finished,
    whether or not this object is still alive; dropping it releases the server's record of the
    frame (at once if the frame has finished, else once it has)."""

    def __init__(self, server, tid, out):
        self.server, self.id, self.out = server, tid, out

    def done(self) -> int:
        return self.server.poll(self)

    def result(self, timeout: float | None = None) -> dict:
        """The frame's outputs; with a timeout (seconds) a frame not done by then raises DpkError
        with DPK_E_TIMEOUT and stays in the server."""
        self.server.wait(self, timeout)
        return self.out

    def cancel(self) -> bool:
        """Withdraw the frame if it is still queued (it then reports DPK_E_CANCELLED); False if it
        was already admitted to a slot or has finished."""
        return self.server.cancel(self)

    def __del__(self):
        srv = getattr(self, "server", None)
        if srv is not None:
            srv._drop(self.id)


class Server:
    """Continuous-batching server over nslots device slots (see dpk_server_* in include/dpk.h)."""

    def __init__(self, model: Model, device: int = 0, precision: str = "mixed", nslots: int = 4,
                 budget_bytes: int = 0):
        L = lib()
        _server_sigs(L)
        self.model = model
        # frames not yet seen finished: ticket id -> the host buffers the server reads and writes
        # (kept here, not only in the Ticket, so that a dropped Ticket cannot free them early)
        self._live = {}
        self._orphans = set()   # dropped tickets whose frames had not finished yet
        self._nsub = 0
        h = C.c_void_p()
        _check(L.dpk_server_create(model.handle, device, PRECISIONS[precision], nslots, budget_bytes, C.byref(h)))
        self.handle = h

    def submit(self, coord, atype, box=None, simulation: int = -1, atom_energy: bool = False) -> Ticket:
        coord = np.ascontiguousarray(coord, dtype=np.float64)
        atype = np.ascontiguousarray(atype, dtype=np.int32)
        n = coord.shape[0]
        box = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        e, f, v = np.zeros(1), np.zeros((n, 3)), np.zeros(9)
        ae = np.zeros(n) if atom_energy else None
        fr = _Frame(n, _dp(coord), _ip(atype), _dp(box), _dp(e), _dp(f), _dp(v), _dp(ae), simulation)
        t = C.c_uint64()
        _check(lib().dpk_server_submit(self.handle, C.byref(fr), C.byref(t)))
        out = {"energy_buf": e, "force": f, "virial_buf": v, "atom_energy": ae}
        self._live[t.value] = (coord, atype, box, out)
        self._nsub += 1
        if self._nsub % 64 == 0:
            self._reap()
        return Ticket(self, t.value, out)

    def _state(self, tid: int) -> int:
        d = C.c_int()
        _check(lib().dpk_server_poll(self.handle, tid, C.byref(d)))
        return d.value

    def _reap(self):
        """Drop the buffers of frames that have finished; release the records of dropped tickets."""
        for tid in list(self._live):
            if self._state(tid) != 0:
                del self._live[tid]
                if tid in self._orphans:
                    self._orphans.discard(tid)
                    lib().dpk_server_release(self.handle, tid)

    def _drop(self, tid: int):
        if getattr(self, "handle", None) is None or _lib is None:
            return
        if tid in self._live and self._state(tid) == 0:
            self._orphans.add(tid)          # released once it has finished
            return
        self._live.pop(tid, None)
        _lib.dpk_server_release(self.handle, tid)

    def poll(self, ticket: Ticket) -> int:
        d = self._state(ticket.id)
        if d != 0:
            self._live.pop(ticket.id, None)
        return d

    def wait(self, ticket: Ticket, timeout: float | None = None):
        if timeout is None:
            rc = lib().dpk_server_wait(self.handle, ticket.id)
        else:
            rc = lib().dpk_server_wait_for(self.handle, ticket.id, max(0, int(timeout * 1e6)))
            if rc == DPK_E_TIMEOUT:
                _check(rc)   # still queued or running: its buffers stay with the server
        self._live.pop(ticket.id, None)
        _check(rc)
        o = ticket.out
        o["energy"] = float(o["energy_buf"][0])
        o["virial"] = o["virial_buf"].reshape(3, 3)
        return o

    def cancel(self, ticket: Ticket) -> bool:
        rc = lib().dpk_server_cancel(self.handle, ticket.id)
        if rc == DPK_OK:
            self._live.pop(ticket.id, None)   # the server no longer reads or writes its buffers
            return True
        return False

    def times(self, ticket: Ticket):
        t = np.zeros(3, dtype=np.int64)
        _check(lib().dpk_server_times(self.handle, ticket.id, t.ctypes.data_as(C.POINTER(C.c_int64))))
        return t

    def stats(self) -> dict:
        c = _Counters()
        _check(lib().dpk_server_stats(self.handle, C.byref(c)))
        return {k: getattr(c, k) for k, _ in _Counters._fields_}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dpk_server_free(self.handle)   # waits for every queued frame
            self.handle = None
        self._live = {}
        self._orphans = set()

    def __del__(self):
        self.close()
