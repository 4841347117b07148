"""Python binding of libhsd.so (include/hsd.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; this module checks
shapes and dtypes of PyTorch tensors, passes their device pointers and the
current HIP stream through ctypes, and turns status codes into exceptions.
It raises at import time if the library has not been built, and never falls
back to any other implementation.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsd.so")

HSD_OK = 0
STATUS_NAMES = {
    0: "HSD_OK", -1: "HSD_ERR_INVALID_ARG", -2: "HSD_ERR_UNSUPPORTED_GRID", -3: "HSD_ERR_OOM",
    -4: "HSD_ERR_HIP", -5: "HSD_ERR_NONFINITE_INPUT", -6: "HSD_ERR_STATE",
}

# exported symbols declared in include/hsd.h
SYMBOLS = (
    "hsd_create", "hsd_destroy", "hsd_last_error", "hsd_add_grain", "hsd_grain_tables",
    "hsd_solve", "hsd_solve_P", "hsd_solve_from_rates", "hsd_sync", "hsd_set_timing", "hsd_phase_ms",
    "hsd_get_class_cfg", "hsd_set_class_cfg", "hsd_set_contract", "hsd_get_contract", "hsd_plan_create", "hsd_plan_launch", "hsd_plan_phase_ms",
    "hsd_plan_destroy", "hsd_autotune", "hsd_autotune_plan", "hsd_set_contract_waves", "hsd_get_contract_waves",
    "hsd_sur_create", "hsd_sur_destroy", "hsd_sur_n_params", "hsd_sur_set_params", "hsd_sur_get_params",
    "hsd_sur_set_norm", "hsd_sur_get_norm", "hsd_sur_features", "hsd_sur_targets", "hsd_sur_fit_norm",
    "hsd_sur_loss_grad", "hsd_sur_train", "hsd_sur_predict", "hsd_solve_surrogate", "hsd_size_convolve",
    "hsd_surrogate_save", "hsd_surrogate_load", "hsd_solve_noalloc", "hsd_sur_set_loss", "hsd_measure_exp2",
    "hsd_table_build", "hsd_table_eval", "hsd_sur_set_train_graph", "hsd_set_energy_budget",
)

N_CLASSES = 4
CLASS_BINS = ((513, 1024), (257, 512), (129, 256), (16, 128))   # bin-count range of each solver class
CONTRACT_FP32 = 0       # emission contraction on FP32 matrix cores
CONTRACT_BF16X3 = 1     # ... as three BF16 products of hi/lo split operands (the default)
PLAN_TIMING = 1
PLAN_CONCURRENT = 2
CHECK_ABSORBED = 0      # surrogate energy check against the absorbed power A
CHECK_MODEL = 1         # ... against rho A, rho the predicted energy ratio of the plain model
CHECK_TABLE = 2         # ... against the table budget of hsd_set_energy_budget
SAVE_WEIGHTS_ONLY = 1   # checkpoint without the Adam moments
SIZE_LAMBDA = 1         # size convolution: lambda j_lambda
SIZE_EV = 2             # ... in eV instead of erg


class HsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class hsd_grain_desc(ctypes.Structure):
    _fields_ = [
        ("radius_cm", ctypes.c_double),
        ("n_atoms", ctypes.c_double),
        ("theta_debye_K", ctypes.c_double),
        ("n_bins", ctypes.c_int32),
        ("E_lo_erg", ctypes.c_double),
        ("E_hi_erg", ctypes.c_double),
        ("cabs_host", ctypes.POINTER(ctypes.c_double)),
        ("longwave_index", ctypes.c_double),
    ]


class hsd_class_cfg(ctypes.Structure):
    _fields_ = [("kg", ctypes.c_int32), ("wide", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class hsd_tune_record(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("cfg", hsd_class_cfg), ("contract_waves", ctypes.c_int32),
                ("n_grains", ctypes.c_int32), ("ms", ctypes.c_double)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1311_4627_amd.build_lib`")
    lib = ctypes.CDLL(path)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    lib.hsd_create.argtypes = [i32, dp, i32, ctypes.POINTER(vp)]
    lib.hsd_create.restype = ctypes.c_int
    lib.hsd_destroy.argtypes = [vp]
    lib.hsd_destroy.restype = None
    lib.hsd_last_error.argtypes = [vp]
    lib.hsd_last_error.restype = ctypes.c_char_p
    lib.hsd_add_grain.argtypes = [vp, ctypes.POINTER(hsd_grain_desc), ctypes.POINTER(i32)]
    lib.hsd_add_grain.restype = ctypes.c_int
    lib.hsd_grain_tables.argtypes = [vp, i32, dp, dp, dp, dp]
    lib.hsd_grain_tables.restype = ctypes.c_int
    lib.hsd_solve.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, vp, vp]
    lib.hsd_solve.restype = ctypes.c_int
    lib.hsd_solve_noalloc.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, vp, vp]
    lib.hsd_solve_noalloc.restype = ctypes.c_int
    lib.hsd_solve_P.argtypes = [vp, i32, vp, i32, vp, vp]
    lib.hsd_solve_P.restype = ctypes.c_int
    lib.hsd_solve_from_rates.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.hsd_solve_from_rates.restype = ctypes.c_int
    lib.hsd_sync.argtypes = [vp]
    lib.hsd_sync.restype = ctypes.c_int
    lib.hsd_set_timing.argtypes = [vp, i32]
    lib.hsd_set_timing.restype = ctypes.c_int
    lib.hsd_phase_ms.argtypes = [vp, dp]
    lib.hsd_phase_ms.restype = ctypes.c_int
    cp = ctypes.POINTER(hsd_class_cfg)
    lib.hsd_get_class_cfg.argtypes = [vp, i32, cp]
    lib.hsd_get_class_cfg.restype = ctypes.c_int
    lib.hsd_set_class_cfg.argtypes = [vp, i32, cp]
    lib.hsd_set_contract.argtypes = [vp, i32]
    lib.hsd_set_contract.restype = ctypes.c_int
    lib.hsd_get_contract.argtypes = [vp, ctypes.POINTER(i32)]
    lib.hsd_get_contract.restype = ctypes.c_int
    lib.hsd_set_class_cfg.restype = ctypes.c_int
    lib.hsd_plan_create.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, vp, i32, ctypes.POINTER(vp)]
    lib.hsd_plan_create.restype = ctypes.c_int
    lib.hsd_plan_launch.argtypes = [vp, vp]
    lib.hsd_plan_launch.restype = ctypes.c_int
    lib.hsd_plan_phase_ms.argtypes = [vp, dp]
    lib.hsd_plan_phase_ms.restype = ctypes.c_int
    lib.hsd_plan_destroy.argtypes = [vp]
    lib.hsd_plan_destroy.restype = None
    lib.hsd_autotune.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), i32, ctypes.POINTER(hsd_tune_record), i32,
                                 ctypes.POINTER(i32)]
    lib.hsd_autotune.restype = ctypes.c_int
    lib.hsd_autotune_plan.argtypes = lib.hsd_autotune.argtypes
    lib.hsd_autotune_plan.restype = ctypes.c_int
    lib.hsd_set_contract_waves.argtypes = [vp, i32]
    lib.hsd_set_contract_waves.restype = ctypes.c_int
    lib.hsd_get_contract_waves.argtypes = [vp, ctypes.POINTER(i32)]
    lib.hsd_get_contract_waves.restype = ctypes.c_int
    i64, fp = ctypes.c_int64, ctypes.POINTER(ctypes.c_float)
    lib.hsd_sur_create.argtypes = [vp, ctypes.POINTER(vp)]
    lib.hsd_sur_destroy.argtypes = [vp]
    lib.hsd_sur_destroy.restype = None
    lib.hsd_sur_n_params.argtypes = [vp, ctypes.POINTER(i64)]
    lib.hsd_sur_set_params.argtypes = [vp, fp]
    lib.hsd_sur_get_params.argtypes = [vp, fp]
    lib.hsd_sur_set_norm.argtypes = [vp, dp, dp, dp, dp]
    lib.hsd_sur_get_norm.argtypes = [vp, dp, dp, dp, dp]
    lib.hsd_sur_features.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, vp, vp]
    lib.hsd_sur_targets.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.hsd_sur_fit_norm.argtypes = [vp, i64, vp, vp]
    lib.hsd_sur_loss_grad.argtypes = [vp, i32, vp, vp, dp, fp]
    lib.hsd_sur_train.argtypes = [vp, i64, vp, vp, i32, i32, ctypes.c_float, ctypes.c_uint64, fp]
    lib.hsd_sur_set_train_graph.argtypes = [vp, i32]
    lib.hsd_sur_set_train_graph.restype = ctypes.c_int
    lib.hsd_sur_predict.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, vp, vp]
    lib.hsd_solve_surrogate.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.c_float,
                                        i32, vp, vp, ctypes.POINTER(i64), vp]
    for name in ("hsd_sur_create", "hsd_sur_n_params", "hsd_sur_set_params", "hsd_sur_get_params",
                 "hsd_sur_set_norm", "hsd_sur_get_norm", "hsd_sur_features", "hsd_sur_targets", "hsd_sur_fit_norm",
                 "hsd_sur_loss_grad", "hsd_sur_train", "hsd_sur_predict", "hsd_solve_surrogate"):
        getattr(lib, name).restype = ctypes.c_int
    lib.hsd_size_convolve.argtypes = [vp, i32, i32, vp, dp, i32, vp, vp]
    lib.hsd_size_convolve.restype = ctypes.c_int
    lib.hsd_surrogate_save.argtypes = [vp, ctypes.c_char_p, i32]
    lib.hsd_surrogate_save.restype = ctypes.c_int
    lib.hsd_table_build.argtypes = [vp, i32, ctypes.POINTER(i32), vp, i32, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.hsd_table_build.restype = ctypes.c_int
    lib.hsd_table_eval.argtypes = [vp, i32, vp, i32, ctypes.POINTER(i32), vp, i32, ctypes.c_double, ctypes.c_double,
                                   vp, vp, vp]
    lib.hsd_table_eval.restype = ctypes.c_int
    lib.hsd_set_energy_budget.argtypes = [vp, i32, ctypes.POINTER(i32), vp, i32, ctypes.c_double, ctypes.c_double,
                                          vp, vp]
    lib.hsd_set_energy_budget.restype = ctypes.c_int
    lib.hsd_measure_exp2.argtypes = [vp, dp]
    lib.hsd_measure_exp2.restype = ctypes.c_int
    lib.hsd_sur_set_loss.argtypes = [vp, ctypes.c_float]
    lib.hsd_sur_set_loss.restype = ctypes.c_int
    lib.hsd_surrogate_load.argtypes = [vp, ctypes.c_char_p]
    lib.hsd_surrogate_load.restype = ctypes.c_int
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_dev(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """Owns one hsd_ctx.  Methods mirror the C entry points one to one."""

    def __init__(self, lam_cm: np.ndarray, device: int = 0):
        self._lib = lib()
        lam = np.ascontiguousarray(lam_cm, dtype=np.float64)
        h = ctypes.c_void_p()
        st = self._lib.hsd_create(int(device), _dptr(lam), int(lam.shape[0]), ctypes.byref(h))
        if st != HSD_OK:
            raise HsdError(st, "hsd_create failed")
        self._h = h
        self.L = int(lam.shape[0])
        self.n_bins = {}

    def _raise(self, st: int, what: str):
        msg = self._lib.hsd_last_error(self._h).decode()
        raise HsdError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hsd_add_grain(self, n_atoms: float, theta_K: float, n_bins: int, E_lo: float, E_hi: float,
                      cabs: np.ndarray, longwave_index: float, radius_cm: float = 0.0) -> int:
        c = np.ascontiguousarray(cabs, dtype=np.float64)
        if c.shape != (self.L,):
            raise ValueError("C_abs table must have one value per grid wavelength")
        d = hsd_grain_desc(radius_cm, n_atoms, theta_K, int(n_bins), E_lo, E_hi, _dptr(c), longwave_index)
        gid = ctypes.c_int32()
        st = self._lib.hsd_add_grain(self._h, ctypes.byref(d), ctypes.byref(gid))
        if st != HSD_OK:
            self._raise(st, "hsd_add_grain")
        self.n_bins[gid.value] = int(n_bins)
        return gid.value

    def add_grain(self, grain) -> int:
        """Register a synth.Grain."""
        return self.hsd_add_grain(grain.n_atoms, grain.theta_K, grain.n_bins, grain.E_lo_erg, grain.E_hi_erg,
                                  grain.cabs_cm2, grain.longwave_index, grain.radius_cm)

    def hsd_grain_tables(self, gid: int):
        n = self.n_bins[gid]
        E, dE, T, cool = (np.empty(n) for _ in range(4))
        st = self._lib.hsd_grain_tables(self._h, gid, _dptr(E), _dptr(dE), _dptr(T), _dptr(cool))
        if st != HSD_OK:
            self._raise(st, "hsd_grain_tables")
        return E, dE, T, cool

    def hsd_solve(self, u, grain_ids: Sequence[int], j, diag=None, stream=None):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(j, torch.float32, (n_cells, ids.shape[0], self.L), "j")
        if diag is not None:
            _check_dev(diag, torch.float32, (n_cells, ids.shape[0], 4), "diag")
        st = self._lib.hsd_solve(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                 ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), j.data_ptr(),
                                 diag.data_ptr() if diag is not None else None, _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_solve")

    def hsd_solve_noalloc(self, u, grain_ids: Sequence[int], j, diag=None, stream=None):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(j, torch.float32, (n_cells, ids.shape[0], self.L), "j")
        if diag is not None:
            _check_dev(diag, torch.float32, (n_cells, ids.shape[0], 4), "diag")
        st = self._lib.hsd_solve_noalloc(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                         ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), j.data_ptr(),
                                         diag.data_ptr() if diag is not None else None, _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_solve_noalloc")

    def hsd_solve_P(self, u, gid: int, P, stream=None):
        import torch
        n_cells = int(u.shape[0])
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(P, torch.float64, (n_cells, self.n_bins[gid]), "P")
        st = self._lib.hsd_solve_P(self._h, n_cells, u.data_ptr(), int(gid), P.data_ptr(), _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_solve_P")

    def hsd_solve_from_rates(self, A, cool, P, stream=None):
        import torch
        n_pairs, nb = int(A.shape[0]), int(A.shape[1])
        _check_dev(A, torch.float64, (n_pairs, nb, nb), "A")
        _check_dev(cool, torch.float64, (n_pairs, nb), "cool")
        _check_dev(P, torch.float64, (n_pairs, nb), "P")
        st = self._lib.hsd_solve_from_rates(self._h, nb, n_pairs, A.data_ptr(), cool.data_ptr(), P.data_ptr(),
                                            _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_solve_from_rates")

    def hsd_set_timing(self, enable: bool):
        st = self._lib.hsd_set_timing(self._h, 1 if enable else 0)
        if st != HSD_OK:
            self._raise(st, "hsd_set_timing")

    def hsd_phase_ms(self):
        ms = np.zeros(3)
        st = self._lib.hsd_phase_ms(self._h, _dptr(ms))
        if st != HSD_OK:
            self._raise(st, "hsd_phase_ms")
        return ms

    def hsd_get_class_cfg(self, cls: int) -> dict:
        c = hsd_class_cfg()
        st = self._lib.hsd_get_class_cfg(self._h, int(cls), ctypes.byref(c))
        if st != HSD_OK:
            self._raise(st, "hsd_get_class_cfg")
        return {"kg": c.kg, "wide": c.wide, "persistent": c.persistent}

    def hsd_set_class_cfg(self, cls: int, kg: int = 2, wide: int = 0, persistent: int = 0):
        c = hsd_class_cfg(int(kg), int(wide), int(persistent))
        st = self._lib.hsd_set_class_cfg(self._h, int(cls), ctypes.byref(c))
        if st != HSD_OK:
            self._raise(st, "hsd_set_class_cfg")

    def hsd_set_contract(self, mode: int):
        st = self._lib.hsd_set_contract(self._h, int(mode))
        if st != HSD_OK:
            self._raise(st, "hsd_set_contract")

    def hsd_get_contract(self) -> int:
        m = ctypes.c_int32()
        st = self._lib.hsd_get_contract(self._h, ctypes.byref(m))
        if st != HSD_OK:
            self._raise(st, "hsd_get_contract")
        return int(m.value)

    def _tune(self, fn: str, u, grain_ids: Sequence[int], runs: int):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        cap = 64
        recs = (hsd_tune_record * cap)()
        n = ctypes.c_int32()
        st = getattr(self._lib, fn)(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                    ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(runs), recs, cap,
                                    ctypes.byref(n))
        if st != HSD_OK:
            self._raise(st, fn)
        return [{"cls": r.cls, "kg": r.cfg.kg, "wide": r.cfg.wide, "persistent": r.cfg.persistent,
                 "contract_waves": r.contract_waves, "n_grains": r.n_grains, "ms": r.ms}
                for r in recs[:min(n.value, cap)]]

    def hsd_autotune(self, u, grain_ids: Sequence[int], runs: int = 4):
        """Time every class configuration on this batch, each class alone; the
        context keeps the fastest per class.  One dict per configuration timed."""
        return self._tune("hsd_autotune", u, grain_ids, runs)

    def hsd_autotune_plan(self, u, grain_ids: Sequence[int], runs: int = 4):
        """Tune for concurrent plans, each candidate timed as a whole plan
        replay; the context keeps the winners.  One dict per plan timed."""
        return self._tune("hsd_autotune_plan", u, grain_ids, runs)

    def hsd_set_contract_waves(self, waves: int):
        st = self._lib.hsd_set_contract_waves(self._h, int(waves))
        if st != HSD_OK:
            self._raise(st, "hsd_set_contract_waves")

    def hsd_get_contract_waves(self) -> int:
        w = ctypes.c_int32()
        st = self._lib.hsd_get_contract_waves(self._h, ctypes.byref(w))
        if st != HSD_OK:
            self._raise(st, "hsd_get_contract_waves")
        return int(w.value)

    def hsd_plan_create(self, u, grain_ids: Sequence[int], j, diag=None, flags: int = 0) -> "Plan":
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(j, torch.float32, (n_cells, ids.shape[0], self.L), "j")
        if diag is not None:
            _check_dev(diag, torch.float32, (n_cells, ids.shape[0], 4), "diag")
        h = ctypes.c_void_p()
        st = self._lib.hsd_plan_create(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                       ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), j.data_ptr(),
                                       diag.data_ptr() if diag is not None else None, int(flags), ctypes.byref(h))
        if st != HSD_OK:
            self._raise(st, "hsd_plan_create")
        return Plan(self, h, (u, j, diag))

    def hsd_sur_features(self, u, grain_ids: Sequence[int], X=None, A=None, stream=None):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        n = n_cells * int(ids.shape[0])
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        if X is not None:
            _check_dev(X, torch.float32, (n, 33), "X")
        if A is not None:
            _check_dev(A, torch.float64, (n,), "A")
        st = self._lib.hsd_sur_features(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                        ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        X.data_ptr() if X is not None else None,
                                        A.data_ptr() if A is not None else None, _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_sur_features")

    def hsd_sur_targets(self, j, A, Y, stream=None):
        import torch
        n = int(A.shape[0])
        _check_dev(j, torch.float32, (n, self.L), "j")
        _check_dev(A, torch.float64, (n,), "A")
        _check_dev(Y, torch.float32, (n, self.L + 1), "Y")
        st = self._lib.hsd_sur_targets(self._h, n, j.data_ptr(), A.data_ptr(), Y.data_ptr(), _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_sur_targets")

    def hsd_solve_surrogate(self, u, grain_ids: Sequence[int], surs: Sequence["Surrogate"], j, diag, tol=0.01,
                            check: int = CHECK_MODEL, stream=None) -> int:
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        G = int(ids.shape[0])
        if len(surs) != G:
            raise ValueError("one surrogate per grain")
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(j, torch.float32, (n_cells, G, self.L), "j")
        _check_dev(diag, torch.float32, (n_cells, G, 4), "diag")
        hs = (ctypes.c_void_p * G)(*[s._h.value for s in surs])
        nfb = ctypes.c_int64()
        st = self._lib.hsd_solve_surrogate(self._h, n_cells, u.data_ptr(), G,
                                           ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), hs, float(tol),
                                           int(check), j.data_ptr(), diag.data_ptr(), ctypes.byref(nfb),
                                           _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_solve_surrogate")
        return int(nfb.value)

    def hsd_size_convolve(self, j, weights, out, lambda_weighted: bool = True, per_ev: bool = False, stream=None):
        import torch
        n_cells, G = int(j.shape[0]), int(j.shape[1])
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.shape != (G,):
            raise ValueError("one weight per grain")
        _check_dev(j, torch.float32, (n_cells, G, self.L), "j")
        _check_dev(out, torch.float64, (n_cells, self.L), "out")
        flags = (SIZE_LAMBDA if lambda_weighted else 0) | (SIZE_EV if per_ev else 0)
        st = self._lib.hsd_size_convolve(self._h, n_cells, G, j.data_ptr(), _dptr(w), flags, out.data_ptr(),
                                         _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_size_convolve")

    def hsd_table_build(self, grain_ids: Sequence[int], u_ref, log10U_lo: float, log10U_hi: float, table, stream=None):
        import torch
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        G, K = int(ids.shape[0]), int(table.shape[1])
        _check_dev(u_ref, torch.float64, (self.L,), "u_ref")
        _check_dev(table, torch.float32, (G, K, self.L), "table")
        st = self._lib.hsd_table_build(self._h, G, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), u_ref.data_ptr(),
                                       K, float(log10U_lo), float(log10U_hi), table.data_ptr(), _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_table_build")

    def hsd_table_eval(self, u, grain_ids: Sequence[int], u_ref, log10U_lo: float, log10U_hi: float, table, j,
                       stream=None):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        G, K = int(ids.shape[0]), int(table.shape[1])
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(u_ref, torch.float64, (self.L,), "u_ref")
        _check_dev(table, torch.float32, (G, K, self.L), "table")
        _check_dev(j, torch.float32, (n_cells, G, self.L), "j")
        st = self._lib.hsd_table_eval(self._h, n_cells, u.data_ptr(), G, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      u_ref.data_ptr(), K, float(log10U_lo), float(log10U_hi), table.data_ptr(),
                                      j.data_ptr(), _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_table_eval")

    def hsd_set_energy_budget(self, grain_ids: Sequence[int], u_ref, log10U_lo: float, log10U_hi: float, table,
                              stream=None):
        import torch
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        G, K = int(ids.shape[0]), int(table.shape[1])
        _check_dev(u_ref, torch.float64, (self.L,), "u_ref")
        _check_dev(table, torch.float32, (G, K, self.L), "table")
        st = self._lib.hsd_set_energy_budget(self._h, G, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             u_ref.data_ptr(), K, float(log10U_lo), float(log10U_hi),
                                             table.data_ptr(), _stream_ptr(stream))
        if st != HSD_OK:
            self._raise(st, "hsd_set_energy_budget")

    def hsd_measure_exp2(self) -> float:
        r = ctypes.c_double()
        st = self._lib.hsd_measure_exp2(self._h, ctypes.byref(r))
        if st != HSD_OK:
            self._raise(st, "hsd_measure_exp2")
        return float(r.value)

    def hsd_sync(self):
        st = self._lib.hsd_sync(self._h)
        if st != HSD_OK:
            self._raise(st, "hsd_sync")


class Plan:
    """Owns one hsd_plan; keeps the tensors it was built on alive."""

    def __init__(self, ctx: Context, h, buffers):
        self._ctx = ctx
        self._h = h
        self._buffers = buffers

    def hsd_plan_launch(self, stream=None):
        st = self._ctx._lib.hsd_plan_launch(self._h, _stream_ptr(stream))
        if st != HSD_OK:
            self._ctx._raise(st, "hsd_plan_launch")

    def hsd_plan_phase_ms(self):
        ms = np.zeros(3)
        st = self._ctx._lib.hsd_plan_phase_ms(self._h, _dptr(ms))
        if st != HSD_OK:
            self._ctx._raise(st, "hsd_plan_phase_ms")
        return ms

    def close(self):
        if getattr(self, "_h", None):
            self._ctx._lib.hsd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Surrogate:
    """Owns one hsd_sur (a network on the context's device)."""

    def __init__(self, ctx: Context):
        self._ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        st = self._lib.hsd_sur_create(ctx._h, ctypes.byref(h))
        if st != HSD_OK:
            ctx._raise(st, "hsd_sur_create")
        self._h = h
        n = ctypes.c_int64()
        self._check(self._lib.hsd_sur_n_params(h, ctypes.byref(n)), "hsd_sur_n_params")
        self.n_params = int(n.value)
        self.L = ctx.L                  # spectrum length
        self.n_out = ctx.L + 1          # network outputs: the spectrum, then the energy ratio

    def _check(self, st, what):
        if st != HSD_OK:
            self._ctx._raise(st, what)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsd_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hsd_sur_set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.n_params,):
            raise ValueError(f"need {self.n_params} parameters")
        self._check(self._lib.hsd_sur_set_params(self._h, _fptr(p)), "hsd_sur_set_params")

    def hsd_sur_get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.hsd_sur_get_params(self._h, _fptr(p)), "hsd_sur_get_params")
        return p

    def hsd_sur_set_norm(self, x_mean, x_std, y_mean, y_std):
        a, b = (np.ascontiguousarray(v, dtype=np.float64) for v in (x_mean, x_std))
        c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (y_mean, y_std))
        if a.shape != (33,) or b.shape != (33,) or c.shape != (self.n_out,) or d.shape != (self.n_out,):
            raise ValueError("statistics have the wrong shape")
        self._check(self._lib.hsd_sur_set_norm(self._h, _dptr(a), _dptr(b), _dptr(c), _dptr(d)), "hsd_sur_set_norm")

    def hsd_sur_get_norm(self):
        a, b, c, d = np.empty(33), np.empty(33), np.empty(self.n_out), np.empty(self.n_out)
        self._check(self._lib.hsd_sur_get_norm(self._h, _dptr(a), _dptr(b), _dptr(c), _dptr(d)), "hsd_sur_get_norm")
        return a, b, c, d

    def hsd_sur_fit_norm(self, X, Y):
        import torch
        n = int(X.shape[0])
        _check_dev(X, torch.float32, (n, 33), "X")
        _check_dev(Y, torch.float32, (n, self.n_out), "Y")
        self._check(self._lib.hsd_sur_fit_norm(self._h, n, X.data_ptr(), Y.data_ptr()), "hsd_sur_fit_norm")

    def hsd_sur_loss_grad(self, X, Y):
        import torch
        n = int(X.shape[0])
        _check_dev(X, torch.float32, (n, 33), "X")
        _check_dev(Y, torch.float32, (n, self.n_out), "Y")
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.hsd_sur_loss_grad(self._h, n, X.data_ptr(), Y.data_ptr(), ctypes.byref(loss), _fptr(g)),
                    "hsd_sur_loss_grad")
        return float(loss.value), g

    def hsd_sur_train(self, X, Y, steps: int, batch: int, lr: float, seed: int = 4627):
        import torch
        n = int(X.shape[0])
        _check_dev(X, torch.float32, (n, 33), "X")
        _check_dev(Y, torch.float32, (n, self.n_out), "Y")
        trace = np.zeros(max(int(steps), 1), dtype=np.float32)
        self._check(self._lib.hsd_sur_train(self._h, n, X.data_ptr(), Y.data_ptr(), int(steps), int(batch),
                                            float(lr), int(seed), _fptr(trace)), "hsd_sur_train")
        return trace[:int(steps)]

    def hsd_sur_set_train_graph(self, enable: bool):
        self._check(self._lib.hsd_sur_set_train_graph(self._h, 1 if enable else 0), "hsd_sur_set_train_graph")

    def hsd_sur_set_loss(self, band_weight: float):
        self._check(self._lib.hsd_sur_set_loss(self._h, float(band_weight)), "hsd_sur_set_loss")

    def hsd_surrogate_save(self, path: str, weights_only: bool = False):
        self._check(self._lib.hsd_surrogate_save(self._h, os.fsencode(path), SAVE_WEIGHTS_ONLY if weights_only else 0),
                    "hsd_surrogate_save")

    def hsd_surrogate_load(self, path: str):
        self._check(self._lib.hsd_surrogate_load(self._h, os.fsencode(path)), "hsd_surrogate_load")

    def hsd_sur_predict(self, u, grain_ids: Sequence[int], j, diag=None, stream=None):
        import torch
        n_cells = int(u.shape[0])
        ids = np.ascontiguousarray(grain_ids, dtype=np.int32)
        _check_dev(u, torch.float64, (n_cells, self.L), "u")
        _check_dev(j, torch.float32, (n_cells, ids.shape[0], self.L), "j")
        if diag is not None:
            _check_dev(diag, torch.float32, (n_cells, ids.shape[0], 4), "diag")
        self._check(self._lib.hsd_sur_predict(self._h, n_cells, u.data_ptr(), int(ids.shape[0]),
                                              ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), j.data_ptr(),
                                              diag.data_ptr() if diag is not None else None, _stream_ptr(stream)),
                    "hsd_sur_predict")
