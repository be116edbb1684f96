"""MI355X (gfx950) implementation of the placement hot path of the VSBPP
heuristics of Alenezi, Aboelfotoh, Albdaiwi & Almulla (hybrid P system).

Thin Python binding over the C ABI in ``include/vsbpp.h`` (``libvsbpp.so``):
argument marshalling only, every packing step runs in the HIP kernels.
PyTorch provides device memory and streams for the batched entry point.
The library is loaded on first use; a missing library raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvsbpp.so")

FF, BF, WF, H1, H2 = 0, 1, 2, 3, 4
HEURISTICS = {"FF": FF, "BF": BF, "WF": WF, "H1": H1, "H2": H2}
TYPE_SMALLEST_FIT, TYPE_LARGEST = 0, 1

ERRORS = {
    -1: "E_NULL", -2: "E_SIZE", -3: "E_CAPS", -4: "E_WEIGHT", -5: "E_HEURISTIC",
    -6: "E_OPTION", -7: "E_DEVICE", -8: "E_NOMEM", -9: "E_MODEL",
}

# exported symbols, as declared in include/vsbpp.h
EXPORTS = (
    "vsbpp_options_init", "vsbpp_pack", "vsbpp_pack_ex", "vsbpp_pack_batch",
    "vsbpp_best_of", "vsbpp_strerror", "vsbpp_device_ok", "vsbpp_plan_create",
    "vsbpp_plan_run", "vsbpp_plan_launch", "vsbpp_plan_destroy", "vsbpp_last_error",
    "vsbpp_pack_batch_ex", "vsbpp_rollout_labels", "vsbpp_trainer_create",
    "vsbpp_trainer_step", "vsbpp_trainer_gradient", "vsbpp_trainer_device_model",
    "vsbpp_trainer_export", "vsbpp_trainer_destroy", "vsbpp_trainer_state_bytes",
    "vsbpp_trainer_save", "vsbpp_trainer_restore", "vsbpp_lower_bounds",
    "vsbpp_plan_create_ex", "vsbpp_exact_batch", "vsbpp_cost", "vsbpp_lower_bound",
    "vsbpp_model_load", "vsbpp_model_free", "vsbpp_measure_peaks",
    "vsbpp_pack_batch_static",
)


class VsbppError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = int(code)
        detail = ""
        if self.code == -7 and _lib is not None:
            detail = " " + _lib.vsbpp_last_error().decode()
        super().__init__(f"{what}: {ERRORS.get(self.code, self.code)} ({self.code}){detail}")


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("h1_items_per_sublist", ctypes.c_int32),
        ("h2_subset_size", ctypes.c_int32),
        ("type_rule", ctypes.c_int32),
        ("force_criterion", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("active_limit", ctypes.c_int32),
        ("downsize", ctypes.c_int32),
        ("criterion_rule", ctypes.c_int32),
        ("choice_rule", ctypes.c_int32),
        ("rule2_order", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Loads libvsbpp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1602_08735_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        vp = ctypes.c_void_p
        L.vsbpp_options_init.restype = None
        L.vsbpp_options_init.argtypes = [ctypes.POINTER(Options)]
        L.vsbpp_pack.restype = i32
        L.vsbpp_pack.argtypes = [vp, i32, vp, i32, i32, vp, vp]
        L.vsbpp_pack_ex.restype = i32
        L.vsbpp_pack_ex.argtypes = [vp, i32, vp, i32, i32, ctypes.POINTER(Options), vp, vp,
                                    ctypes.POINTER(i64)]
        L.vsbpp_pack_batch.restype = i32
        L.vsbpp_pack_batch.argtypes = [i32, vp, vp, vp, vp, i32, i32, i32, i32,
                                       ctypes.POINTER(Options), vp, vp, vp, vp, vp, vp, vp]
        L.vsbpp_best_of.restype = i32
        L.vsbpp_best_of.argtypes = [vp, i32, vp, vp]
        L.vsbpp_strerror.restype = ctypes.c_char_p
        L.vsbpp_strerror.argtypes = [i32]
        L.vsbpp_last_error.restype = ctypes.c_char_p
        L.vsbpp_last_error.argtypes = []
        L.vsbpp_device_ok.restype = i32
        L.vsbpp_device_ok.argtypes = []
        L.vsbpp_cost.restype = i64
        L.vsbpp_cost.argtypes = [vp, i32, vp, i32]
        L.vsbpp_lower_bound.restype = i64
        L.vsbpp_lower_bound.argtypes = [vp, i32, vp, i32]
        L.vsbpp_model_load.restype = i32
        L.vsbpp_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.vsbpp_model_free.restype = None
        L.vsbpp_model_free.argtypes = [vp]
        _lib = L
    return _lib


def options(seed: int = 0, s1: int = 10, s2: int = 5, type_rule: int = TYPE_SMALLEST_FIT,
            force_crit: int = -1, active_limit: int = 0, downsize: bool = False,
            criterion_rule: int = 0, choice_rule: int = 0, rule2_order: int = 0) -> Options:
    o = Options()
    lib().vsbpp_options_init(ctypes.byref(o))
    o.seed = seed & (2**64 - 1)
    o.h1_items_per_sublist = s1
    o.h2_subset_size = s2
    o.type_rule = type_rule
    o.force_criterion = force_crit
    o.active_limit = active_limit
    o.downsize = int(downsize)
    o.criterion_rule = int(criterion_rule)
    o.choice_rule = int(choice_rule)
    o.rule2_order = int(rule2_order)
    return o


def cost(bin_types, caps) -> int:
    """vsbpp_cost: the total capacity of the bins of a packing."""
    t = np.ascontiguousarray(np.asarray(bin_types, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(caps, dtype=np.int32))
    rc = lib().vsbpp_cost(t.ctypes.data if t.size else None, int(t.size), c.ctypes.data,
                          int(c.size))
    if rc < 0:
        raise VsbppError(rc, "vsbpp_cost")
    return int(rc)


def lower_bound(weights, caps) -> int:
    """vsbpp_lower_bound: max(LB_cap, LB_big) of one instance (host)."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(caps, dtype=np.int32))
    rc = lib().vsbpp_lower_bound(w.ctypes.data if w.size else None, int(w.size), c.ctypes.data,
                                 int(c.size))
    if rc < 0:
        raise VsbppError(rc, "vsbpp_lower_bound")
    return int(rc)


class DeviceModel:
    """A scorer loaded by vsbpp_model_load into device memory; ``ptr`` is
    the device pointer the learned calls take.  Freed by close()."""

    def __init__(self, path: str):
        h = ctypes.c_void_p()
        rc = lib().vsbpp_model_load(os.fsencode(path), ctypes.byref(h))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_model_load")
        self.ptr = h.value

    def close(self) -> None:
        if getattr(self, "ptr", None):
            lib().vsbpp_model_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks() -> dict:
    """vsbpp_measure_peaks: achievable LDS bytes/s and int32 VALU
    lane-ops/s of the current device."""
    out = (ctypes.c_double * 2)()
    L = lib()
    L.vsbpp_measure_peaks.restype = ctypes.c_int32
    L.vsbpp_measure_peaks.argtypes = [ctypes.c_void_p]
    rc = L.vsbpp_measure_peaks(ctypes.addressof(out))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_measure_peaks")
    return {"lds_bytes_per_s": float(out[0]), "valu_int32_ops_per_s": float(out[1])}


def strerror(code: int) -> str:
    return lib().vsbpp_strerror(code).decode()


def device_ok() -> bool:
    return bool(lib().vsbpp_device_ok())


@dataclass
class Packing:
    assignment: np.ndarray
    bin_types: np.ndarray
    nbins: int
    cost: int


def _heur(h) -> int:
    return HEURISTICS[h] if isinstance(h, str) else int(h)


def pack(weights, caps, heuristic, *, seed: int = 0, s1: int = 10, s2: int = 5,
         type_rule: int = TYPE_SMALLEST_FIT, force_crit: int = -1, order=None,
         active_limit: int = 0, downsize: bool = False, rule2_order: int = 0) -> Packing:
    """One instance through vsbpp_pack_ex (host arrays, synchronous)."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(caps, dtype=np.int32))
    m = int(w.size)
    a = np.zeros(max(m, 1), dtype=np.int32)
    t = np.zeros(max(m, 1), dtype=np.int32)
    cost = ctypes.c_int64(0)
    o = options(seed, s1, s2, type_rule, force_crit, active_limit, downsize,
                rule2_order=rule2_order)
    ordv = None
    if order is not None:
        ordv = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        o.order = ordv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    rc = lib().vsbpp_pack_ex(w.ctypes.data, m, c.ctypes.data, int(c.size), _heur(heuristic),
                             ctypes.byref(o), a.ctypes.data, t.ctypes.data, ctypes.byref(cost))
    if rc < 0:
        raise VsbppError(rc, "vsbpp_pack_ex")
    return Packing(a[:m].copy(), t[:rc].copy(), int(rc), int(cost.value))


class DeviceBatch:
    """A batch of instances resident in device memory (torch tensors).

    ``weights``/``order`` int32 [sum m], ``item_off`` int64 [N+1], ``caps``
    int32 [sum n], ``cap_off`` int32 [N+1], ``seeds`` uint64 as int64 [N]."""

    def __init__(self, batch, device="cuda"):
        import torch

        self.n = batch.n_instances
        self.total = batch.total_items
        self.max_items = max(1, batch.max_m)
        ncap = np.diff(batch.cap_off)
        self.max_types = int(ncap.max()) if ncap.size else 1
        self.max_cap = int(max(
            (batch.caps[batch.cap_off[i]] for i in range(self.n) if ncap[i] > 0), default=1))
        t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dt)
        self.weights = t(batch.weights, torch.int32)
        self.item_off = t(batch.item_off, torch.int64)
        self.caps = t(batch.caps, torch.int32)
        self.cap_off = t(batch.cap_off, torch.int32)
        self.order = None if batch.order is None else t(batch.order, torch.int32)
        self.seeds = None if batch.seeds is None else t(
            batch.seeds.astype(np.uint64).view(np.int64), torch.int64)
        self.assignment = torch.empty(max(self.total, 1), dtype=torch.int32, device=device)
        self.bin_types = torch.empty(max(self.total, 1), dtype=torch.int32, device=device)
        self.nbins = torch.empty(max(self.n, 1), dtype=torch.int32, device=device)
        self.cost = torch.empty(max(self.n, 1), dtype=torch.int64, device=device)


def pack_batch(db: DeviceBatch, heuristic, *, seed: int = 0, s1: int = 10, s2: int = 5,
               type_rule: int = TYPE_SMALLEST_FIT, force_crit: int = -1, stream=None,
               use_order: bool = True, use_seeds: bool = True, active_limit: int = 0,
               downsize: bool = False, choice_rule: int = 0, rule2_order: int = 0) -> None:
    """Launches vsbpp_pack_batch on the given torch stream (default: current).
    Results land in db.assignment / db.bin_types / db.nbins / db.cost."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    o = options(seed, s1, s2, type_rule, force_crit, active_limit, downsize,
                choice_rule=choice_rule, rule2_order=rule2_order)
    ptr = lambda x: None if x is None else x.data_ptr()
    rc = lib().vsbpp_pack_batch(
        db.n, ptr(db.weights), ptr(db.item_off), ptr(db.caps), ptr(db.cap_off),
        db.max_items, db.max_types, db.max_cap, _heur(heuristic), ctypes.byref(o),
        ptr(db.order) if use_order else None, ptr(db.seeds) if use_seeds else None,
        ptr(db.assignment), ptr(db.bin_types), ptr(db.nbins), ptr(db.cost),
        ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_pack_batch")


def best_of(cost_tensor, num: int, out_tensor, stream=None) -> None:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().vsbpp_best_of(cost_tensor.data_ptr(), num, out_tensor.data_ptr(),
                             ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_best_of")


class Launch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("lpt", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("lanes_per_instance", ctypes.c_int32), ("waves_per_instance", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class _BatchDesc(ctypes.Structure):
    _fields_ = [
        ("num_instances", ctypes.c_int32),
        ("weights", ctypes.c_void_p), ("item_off", ctypes.c_void_p),
        ("capacities", ctypes.c_void_p), ("cap_off", ctypes.c_void_p),
        ("order", ctypes.c_void_p), ("seeds", ctypes.c_void_p),
        ("max_items", ctypes.c_int32), ("max_types", ctypes.c_int32),
        ("max_capacity", ctypes.c_int32),
        ("assignment", ctypes.c_void_p), ("bin_types", ctypes.c_void_p),
        ("nbins", ctypes.c_void_p), ("cost", ctypes.c_void_p),
    ]


PLAN_GRAPH, PLAN_AUTOTUNE = 1, 2


def _plan_lib():
    L = lib()
    if not getattr(L, "_plan_ready", False):
        L.vsbpp_plan_create.restype = ctypes.c_int32
        L.vsbpp_plan_create.argtypes = [ctypes.POINTER(_BatchDesc), ctypes.c_int32,
                                        ctypes.POINTER(Options), ctypes.POINTER(Launch),
                                        ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]
        L.vsbpp_plan_run.restype = ctypes.c_int32
        L.vsbpp_plan_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.vsbpp_plan_launch.restype = ctypes.c_int32
        L.vsbpp_plan_launch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Launch)]
        L.vsbpp_plan_destroy.restype = None
        L.vsbpp_plan_destroy.argtypes = [ctypes.c_void_p]
        L._plan_ready = True
    return L


class Plan:
    """A DeviceBatch bound to a heuristic and a launch shape (vsbpp_plan_*).
    The DeviceBatch must outlive the plan."""

    def __init__(self, db: DeviceBatch, heuristic, *, launch: dict | None = None,
                 graph: bool = False, autotune: bool = False, seed: int = 0, s1: int = 10,
                 s2: int = 5, type_rule: int = TYPE_SMALLEST_FIT, force_crit: int = -1,
                 use_order: bool = True, use_seeds: bool = True, model_ptr=None,
                 active_limit: int = 0, downsize: bool = False, criterion_rule: int = 0,
                 choice_rule: int = 0, rule2_order: int = 0):
        L = _plan_lib()
        ptr = lambda x: None if x is None else x.data_ptr()
        self.db = db
        self._desc = _BatchDesc(
            db.n, ptr(db.weights), ptr(db.item_off), ptr(db.caps), ptr(db.cap_off),
            ptr(db.order) if use_order else None, ptr(db.seeds) if use_seeds else None,
            db.max_items, db.max_types, db.max_cap,
            ptr(db.assignment), ptr(db.bin_types), ptr(db.nbins), ptr(db.cost))
        o = options(seed, s1, s2, type_rule, force_crit, active_limit, downsize, criterion_rule,
                    choice_rule, rule2_order)
        lp = None
        if launch is not None:
            lp = Launch(launch.get("mode", 0), launch.get("lpt", 0),
                        launch.get("waves_per_block", 4), launch.get("block_threads", 256),
                        launch.get("lanes_per_instance", 64),
                        launch.get("waves_per_instance", 1))
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0)
        h = ctypes.c_void_p()
        if model_ptr is not None:
            L = _learn_lib()
            rc = L.vsbpp_plan_create_ex(ctypes.byref(self._desc), _heur(heuristic),
                                        ctypes.byref(o), model_ptr,
                                        ctypes.byref(lp) if lp is not None else None, flags,
                                        ctypes.byref(h))
        else:
            rc = L.vsbpp_plan_create(ctypes.byref(self._desc), _heur(heuristic),
                                     ctypes.byref(o),
                                     ctypes.byref(lp) if lp is not None else None, flags,
                                     ctypes.byref(h))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_plan_create")
        self._h = h

    def run(self, stream=None) -> None:
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        rc = _plan_lib().vsbpp_plan_run(self._h, ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_plan_run")

    def launch(self) -> dict:
        out = Launch()
        rc = _plan_lib().vsbpp_plan_launch(self._h, ctypes.byref(out))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_plan_launch")
        return out.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None):
            _plan_lib().vsbpp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_batch_static(db: DeviceBatch, heuristic, *, launch: dict | None = None, stream=None,
                      seed: int = 0, s1: int = 10, s2: int = 5,
                      type_rule: int = TYPE_SMALLEST_FIT, force_crit: int = -1,
                      use_order: bool = True, use_seeds: bool = True,
                      active_limit: int = 0, downsize: bool = False) -> None:
    """One run of the batch with a launch shape, its work counter and schedule
    in the library's own device array (vsbpp_pack_batch_static): allocates
    nothing.  Runs that overlap on one GPU share that array and race."""
    import torch

    L = lib()
    if not getattr(L, "_static_ready", False):
        L.vsbpp_pack_batch_static.restype = ctypes.c_int32
        L.vsbpp_pack_batch_static.argtypes = [ctypes.POINTER(_BatchDesc), ctypes.c_int32,
                                              ctypes.POINTER(Options), ctypes.POINTER(Launch),
                                              ctypes.c_void_p]
        L._static_ready = True
    ptr = lambda x: None if x is None else x.data_ptr()
    desc = _BatchDesc(
        db.n, ptr(db.weights), ptr(db.item_off), ptr(db.caps), ptr(db.cap_off),
        ptr(db.order) if use_order else None, ptr(db.seeds) if use_seeds else None,
        db.max_items, db.max_types, db.max_cap,
        ptr(db.assignment), ptr(db.bin_types), ptr(db.nbins), ptr(db.cost))
    o = options(seed, s1, s2, type_rule, force_crit, active_limit, downsize, 0)
    lp = None
    if launch is not None:
        lp = Launch(launch.get("mode", 0), launch.get("lpt", 0),
                    launch.get("waves_per_block", 4), launch.get("block_threads", 256),
                    launch.get("lanes_per_instance", 64),
                    launch.get("waves_per_instance", 1))
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = L.vsbpp_pack_batch_static(ctypes.byref(desc), _heur(heuristic), ctypes.byref(o),
                                   ctypes.byref(lp) if lp is not None else None,
                                   ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_pack_batch_static")


# ---------------------------------------------------------------------------
# Learned bin-type scorer
# ---------------------------------------------------------------------------
TYPE_LEARNED = 2
NFEAT, HIDDEN, MAX_OUT = 16, 64, 16


class Model(ctypes.Structure):
    """vsbpp_model: bf16 weight bit patterns, fp32 biases, row-major [out][in]."""
    _fields_ = [
        ("n_out", ctypes.c_int32),
        ("w1", ctypes.c_uint16 * (HIDDEN * NFEAT)),
        ("b1", ctypes.c_float * HIDDEN),
        ("w2", ctypes.c_uint16 * (HIDDEN * HIDDEN)),
        ("b2", ctypes.c_float * HIDDEN),
        ("w3", ctypes.c_uint16 * (MAX_OUT * HIDDEN)),
        ("b3", ctypes.c_float * MAX_OUT),
    ]

    def to_bytes(self) -> bytes:
        return bytes(self)

    @classmethod
    def from_bytes(cls, data: bytes) -> "Model":
        m = cls()
        ctypes.memmove(ctypes.addressof(m), data, ctypes.sizeof(cls))
        return m


class _Decisions(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("force", ctypes.c_void_p),
                ("features", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("count", ctypes.c_void_p)]


def _learn_lib():
    L = _plan_lib()
    if not getattr(L, "_learn_ready", False):
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        L.vsbpp_pack_batch_ex.restype = i32
        L.vsbpp_pack_batch_ex.argtypes = [ctypes.POINTER(_BatchDesc), i32, ctypes.POINTER(Options),
                                          vp, ctypes.POINTER(_Decisions), vp]
        L.vsbpp_rollout_labels.restype = i32
        L.vsbpp_rollout_labels.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        L.vsbpp_trainer_create.restype = i32
        L.vsbpp_trainer_create.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(vp)]
        L.vsbpp_trainer_step.restype = i32
        L.vsbpp_trainer_step.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32,
                                         ctypes.POINTER(f32), vp]
        L.vsbpp_trainer_gradient.restype = i32
        L.vsbpp_trainer_gradient.argtypes = [vp, vp, vp, vp, vp, i32, vp, i32]
        L.vsbpp_trainer_device_model.restype = vp
        L.vsbpp_trainer_device_model.argtypes = [vp]
        L.vsbpp_trainer_export.restype = i32
        L.vsbpp_trainer_export.argtypes = [vp, ctypes.POINTER(Model)]
        L.vsbpp_trainer_destroy.restype = None
        L.vsbpp_trainer_destroy.argtypes = [vp]
        L.vsbpp_trainer_state_bytes.restype = ctypes.c_int64
        L.vsbpp_trainer_state_bytes.argtypes = [vp]
        L.vsbpp_trainer_save.restype = i32
        L.vsbpp_trainer_save.argtypes = [vp, vp, ctypes.c_int64]
        L.vsbpp_trainer_restore.restype = i32
        L.vsbpp_trainer_restore.argtypes = [vp, vp, ctypes.c_int64]
        L.vsbpp_plan_create_ex.restype = i32
        L.vsbpp_plan_create_ex.argtypes = [ctypes.POINTER(_BatchDesc), i32, ctypes.POINTER(Options),
                                           vp, ctypes.POINTER(Launch), ctypes.c_uint32,
                                           ctypes.POINTER(vp)]
        L.vsbpp_lower_bounds.restype = i32
        L.vsbpp_lower_bounds.argtypes = [i32, vp, vp, vp, vp, vp, vp]
        L.vsbpp_exact_batch.argtypes = [ctypes.POINTER(_BatchDesc), vp]
        L.vsbpp_exact_batch.restype = i32
        L._learn_ready = True
    return L


def _desc(db: DeviceBatch, use_order=True, use_seeds=True, outputs=True, num=None):
    ptr = lambda x: None if x is None else x.data_ptr()
    return _BatchDesc(
        db.n if num is None else num, ptr(db.weights), ptr(db.item_off), ptr(db.caps),
        ptr(db.cap_off), ptr(db.order) if use_order else None,
        ptr(db.seeds) if use_seeds else None, db.max_items, db.max_types, db.max_cap,
        ptr(db.assignment) if outputs else None, ptr(db.bin_types) if outputs else None,
        ptr(db.nbins), ptr(db.cost))


def pack_batch_ex(db: DeviceBatch, heuristic, *, model_ptr=None, src=None, force=None,
                  features=None, info=None, nbins=None, cost=None, seed: int = 0,
                  type_rule: int = TYPE_SMALLEST_FIT, stream=None,
                  active_limit: int = 0, downsize: bool = False, criterion_rule: int = 0,
                  force_crit: int = -1, choice_rule: int = 0, count=None) -> None:
    """vsbpp_pack_batch_ex.  With `src` (int32 tensor [E]) the batch has E
    entries reading instance src[e]; nbins/cost then receive E results (pass
    tensors of size E)."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    L = _learn_lib()
    ptr = lambda x: None if x is None else x.data_ptr()
    d = _desc(db, outputs=src is None, num=(src.numel() if src is not None else None))
    if nbins is not None:
        d.nbins = nbins.data_ptr()
    if cost is not None:
        d.cost = cost.data_ptr()
    dec = _Decisions(ptr(src), ptr(force), ptr(features), ptr(info), ptr(count))
    o = options(seed, type_rule=type_rule, active_limit=active_limit, downsize=downsize,
                criterion_rule=criterion_rule, force_crit=force_crit, choice_rule=choice_rule)
    rc = L.vsbpp_pack_batch_ex(ctypes.byref(d), _heur(heuristic), ctypes.byref(o), model_ptr,
                               ctypes.byref(dec), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_pack_batch_ex")


def rollout_labels(cost, info, num: int, n_types: int, labels, values=None, stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _learn_lib().vsbpp_rollout_labels(
        cost.data_ptr(), info.data_ptr(), num, n_types, labels.data_ptr(),
        None if values is None else values.data_ptr(), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_rollout_labels")


def lower_bounds(db: DeviceBatch, out, stream=None):
    """out: int64 tensor [3*N] <- (sum of weights, LB_cap, LB_big) per instance."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _learn_lib().vsbpp_lower_bounds(db.n, db.weights.data_ptr(), db.item_off.data_ptr(),
                                         db.caps.data_ptr(), db.cap_off.data_ptr(),
                                         out.data_ptr(), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_lower_bounds")


def exact_batch(db: DeviceBatch, stream=None) -> None:
    """vsbpp_exact_batch: the optimum cost of every instance (at most 12
    items each) and one optimal packing, into db's outputs."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    d = _desc(db, use_order=False, use_seeds=False)
    rc = _learn_lib().vsbpp_exact_batch(ctypes.byref(d), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise VsbppError(rc, "vsbpp_exact_batch")


class Trainer:
    """GPU trainer of the scorer (vsbpp_trainer_*)."""

    def __init__(self, init: Model):
        L = _learn_lib()
        h = ctypes.c_void_p()
        rc = L.vsbpp_trainer_create(ctypes.byref(init), ctypes.byref(h))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_trainer_create")
        self._h = h
        self.n_out = init.n_out

    @property
    def device_model(self):
        return _learn_lib().vsbpp_trainer_device_model(self._h)

    def step(self, x, mask, label, idx, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             want_loss=False, stream=None):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        loss = ctypes.c_float(0.0)
        rc = _learn_lib().vsbpp_trainer_step(
            self._h, x.data_ptr(), mask.data_ptr(), label.data_ptr(), idx.data_ptr(),
            idx.numel(), lr, beta1, beta2, eps, ctypes.byref(loss) if want_loss else None,
            ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_trainer_step")
        return float(loss.value) if want_loss else None

    def gradient(self, x, mask, label, idx) -> np.ndarray:
        np_ = 1024 + 64 + 4096 + 64 + 65 * self.n_out
        out = np.zeros(np_, dtype=np.float32)
        rc = _learn_lib().vsbpp_trainer_gradient(self._h, x.data_ptr(), mask.data_ptr(),
                                                 label.data_ptr(), idx.data_ptr(), idx.numel(),
                                                 out.ctypes.data, np_)
        if rc < 0:
            raise VsbppError(rc, "vsbpp_trainer_gradient")
        return out

    def export(self) -> Model:
        m = Model()
        rc = _learn_lib().vsbpp_trainer_export(self._h, ctypes.byref(m))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_trainer_export")
        return m

    def state(self) -> bytes:
        """The trainer's whole state (step, model, master weights, Adam
        moments) as bytes (vsbpp_trainer_save)."""
        L = _learn_lib()
        n = L.vsbpp_trainer_state_bytes(self._h)
        if n < 0:
            raise VsbppError(int(n), "vsbpp_trainer_state_bytes")
        buf = ctypes.create_string_buffer(int(n))
        rc = L.vsbpp_trainer_save(self._h, buf, n)
        if rc != 0:
            raise VsbppError(rc, "vsbpp_trainer_save")
        return buf.raw

    def restore(self, state: bytes) -> None:
        """Loads a state written by state() (vsbpp_trainer_restore)."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        rc = _learn_lib().vsbpp_trainer_restore(self._h, buf, len(state))
        if rc != 0:
            raise VsbppError(rc, "vsbpp_trainer_restore")

    def close(self):
        if getattr(self, "_h", None):
            _learn_lib().vsbpp_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
