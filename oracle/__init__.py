"""Sequential CPU oracle for the VSBPP placement heuristics (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The oracle checks the HIP path and shares no code
with it.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg may import this package; the product path never does.

The C source (``vsbpp_oracle.c``) states each step of the paper's method
(Section 1 for FF/BF/WF, Section 6.3 for the first heuristic, Section 6.4 for
the second) in plain sequential code.  This module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsbpp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FF, BF, WF, H1, H2 = 0, 1, 2, 3, 4
HEURISTICS = {"FF": FF, "BF": BF, "WF": WF, "H1": H1, "H2": H2}
TYPE_SMALLEST_FIT, TYPE_LARGEST, TYPE_LEARNED = 0, 1, 2
NFEAT, HIDDEN, MAX_OUT = 16, 64, 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Model(ctypes.Structure):
    """The scorer: bf16 weights as raw uint16, fp32 biases, row-major [out][in]."""
    _fields_ = [
        ("n_out", ctypes.c_int32),
        ("w1", ctypes.c_uint16 * (HIDDEN * NFEAT)),
        ("b1", ctypes.c_float * HIDDEN),
        ("w2", ctypes.c_uint16 * (HIDDEN * HIDDEN)),
        ("b2", ctypes.c_float * HIDDEN),
        ("w3", ctypes.c_uint16 * (MAX_OUT * HIDDEN)),
        ("b3", ctypes.c_float * MAX_OUT),
    ]


class Decision(ctypes.Structure):
    _fields_ = [
        ("position", ctypes.c_int32),
        ("weight", ctypes.c_int32),
        ("plain_type", ctypes.c_int32),
        ("chosen", ctypes.c_int32),
        ("feasible", ctypes.c_uint32),
        ("feat", ctypes.c_float * NFEAT),
    ]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("s1", ctypes.c_int32),
        ("s2", ctypes.c_int32),
        ("type_rule", ctypes.c_int32),
        ("force_crit", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("model", ctypes.POINTER(Model)),
        ("force_event", ctypes.c_int32),
        ("force_t1", ctypes.c_int32),
        ("force_t2", ctypes.c_int32),
        ("trace", ctypes.POINTER(Decision)),
        ("trace_cap", ctypes.c_int32),
        ("trace_count", ctypes.POINTER(ctypes.c_int32)),
        ("active_limit", ctypes.c_int32),
        ("downsize", ctypes.c_int32),
        ("criterion_rule", ctypes.c_int32),
        ("choice_rule", ctypes.c_int32),
        ("rule2_order", ctypes.c_int32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("packers", ctypes.c_int64),
        ("perm_packings", ctypes.c_int64),
        ("placements", ctypes.c_int64),
        ("bin_tests", ctypes.c_int64),
        ("live_tests", ctypes.c_int64),
        ("new_bins", ctypes.c_int64),
        ("divisions", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_stream_key.restype = ctypes.c_uint64
        L.orc_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_criterion.restype = ctypes.c_int32
        L.orc_criterion.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_criterion_digit.restype = ctypes.c_int32
        L.orc_criterion_digit.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32]
        L.orc_perm.restype = ctypes.c_int32
        L.orc_perm.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        L.orc_pack.restype = ctypes.c_int32
        L.orc_pack.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(_Opts), i32p, i32p, i64p,
                               ctypes.POINTER(_Stats)]
        L.orc_pack_packer.restype = ctypes.c_int32
        L.orc_pack_packer.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32, i32p,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      i32p, i32p, i64p]
        for name in ("orc_lb_cap", "orc_lb_big", "orc_opt_partitions", "orc_opt_subset_dp"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32]
        L.orc_mlp_forward.restype = None
        L.orc_mlp_forward.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float)]
        L.orc_rollout_label.restype = ctypes.c_int32
        L.orc_rollout_label.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, i64p]
        L.orc_rollout_label_ex.restype = ctypes.c_int32
        L.orc_rollout_label_ex.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, i64p]
        L.orc_choice_label.restype = ctypes.c_int32
        L.orc_choice_label.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, i64p]
        L.orc_lb_sum.restype = ctypes.c_int64
        L.orc_lb_sum.argtypes = [i32p, ctypes.c_int32]
        _lib = L
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Packing:
    assignment: np.ndarray   # int32[m]: bin id per item
    bin_types: np.ndarray    # int32[nbins]: type index per bin (0 = B_1)
    nbins: int
    cost: int
    stats: dict


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def stream_key(seed: int, stream: int) -> int:
    return int(lib().orc_stream_key(seed & (2**64 - 1), stream))


def criterion(key: int, counter: int) -> int:
    return int(lib().orc_criterion(key & (2**64 - 1), counter))


def criterion_digit(key: int, counter: int, t: int) -> int:
    """The second heuristic's draw: digit t+1 (base 3) of output `counter`."""
    return int(lib().orc_criterion_digit(key & (2**64 - 1), counter, t))


def perm(seed: int, m: int) -> np.ndarray:
    """The Rule-1 permutation: entry q is the item at position q."""
    L = lib()
    return np.array([L.orc_perm(seed & (2**64 - 1), m, q) for q in range(m)], dtype=np.int32)


def pack(weights, caps, heuristic, *, seed: int = 0, s1: int = 10, s2: int = 5,
         type_rule: int = TYPE_SMALLEST_FIT, force_crit: int = -1,
         order=None, model: "Model | None" = None, force_event: int = -1,
         force_types=(0, 0), trace: bool = False, active_limit: int = 0,
         downsize: bool = False, criterion_rule: int = 0, choice_rule: int = 0,
         rule2_order: int = 0) -> Packing:
    w = _i32(weights)
    c = _i32(caps)
    m = int(w.size)
    assign = np.zeros(max(m, 1), dtype=np.int32)
    types = np.zeros(max(m, 1), dtype=np.int32)
    cost = ctypes.c_int64(0)
    st = _Stats()
    o = _Opts(seed & (2**64 - 1), s1, s2, type_rule, force_crit, None)
    if model is not None:
        o.model = ctypes.pointer(model)
    o.force_event = force_event
    o.force_t1, o.force_t2 = int(force_types[0]), int(force_types[1])
    o.active_limit = int(active_limit)
    o.downsize = int(downsize)
    o.criterion_rule = int(criterion_rule)
    o.choice_rule = int(choice_rule)
    o.rule2_order = int(rule2_order)
    tr_arr = None
    tr_count = ctypes.c_int32(0)
    if trace:
        tr_arr = (Decision * max(m, 1))()
        o.trace = tr_arr
        o.trace_cap = m
        o.trace_count = ctypes.pointer(tr_count)
    order_arr = None
    if order is not None:
        order_arr = _i32(order)
        o.order = _p32(order_arr)
    if isinstance(heuristic, str):
        heuristic = HEURISTICS[heuristic]
    rc = lib().orc_pack(_p32(w), m, _p32(c), int(c.size), int(heuristic), ctypes.byref(o),
                        _p32(assign), _p32(types), ctypes.byref(cost), ctypes.byref(st))
    if rc < 0:
        raise OracleError(rc)
    stats = {f: int(getattr(st, f)) for f, _ in _Stats._fields_}
    if trace:
        stats["decisions"] = [tr_arr[i] for i in range(tr_count.value)]
    return Packing(assign[:m].copy(), types[:rc].copy(), int(rc), int(cost.value), stats)


def pack_packer(weights, caps, crit, *, rule2: bool, rule5: bool,
                type_rule: int = TYPE_SMALLEST_FIT) -> Packing:
    """One hybrid-P-system packer with explicit per-placement criteria."""
    w = _i32(weights)
    c = _i32(caps)
    cr = _i32(crit)
    m = int(w.size)
    assign = np.zeros(max(m, 1), dtype=np.int32)
    types = np.zeros(max(m, 1), dtype=np.int32)
    cost = ctypes.c_int64(0)
    rc = lib().orc_pack_packer(_p32(w), m, _p32(c), int(c.size), _p32(cr), int(rule2),
                               int(rule5), type_rule, _p32(assign), _p32(types),
                               ctypes.byref(cost))
    if rc < 0:
        raise OracleError(rc)
    return Packing(assign[:m].copy(), types[:rc].copy(), int(rc), int(cost.value), {})


def lb_sum(weights) -> int:
    w = _i32(weights)
    return int(lib().orc_lb_sum(_p32(w), int(w.size)))


def lb_cap(weights, caps) -> int:
    w, c = _i32(weights), _i32(caps)
    return int(lib().orc_lb_cap(_p32(w), int(w.size), _p32(c), int(c.size)))


def lb_big(weights, caps) -> int:
    w, c = _i32(weights), _i32(caps)
    return int(lib().orc_lb_big(_p32(w), int(w.size), _p32(c), int(c.size)))


def lower_bound(weights, caps) -> int:
    """LB = max(LB_cap, LB_big), the denominator of the cost/LB metric."""
    return max(lb_cap(weights, caps), lb_big(weights, caps))


def opt_partitions(weights, caps) -> int:
    w, c = _i32(weights), _i32(caps)
    return int(lib().orc_opt_partitions(_p32(w), int(w.size), _p32(c), int(c.size)))


def opt_subset_dp(weights, caps) -> int:
    w, c = _i32(weights), _i32(caps)
    return int(lib().orc_opt_subset_dp(_p32(w), int(w.size), _p32(c), int(c.size)))


def bf16_bits(x) -> np.ndarray:
    """fp32 -> bfloat16 bit patterns, round to nearest even (test helper)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = (a + 0x7FFF + ((a >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def make_model(w1, b1, w2, b2, w3, b3) -> Model:
    """Model from fp32 arrays (weights rounded to bf16)."""
    mdl = Model()
    n_out = int(np.asarray(b3).size)
    mdl.n_out = n_out
    mdl.w1[:] = bf16_bits(np.asarray(w1).reshape(-1)).tolist()
    mdl.b1[:] = np.asarray(b1, dtype=np.float32).tolist()
    mdl.w2[:] = bf16_bits(np.asarray(w2).reshape(-1)).tolist()
    mdl.b2[:] = np.asarray(b2, dtype=np.float32).tolist()
    w3b = np.zeros(MAX_OUT * HIDDEN, dtype=np.uint16)
    w3b[:n_out * HIDDEN] = bf16_bits(np.asarray(w3).reshape(-1))
    mdl.w3[:] = w3b.tolist()
    b3f = np.zeros(MAX_OUT, dtype=np.float32)
    b3f[:n_out] = np.asarray(b3, dtype=np.float32)
    mdl.b3[:] = b3f.tolist()
    return mdl


def mlp_forward(model: Model, x) -> np.ndarray:
    xv = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    z = np.zeros(MAX_OUT, dtype=np.float32)
    lib().orc_mlp_forward(ctypes.byref(model), xv.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          z.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return z[:model.n_out].copy()


def rollout_label(weights, caps, crit: int, d: int, *, type_rule: int = TYPE_SMALLEST_FIT,
                  downsize: bool = False):
    """(label, values) of decision d of a plain run (depth-2 lookahead) whose
    base rule opens bins by `type_rule`, costs after the downsizing pass when
    `downsize`."""
    w, c = _i32(weights), _i32(caps)
    vals = np.zeros(c.size, dtype=np.int64)
    lab = lib().orc_rollout_label_ex(_p32(w), int(w.size), _p32(c), int(c.size), crit, d,
                                     int(type_rule), int(downsize),
                                     vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return int(lab), vals


def choice_label(weights, caps, crit: int, d: int):
    """(label, values) of contested placement d of a plain run under the
    largest type rule with downsizing (depth-2 lookahead over {the criterion's
    bin, a new bin})."""
    w, c = _i32(weights), _i32(caps)
    vals = np.zeros(2, dtype=np.int64)
    lab = lib().orc_choice_label(_p32(w), int(w.size), _p32(c), int(c.size), crit, d,
                                 vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return int(lab), vals
