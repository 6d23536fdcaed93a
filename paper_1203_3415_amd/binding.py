"""ctypes binding of libmotif.so (argument marshalling only).

Device buffers are torch CUDA tensors (torch provides memory and streams).
Histograms come back as numpy uint64 arrays copied from the device.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmotif.so")
NUM_CLASSES = {3: 13, 4: 199, 5: 9364}

_ERRORS = {
    -1: "EINVAL_K", -2: "EINVAL_SHAPE", -3: "EINDEX", -4: "ESELFLOOP", -5: "EDUP", -6: "ETRANSPOSE",
    -7: "ENOMEM", -8: "EDEVICE", -9: "EAGAIN", -10: "ETOOBIG", -11: "ETIMEOUT", -12: "ECANCELED",
    -13: "EINVAL_ARG", -14: "EINTERNAL", -15: "EPARSE", -16: "EIO",
}


class MotifError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        self.name = _ERRORS.get(self.code, "UNKNOWN")
        msg = lib().motif_strerror(self.code).decode() if _lib_loaded() else self.name
        super().__init__(f"{where}: MOTIF_{self.name} ({self.code}): {msg}")


class _Graph(ctypes.Structure):
    _fields_ = [
        ("out_off", ctypes.c_void_p), ("out_idx", ctypes.c_void_p),
        ("in_off", ctypes.c_void_p), ("in_idx", ctypes.c_void_p),
        ("n", ctypes.c_int32), ("m", ctypes.c_int64),
    ]


_TUNING_FIELDS = ("block", "grid_per_cu", "tile", "heavy", "solo_deg", "light_deg", "light5")


class _Tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in _TUNING_FIELDS]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f in _TUNING_FIELDS}


class _ReadStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("lines", "arcs_read", "self_loops_dropped", "duplicates_merged",
                                              "isolated_dropped")]


_LOCK = threading.Lock()
_LIB = None


def lib_path() -> str:
    return _LIB_PATH


def _lib_loaded() -> bool:
    return _LIB is not None


def lib():
    """Load libmotif.so (once).  Raises if it has not been built: there is no
    fallback implementation."""
    global _LIB
    with _LOCK:
        if _LIB is not None:
            return _LIB
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(_LIB_PATH)
        I32, I64, P, U32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint32
        sig = {
            "motif_init": ([], I32),
            "motif_shutdown": ([], I32),
            "motif_num_classes": ([I32], I32),
            "motif_class_code": ([I32, I32, ctypes.POINTER(U32)], I32),
            "motif_class_multiplicity": ([I32, I32], I32),
            "motif_class_of_code": ([I32, U32], I32),
            "motif_num_undirected_classes": ([I32], I32),
            "motif_undirected_class_code": ([I32, I32, ctypes.POINTER(U32)], I32),
            "motif_class_undirected": ([I32, I32], I32),
            "motif_census_undirected": ([P, P, I32, I64, I32, P, P], I32),
            "motif_strerror": ([I32], ctypes.c_char_p),
            "motif_read_network": ([ctypes.c_char_p, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I64),
                                    ctypes.POINTER(ctypes.POINTER(I32)), ctypes.POINTER(ctypes.POINTER(I32)),
                                    ctypes.POINTER(ctypes.POINTER(I64)), ctypes.POINTER(_ReadStats)], I32),
            "motif_free": ([P], None),
            "motif_census": ([P, P, P, P, I32, I64, I32, P, P], I32),
            "motif_census6": ([P, P, P, P, I32, I64, P, P], I32),
            "motif_class6_codes": ([P], I32),
            "motif_class6_multiplicities": ([P], I32),
            "motif_census_async": ([P, P, P, P, I32, I64, I32, P, P, P], I32),
            "motif_census_noalloc": ([P, P, P, P, I32, I64, I32, P, P], I32),
            "motif_census_batch": ([P, I32, I32, P, P], I32),
            "motif_census_multi": ([P, I32, P, P, P], I32),
            "motif_census_batch_loop": ([P, I32, I32, P, P], I32),
            "motif_get_tuning": ([I32, ctypes.POINTER(_Tuning)], I32),
            "motif_set_tuning": ([I32, ctypes.POINTER(_Tuning)], I32),
            "motif_autotune": ([P, I32, I32, P, P, ctypes.POINTER(_Tuning)], I32),
            "motif_tune_cache_save": ([ctypes.c_char_p], I32),
            "motif_tune_cache_load": ([ctypes.c_char_p], I32),
            "motif_null_randomize": ([P, I32, I32, I32, ctypes.c_uint64, P], I32),
            "motif_null_model": ([P, I32, I32, I32, I32, ctypes.c_uint64, P, P, P], I32),
            "motif_batch_plan_create": ([P, I32, I32, P, P, ctypes.POINTER(I32)], P),
            "motif_batch_plan_run": ([P], I32),
            "motif_batch_plan_destroy": ([P], I32),
            "motif_profile_enable": ([I32], I32),
            "motif_profile_read": ([I32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)], I32),
            "motif_server_create": ([ctypes.c_size_t, I32], P),
            "motif_request_footprint": ([I32, I64, I32], I64),
            "motif_server_submit": ([P, ctypes.POINTER(_Graph), I32, P, ctypes.POINTER(ctypes.c_uint64)], I32),
            "motif_server_wait": ([P, ctypes.c_uint64, I64], I32),
            "motif_server_cancel": ([P, ctypes.c_uint64], I32),
            "motif_server_stats": ([P] + [ctypes.POINTER(I64)] * 4, I32),
            "motif_server_destroy": ([P], I32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
        return L


def _check(rc: int, where: str):
    if rc != 0:
        raise MotifError(rc, where)


def num_classes(k: int) -> int:
    return int(lib().motif_num_classes(k))


def class_code(k: int, cls: int) -> int:
    out = ctypes.c_uint32()
    _check(lib().motif_class_code(k, cls, ctypes.byref(out)), "motif_class_code")
    return int(out.value)


def class_multiplicity(k: int, cls: int) -> int:
    r = lib().motif_class_multiplicity(k, cls)
    if r < 0:
        raise MotifError(r, "motif_class_multiplicity")
    return int(r)


def class_of_code(k: int, code: int) -> int:
    return int(lib().motif_class_of_code(k, code))


_FORMATS = {"auto": 0, "pajek": 1, "edgelist": 2}


def read_network(path: str, fmt: str = "auto", undirected: bool = False, keep_isolated: bool = False):
    """Read a Pajek (.net) or edge-list file into a host CSR (numpy), the way
    the paper prepares its instances: self-loops dropped, repeated arcs merged,
    vertices without neighbours removed.  Returns (n, out_off int32 [n+1],
    out_idx int32 [m], file_ids int64 [n], stats dict)."""
    L = lib()
    n, m = ctypes.c_int32(), ctypes.c_int64()
    po, pi = ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)()
    pid = ctypes.POINTER(ctypes.c_int64)()
    st = _ReadStats()
    flags = (1 if undirected else 0) | (2 if keep_isolated else 0)
    rc = L.motif_read_network(os.fsencode(path), _FORMATS[fmt], flags, ctypes.byref(n), ctypes.byref(m),
                              ctypes.byref(po), ctypes.byref(pi), ctypes.byref(pid), ctypes.byref(st))
    _check(rc, "motif_read_network")
    try:
        off = np.ctypeslib.as_array(po, shape=(n.value + 1,)).copy()
        idx = np.ctypeslib.as_array(pi, shape=(max(1, m.value),))[: m.value].copy()
        ids = np.ctypeslib.as_array(pid, shape=(max(1, n.value),))[: n.value].copy()
    finally:
        for p in (po, pi, pid):
            L.motif_free(ctypes.cast(p, ctypes.c_void_p))
    return n.value, off, idx, ids, {f: int(getattr(st, f)) for f, _ in _ReadStats._fields_}


# ---------------------------------------------------------------- device --

def _torch():
    import torch
    return torch


def to_device(off, idx, device="cuda"):
    """Copy a CSR (numpy or torch) to int32 device tensors."""
    torch = _torch()
    off_t = torch.as_tensor(np.ascontiguousarray(off, dtype=np.int32) if not torch.is_tensor(off) else off)
    idx_t = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32) if not torch.is_tensor(idx) else idx)
    return off_t.to(device=device, dtype=torch.int32).contiguous(), idx_t.to(device=device, dtype=torch.int32).contiguous()


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else ctypes.c_void_p(0)


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(t, name):
    torch = _torch()
    if t is None:
        return
    if not (torch.is_tensor(t) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous int32 CUDA tensor")


def census(out_off, out_idx, n: int, k: int, in_off=None, in_idx=None, stream=None, out=None):
    """Census of one graph given as int32 CUDA tensors.  Returns numpy uint64
    [C] (or fills `out`, an int64 CUDA tensor of C entries, and returns it)."""
    torch = _torch()
    for t, nm in ((out_off, "out_off"), (out_idx, "out_idx"), (in_off, "in_off"), (in_idx, "in_idx")):
        _check_dev(t, nm)
    C = NUM_CLASSES.get(k)
    if C is None:
        raise MotifError(-1, "census")
    hist = out if out is not None else torch.empty(C, dtype=torch.int64, device=out_off.device)
    m = int(out_idx.numel())
    rc = lib().motif_census(_ptr(out_off), _ptr(out_idx), _ptr(in_off), _ptr(in_idx), int(n), m, int(k),
                            _ptr(hist), _stream_handle(stream))
    _check(rc, "motif_census")
    if out is not None:
        return out
    return hist.cpu().numpy().view(np.uint64)


NUM_CLASSES6 = 1_530_843


def census6(out_off, out_idx, n: int, in_off=None, in_idx=None, stream=None, out=None):
    """Census of the connected 6-sets (motif_census6).  Returns numpy uint64
    [NUM_CLASSES6] (or fills `out`, an int64 CUDA tensor, and returns it)."""
    torch = _torch()
    for t, nm in ((out_off, "out_off"), (out_idx, "out_idx"), (in_off, "in_off"), (in_idx, "in_idx")):
        _check_dev(t, nm)
    hist = out if out is not None else torch.empty(NUM_CLASSES6, dtype=torch.int64, device=out_off.device)
    rc = lib().motif_census6(_ptr(out_off), _ptr(out_idx), _ptr(in_off), _ptr(in_idx), int(n),
                             int(out_idx.numel()), _ptr(hist), _stream_handle(stream))
    _check(rc, "motif_census6")
    if out is not None:
        return out
    return hist.cpu().numpy().view(np.uint64)


def class6_codes() -> np.ndarray:
    """Canonical code of every k = 6 class (uint32, increasing)."""
    out = np.zeros(NUM_CLASSES6, np.uint32)
    _check(lib().motif_class6_codes(out.ctypes.data), "motif_class6_codes")
    return out


def class6_multiplicities() -> np.ndarray:
    """Anchors per occurrence of every k = 6 class (uint8)."""
    out = np.zeros(NUM_CLASSES6, np.uint8)
    _check(lib().motif_class6_multiplicities(out.ctypes.data), "motif_class6_multiplicities")
    return out


NUM_UNDIRECTED_CLASSES = {3: 2, 4: 6, 5: 21}


def num_undirected_classes(k: int) -> int:
    return int(lib().motif_num_undirected_classes(k))


def undirected_class_code(k: int, cls: int) -> int:
    out = ctypes.c_uint32()
    _check(lib().motif_undirected_class_code(k, cls, ctypes.byref(out)), "motif_undirected_class_code")
    return int(out.value)


def class_undirected(k: int, cls: int) -> int:
    return int(lib().motif_class_undirected(k, cls))


def census_undirected(out_off, out_idx, n: int, k: int, stream=None, out=None):
    """Undirected census of the graph's undirected version: numpy uint64
    [2 / 6 / 21] (or fills `out`, an int64 CUDA tensor of that size)."""
    torch = _torch()
    for t, nm in ((out_off, "out_off"), (out_idx, "out_idx")):
        _check_dev(t, nm)
    U = NUM_UNDIRECTED_CLASSES.get(k)
    if U is None:
        raise MotifError(-1, "census_undirected")
    hist = out if out is not None else torch.empty(U, dtype=torch.int64, device=out_off.device)
    rc = lib().motif_census_undirected(_ptr(out_off), _ptr(out_idx), int(n), int(out_idx.numel()), int(k),
                                       _ptr(hist), _stream_handle(stream))
    _check(rc, "motif_census_undirected")
    if out is not None:
        return out
    return hist.cpu().numpy().view(np.uint64)


def census_async(out_off, out_idx, n: int, k: int, hist, status, in_off=None, in_idx=None, stream=None):
    """Enqueue a census without waiting: `hist` (int64 CUDA tensor of C
    entries) is written, and `status` (int32 CUDA tensor of 1 entry) receives
    0 or the error code, on the stream.  Raises only for errors found before
    anything is enqueued."""
    torch = _torch()
    for t, nm in ((out_off, "out_off"), (out_idx, "out_idx"), (in_off, "in_off"), (in_idx, "in_idx"),
                  (status, "status")):
        _check_dev(t, nm)
    C = NUM_CLASSES.get(k)
    if C is None:
        raise MotifError(-1, "census_async")
    if not (torch.is_tensor(hist) and hist.is_cuda and hist.dtype == torch.int64 and hist.numel() == C):
        raise TypeError("hist must be an int64 CUDA tensor of C entries")
    rc = lib().motif_census_async(_ptr(out_off), _ptr(out_idx), _ptr(in_off), _ptr(in_idx), int(n),
                                  int(out_idx.numel()), int(k), _ptr(hist), _ptr(status), _stream_handle(stream))
    _check(rc, "motif_census_async")


def census_multi(out_off, out_idx, n: int, ks, in_off=None, in_idx=None, stream=None, outs=None):
    """Census of one graph for several sizes ks (distinct values of 3, 4, 5)
    over one shared G* build.  Returns a list of numpy uint64 [C_k] (or fills
    `outs`, int64 CUDA tensors of C_k entries each, and returns them)."""
    torch = _torch()
    ks = [int(k) for k in ks]
    if any(k not in NUM_CLASSES for k in ks):
        raise MotifError(-1, "census_multi")
    g = _graph_array([(out_off, out_idx, n) + ((in_off, in_idx) if in_off is not None else ())])
    hists = outs if outs is not None else [torch.empty(NUM_CLASSES[k], dtype=torch.int64, device=out_off.device)
                                           for k in ks]
    for h, k in zip(hists, ks):
        if not (torch.is_tensor(h) and h.is_cuda and h.dtype == torch.int64 and h.is_contiguous()
                and h.numel() == NUM_CLASSES[k]):
            raise TypeError("outs must be contiguous int64 CUDA tensors of C_k entries")
    karr = (ctypes.c_int32 * len(ks))(*ks)
    parr = (ctypes.c_void_p * len(ks))(*[h.data_ptr() for h in hists])
    rc = lib().motif_census_multi(ctypes.cast(g, ctypes.c_void_p), len(ks), ctypes.cast(karr, ctypes.c_void_p),
                                  ctypes.cast(parr, ctypes.c_void_p), _stream_handle(stream))
    _check(rc, "motif_census_multi")
    if outs is not None:
        return outs
    return [h.cpu().numpy().view(np.uint64) for h in hists]


def _graph_array(graphs):
    arr = (_Graph * len(graphs))()
    for i, g in enumerate(graphs):
        out_off, out_idx, n = g[0], g[1], g[2]
        in_off = g[3] if len(g) > 3 else None
        in_idx = g[4] if len(g) > 4 else None
        for t, nm in ((out_off, "out_off"), (out_idx, "out_idx"), (in_off, "in_off"), (in_idx, "in_idx")):
            _check_dev(t, nm)
        arr[i] = _Graph(out_off.data_ptr() if out_off.numel() else 0,
                        out_idx.data_ptr() if out_idx.numel() else 0,
                        in_off.data_ptr() if in_off is not None else None,
                        in_idx.data_ptr() if in_idx is not None and in_idx.numel() else None,
                        int(n), int(out_idx.numel()))
    return arr


def census_batch(graphs, k: int, stream=None, out=None, loop: bool = False):
    """Census of many graphs [(out_off, out_idx, n[, in_off, in_idx]), ...]
    in one fused launch (loop=False) or by the per-graph launch loop.
    Returns numpy uint64 [len(graphs), C] (or fills `out`)."""
    torch = _torch()
    C = NUM_CLASSES.get(k)
    if C is None:
        raise MotifError(-1, "census_batch")
    arr = _graph_array(graphs)
    dev = graphs[0][0].device if graphs else torch.device("cuda")
    hist = out if out is not None else torch.empty((len(graphs), C), dtype=torch.int64, device=dev)
    fn = lib().motif_census_batch_loop if loop else lib().motif_census_batch
    _check(fn(ctypes.cast(arr, ctypes.c_void_p), len(graphs), int(k), _ptr(hist), _stream_handle(stream)),
           "motif_census_batch")
    if out is not None:
        return out
    return hist.cpu().numpy().view(np.uint64)


def census_batch_loop(graphs, k: int, stream=None, out=None):
    return census_batch(graphs, k, stream=stream, out=out, loop=True)


SWITCH_MUTUAL = 1


def null_randomize(graphs, switches_per_arc: int, seed: int, stream=None, mutual: bool = False) -> None:
    """Randomise device graphs [(out_off, out_idx, n), ...] in place by
    switches_per_arc * m degree-preserving arc switches each (out_idx is
    rewritten; rows end up unsorted).  mutual: one-way arcs and reciprocated
    pairs are switched separately (MOTIF_SWITCH_MUTUAL)."""
    arr = _graph_array([g[:3] for g in graphs])
    _check(lib().motif_null_randomize(ctypes.cast(arr, ctypes.c_void_p), len(graphs), int(switches_per_arc),
                                      SWITCH_MUTUAL if mutual else 0, ctypes.c_uint64(seed), _stream_handle(stream)),
           "motif_null_randomize")


def null_model(out_off, out_idx, n: int, count: int, k: int, switches_per_arc: int = 100, seed: int = 0,
               in_off=None, in_idx=None, stream=None, out=None, z_out=None, mutual: bool = False):
    """Randomise, census and score on the device: returns (hists, z) as numpy
    (uint64 [count + 1, C], row 0 the real graph; float64 [C]), or fills the
    CUDA tensors `out` (int64 [count + 1, C]) and `z_out` (float64 [C]).
    mutual: the mutual-preserving switch (MOTIF_SWITCH_MUTUAL)."""
    torch = _torch()
    C = NUM_CLASSES.get(k)
    if C is None:
        raise MotifError(-1, "null_model")
    g = _graph_array([(out_off, out_idx, n) + ((in_off, in_idx) if in_off is not None else ())])
    hist = out if out is not None else torch.empty((count + 1, C), dtype=torch.int64, device=out_off.device)
    z = z_out if z_out is not None else torch.empty(C, dtype=torch.float64, device=out_off.device)
    _check(lib().motif_null_model(ctypes.cast(g, ctypes.c_void_p), int(count), int(k), int(switches_per_arc),
                                  SWITCH_MUTUAL if mutual else 0, ctypes.c_uint64(seed), _ptr(hist), _ptr(z),
                                  _stream_handle(stream)),
           "motif_null_model")
    if out is not None:
        return out, z
    return hist.cpu().numpy().view(np.uint64), z.cpu().numpy()


class BatchPlan:
    """Fused batched census captured once in a hipGraph and replayed.

    The graph tensors must stay alive (and keep their shapes) while the plan
    exists; their contents may change between runs."""

    def __init__(self, graphs, k: int, stream=None, out=None):
        torch = _torch()
        C = NUM_CLASSES.get(k)
        if C is None:
            raise MotifError(-1, "BatchPlan")
        self._graphs = list(graphs)  # keep the device tensors alive
        arr = _graph_array(self._graphs)
        dev = self._graphs[0][0].device
        self.out = out if out is not None else torch.empty((len(self._graphs), C), dtype=torch.int64, device=dev)
        self._stream = stream
        err = ctypes.c_int32()
        self._h = lib().motif_batch_plan_create(ctypes.cast(arr, ctypes.c_void_p), len(self._graphs), int(k),
                                                _ptr(self.out), _stream_handle(stream), ctypes.byref(err))
        if not self._h:
            raise MotifError(err.value, "motif_batch_plan_create")

    def run(self) -> None:
        _check(lib().motif_batch_plan_run(self._h), "motif_batch_plan_run")

    def hists(self) -> np.ndarray:
        return self.out.cpu().numpy().view(np.uint64)

    def close(self):
        if self._h:
            lib().motif_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def get_tuning(k: int) -> dict:
    t = _Tuning()
    _check(lib().motif_get_tuning(k, ctypes.byref(t)), "motif_get_tuning")
    return t.as_dict()


def set_tuning(k: int, block=0, grid_per_cu=0, tile=0, heavy=0, solo_deg=0, light_deg=0, light5=0):
    t = _Tuning(block, grid_per_cu, tile, heavy, solo_deg, light_deg, light5)
    _check(lib().motif_set_tuning(k, ctypes.byref(t)), "motif_set_tuning")


def tune_cache_save(path: str) -> None:
    _check(lib().motif_tune_cache_save(os.fsencode(path)), "motif_tune_cache_save")


def tune_cache_load(path: str) -> int:
    """Entries taken from the file into the current device's tuning cache."""
    r = lib().motif_tune_cache_load(os.fsencode(path))
    if r < 0:
        raise MotifError(r, "motif_tune_cache_load")
    return int(r)


def autotune(graphs, k: int, stream=None) -> dict:
    torch = _torch()
    C = NUM_CLASSES[k]
    arr = _graph_array(graphs)
    hist = torch.empty((len(graphs), C), dtype=torch.int64, device=graphs[0][0].device)
    t = _Tuning()
    _check(lib().motif_autotune(ctypes.cast(arr, ctypes.c_void_p), len(graphs), int(k), _ptr(hist),
                                _stream_handle(stream), ctypes.byref(t)), "motif_autotune")
    return t.as_dict()


def profile_enable(on: bool = True, census_only: bool = False):
    """Record HIP events around the build and the census kernel of every
    call (census_only: around the census kernel only; the build time then
    reads as -1)."""
    _check(lib().motif_profile_enable((2 if census_only else 1) if on else 0), "motif_profile_enable")


def profile_read(k: int):
    """(census kernel ms, build ms) of the last profiled call for k."""
    a, b = ctypes.c_float(), ctypes.c_float()
    _check(lib().motif_profile_read(k, ctypes.byref(a), ctypes.byref(b)), "motif_profile_read")
    return float(a.value), float(b.value)


# --------------------------------------------------------------- serving --

def request_footprint(n: int, m: int, k: int) -> int:
    return int(lib().motif_request_footprint(int(n), int(m), int(k)))


class Server:
    """Continuous-batching census server (host CSR in, host histogram out)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8):
        self._h = lib().motif_server_create(int(hbm_budget_bytes), int(max_inflight))
        if not self._h:
            raise MotifError(-8, "motif_server_create")
        self._keep = {}

    def submit(self, out_off: np.ndarray, out_idx: np.ndarray, n: int, k: int) -> int:
        off = np.ascontiguousarray(out_off, dtype=np.int32)
        idx = np.ascontiguousarray(out_idx, dtype=np.int32)
        hist = np.zeros(NUM_CLASSES[k], dtype=np.uint64)
        g = _Graph(off.ctypes.data, idx.ctypes.data if idx.size else 0, None, None, int(n), int(idx.size))
        ticket = ctypes.c_uint64()
        rc = lib().motif_server_submit(self._h, ctypes.byref(g), int(k), hist.ctypes.data, ctypes.byref(ticket))
        _check(rc, "motif_server_submit")
        self._keep[ticket.value] = hist
        return int(ticket.value)

    def wait(self, ticket: int, timeout_us: int = -1) -> np.ndarray:
        rc = lib().motif_server_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us))
        if rc == -11:
            raise TimeoutError(f"ticket {ticket}")
        hist = self._keep.pop(ticket)
        _check(rc, "motif_server_wait")
        return hist

    def cancel(self, ticket: int) -> int:
        return int(lib().motif_server_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().motif_server_stats(self._h, *[ctypes.byref(x) for x in v]), "motif_server_stats")
        return dict(zip(["completed", "inflight", "bytes_inflight", "peak_bytes"], [x.value for x in v]))

    def close(self):
        if self._h:
            lib().motif_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
