"""Thin Python binding of the tgw C ABI (include/tgw.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the scan runs in the library's gfx950 kernels.  The
names mirror the C entry points without the ``tgw_`` prefix.  If libtgw.so
is missing this module raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Dict, List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtgw.so")
INCLUDE_DIR = os.path.join(os.path.dirname(_HERE), "include")
HEADER_PATH = os.path.join(INCLUDE_DIR, "tgw.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not built; run paper_2604_21095_amd/build.py (or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

# status codes
OK = 0
ERR_INVALID_ARG = 1
ERR_SHAPE = 2
ERR_RANK_DEFICIENT = 3
ERR_NONFINITE = 4
ERR_DEVICE = 5
ERR_OUT_OF_MEMORY = 6
ERR_UNSUPPORTED = 7
ERR_TAIL_OVERFLOW = 8

PREC_FP32 = 0
PREC_SPLIT = 1
PREC_SPLIT_F16 = 2
PREC_SPLIT_F8 = 3
F16_SCALE = 4096.0  # the FP16 forms store 2^12 times the operand
CODE_DOSAGE = 0
CODE_PLINK_BED = 1
CODE_DOSAGE8 = 2  # one byte per sample: q / 127 copies, 255 missing
_PREC = {"fp32": PREC_FP32, "split": PREC_SPLIT, "split16": PREC_SPLIT_F16, "split8": PREC_SPLIT_F8,
         PREC_FP32: PREC_FP32, PREC_SPLIT: PREC_SPLIT, PREC_SPLIT_F16: PREC_SPLIT_F16,
         PREC_SPLIT_F8: PREC_SPLIT_F8}

OUTPUT_NAMES = ("r", "beta", "se", "t", "nlog10p")


class Outputs(ctypes.Structure):
    _fields_ = [("r", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("se", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("nlog10p", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("best", ctypes.c_void_p), ("topk", ctypes.c_void_p), ("topk_k", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Hit(ctypes.Structure):
    _fields_ = [("marker", ctypes.c_int64), ("panel", ctypes.c_int32), ("pheno", ctypes.c_int32),
                ("nlog10p", ctypes.c_float), ("r", ctypes.c_float)]


HIT_DTYPE_BYTES = ctypes.sizeof(Hit)  # 24


class PlanOptions(ctypes.Structure):
    _fields_ = [("block_markers", ctypes.c_int64), ("tail_capacity", ctypes.c_int64),
                ("tile", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_pp = ctypes.POINTER(ctypes.c_void_p)


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_status_string = _sig("tgw_status_string", ctypes.c_char_p, ctypes.c_int)
_last_error = _sig("tgw_last_error", ctypes.c_char_p)
abi_version = _sig("tgw_abi_version", _i32)
_init = _sig("tgw_init", ctypes.c_int)
_fit = _sig("tgw_fit_covariates", ctypes.c_int, _i64, _i32, _vp, _i64, _vp, _pp)
_cov_free = _sig("tgw_covariates_free", None, _vp)
_cov_q = _sig("tgw_covariates_q", ctypes.c_int, _vp, _vp, _i64, _vp)
_prep = _sig("tgw_prepare_phenotypes", ctypes.c_int, _vp, _i64, _vp, _i32, _i64, ctypes.c_int, _vp, _pp)
_panel_free = _sig("tgw_panel_free", None, _vp)
_panel_info = _sig("tgw_panel_info", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                   ctypes.POINTER(_i32), ctypes.POINTER(_i64))
_plan_create = _sig("tgw_plan_create", ctypes.c_int, ctypes.POINTER(_vp), _i32, ctypes.POINTER(PlanOptions), _pp)
_plan_free = _sig("tgw_plan_free", None, _vp)
_plan_info = _sig("tgw_plan_info", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                  ctypes.POINTER(_i64))
_tile_shape = _sig("tgw_tile_shape", ctypes.c_int, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                   ctypes.POINTER(_i32))
_autotune = _sig("tgw_plan_autotune", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.c_int, _i64, _i64,
                 ctypes.POINTER(Outputs), _vp, ctypes.POINTER(ctypes.c_double))
_scan = _sig("tgw_scan", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.c_int, _i64, _i64, ctypes.POINTER(Outputs), _vp)
_plan_check = _sig("tgw_plan_check", ctypes.c_int, _vp, _vp, ctypes.POINTER(_i64))
_plan_set_hits = _sig("tgw_plan_set_hits", ctypes.c_int, _vp, _vp, _i64, _vp, ctypes.c_float)
_profile = _sig("tgw_plan_profile", ctypes.c_int, _vp, _i32)
_profile_read = _sig("tgw_plan_profile_read", ctypes.c_int, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                     ctypes.POINTER(_i64))
_graph_create = _sig("tgw_graph_create", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.c_int, _i64, _i64,
                     ctypes.POINTER(Outputs), _pp)
_graph_launch = _sig("tgw_graph_launch", ctypes.c_int, _vp, _vp)
_graph_free = _sig("tgw_graph_free", None, _vp)
_bed_open = _sig("tgw_bed_open", ctypes.c_int, ctypes.c_char_p, _i64, _pp)
_bed_close = _sig("tgw_bed_close", None, _vp)
_bed_info = _sig("tgw_bed_info", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_bed_select = _sig("tgw_bed_select", ctypes.c_int, _vp, ctypes.POINTER(_i64), _i64)
_bed_read = _sig("tgw_bed_read", ctypes.c_int, _vp, _i64, _i64, _vp, _i64)
_fam_match = _sig("tgw_fam_match", ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p), _i64,
                  ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_scan_bed = _sig("tgw_scan_bed", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.POINTER(Outputs), _i64, _i32, _vp)
_dbg_contract = _sig("tgw_debug_contract", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.c_int, _i64, _i64, _vp, _i64,
                     _vp)
_dbg_set_operand = _sig("tgw_debug_set_operand", ctypes.c_int, _vp, _vp, _i64, _vp)
_dbg_stats = _sig("tgw_debug_marker_stats", ctypes.c_int, _vp, _vp, _i64, _i64, ctypes.c_int, _i64, _i64, _vp, _vp,
                  _vp, _vp)
_set_allocator = _sig("tgw_set_allocator", ctypes.c_int, _vp, _vp, _vp)
_topk_read = _sig("tgw_topk_read", ctypes.c_int, _vp, _vp, _i32, _vp, _vp, _vp)
_arena_create = _sig("tgw_arena_create", ctypes.c_int, _vp, ctypes.c_size_t, _pp)
_arena_alloc = _sig("tgw_arena_alloc", _vp, ctypes.c_size_t, _vp, _vp)
_arena_free = _sig("tgw_arena_free", None, _vp, _vp, _vp)
_arena_destroy = _sig("tgw_arena_destroy", ctypes.c_int, _vp)
_scan_static = _sig("tgw_scan_static", ctypes.c_int, ctypes.POINTER(_vp), _i32, _vp, _i64, _i64, ctypes.c_int, _i64,
                    _i64, ctypes.POINTER(Outputs), _i32, _vp, _vp)


class AllocCounts(ctypes.Structure):
    """tgw_debug_alloc_counts: what the test allocator (debug_counting_allocator) recorded."""
    _fields_ = [("n_alloc", _i64), ("n_free", _i64), ("bytes", _i64)]


def debug_counting_allocator():
    """Addresses of the library's counting test allocator (hipMalloc / hipFree that
    record into an AllocCounts passed as ctx)."""
    return (ctypes.cast(_lib.tgw_debug_counting_alloc, _vp), ctypes.cast(_lib.tgw_debug_counting_free, _vp))


def set_allocator(alloc_fn=None, free_fn=None, ctx=None):
    """Register C allocator functions (addresses of tgw_alloc_fn / tgw_free_fn) for the
    device memory of handles made afterwards; no arguments restores hipMalloc / hipFree."""
    _check(_set_allocator(alloc_fn, free_fn, ctx), "tgw_set_allocator")


class ArenaStats(ctypes.Structure):
    """tgw_arena_stats."""
    _fields_ = [("capacity", ctypes.c_size_t), ("in_use", ctypes.c_size_t), ("peak", ctypes.c_size_t),
                ("largest_free", ctypes.c_size_t), ("n_blocks", _i64), ("n_free_ranges", _i64),
                ("n_failed", _i64), ("n_bad_free", _i64)]


_arena_info = _sig("tgw_arena_info", ctypes.c_int, _vp, ctypes.POINTER(ArenaStats))


class Arena:
    """tgw_arena over one device buffer: `buffer` is a device tensor (its storage is
    used from its data pointer for nbytes) or, with `nbytes`, a bare device address.
    The arena keeps a reference to the tensor.  register() makes it the allocator of
    the handles created afterwards; close() (TgwError while handles made under it are
    alive) releases the bookkeeping."""

    def __init__(self, buffer, nbytes=None):
        if nbytes is None:
            self.buffer = buffer
            base, nbytes = buffer.data_ptr(), buffer.numel() * buffer.element_size()
        else:
            self.buffer, base = None, int(buffer)
        h = _vp()
        _check(_arena_create(base, nbytes, ctypes.byref(h)), "tgw_arena_create")
        self.handle = h

    @property
    def functions(self):
        """(alloc_fn, free_fn, ctx) for set_allocator."""
        return (ctypes.cast(_lib.tgw_arena_alloc, _vp), ctypes.cast(_lib.tgw_arena_free, _vp), self.handle)

    def register(self):
        set_allocator(*self.functions)
        return self

    def alloc(self, nbytes) -> int:
        """One block straight from the arena (0 when it cannot hold it)."""
        return _arena_alloc(nbytes, None, self.handle) or 0

    def free(self, ptr):
        _arena_free(ptr, None, self.handle)

    def info(self) -> ArenaStats:
        st = ArenaStats()
        _check(_arena_info(self.handle, ctypes.byref(st)), "tgw_arena_info")
        return st

    def close(self):
        if self.handle:
            _check(_arena_destroy(self.handle), "tgw_arena_destroy")
            self.handle = None
            self.buffer = None


def torch_arena(nbytes: int, device=None) -> Arena:
    """An arena over one torch allocation of nbytes on the current (or given) device:
    handles made after .register() take their device memory from torch."""
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device if device is not None else "cuda")
    return Arena(buf)


class TgwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _last_error().decode(errors="replace")
        super().__init__(f"{where}: {_status_string(status).decode()} ({status}): {detail}")


def _check(status: int, where: str):
    if status != OK:
        raise TgwError(status, where)


def status_string(status: int) -> str:
    return _status_string(status).decode()


def header_symbols() -> List[str]:
    """Every function declared in the headers under include/ (tgw.h, tgw_debug.h)."""
    names = set()
    for fn in sorted(os.listdir(INCLUDE_DIR)):
        if fn.endswith(".h"):
            text = open(os.path.join(INCLUDE_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(tgw_\w+)\s*\(", text))
    return sorted(names)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _colmajor(x: torch.Tensor, dtype) -> torch.Tensor:
    """(rows, cols) tensor -> tensor whose memory is column-major rows x cols."""
    x = x.to(dtype)
    if x.dim() == 1:
        x = x[:, None]
    if x.stride(0) == 1 and (x.shape[1] == 1 or x.stride(1) >= x.shape[0]):
        return x
    return x.t().contiguous().t()


def _dev_check(*ts):
    dev = torch.cuda.current_device()
    for t in ts:
        if t is not None and (not t.is_cuda or t.device.index != dev):
            raise ValueError("tensors must be on the current CUDA/HIP device")


def init():
    _check(_init(), "tgw_init")


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------
class Covariates:
    def __init__(self, handle, n, k):
        self._h = handle
        self.n_samples = n
        self.n_cov = k
        self.q = k + 1

    @property
    def handle(self):
        return self._h

    def Q(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.q, self.n_samples), dtype=torch.float64, device="cuda")
        _check(_cov_q(self._h, _ptr(out), self.n_samples, _stream(stream)), "tgw_covariates_q")
        return out.t()

    def __del__(self, _free=_cov_free):  # bound early: module globals are gone at interpreter exit
        if getattr(self, "_h", None):
            _free(self._h)
            self._h = None


def fit_covariates(C: Optional[torch.Tensor], n_samples: Optional[int] = None, stream=None) -> Covariates:
    """C: (N, K) float64 CUDA tensor (or None / K = 0 for intercept only); a
    column-major C is passed through, any other layout is copied transposed."""
    if C is None or C.numel() == 0:
        if n_samples is None:
            n_samples = 0 if C is None else C.shape[0]
        Cc, k, ld = None, 0, max(1, n_samples)
    else:
        _dev_check(C)
        Cc = _colmajor(C, torch.float64)
        n_samples, k = Cc.shape
        ld = Cc.stride(1) if k > 1 else n_samples
    h = ctypes.c_void_p()
    _check(_fit(n_samples, k, _ptr(Cc), ld, _stream(stream), ctypes.byref(h)), "tgw_fit_covariates")
    return Covariates(h, n_samples, k)


class Panel:
    def __init__(self, handle, cov: Covariates, precision: int):
        self._h = handle
        self.cov = cov  # keeps Q alive
        self.precision = precision
        n, p, q, df = _i64(), _i64(), _i32(), _i64()
        _check(_panel_info(handle, ctypes.byref(n), ctypes.byref(p), ctypes.byref(q), ctypes.byref(df)),
               "tgw_panel_info")
        self.n_samples, self.n_pheno, self.q, self.df = n.value, p.value, q.value, df.value

    @property
    def handle(self):
        return self._h

    def debug_set_operand(self, V: torch.Tensor, stream=None):
        """Test hook: overwrite the stored operand with raw (N, P) values."""
        _dev_check(V)
        Vc = _colmajor(V, torch.float32)
        ld = Vc.stride(1) if Vc.shape[1] > 1 else Vc.shape[0]
        _check(_dbg_set_operand(self._h, _ptr(Vc), ld, _stream(stream)), "tgw_debug_set_operand")
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def __del__(self, _free=_panel_free):  # bound early: module globals are gone at interpreter exit
        if getattr(self, "_h", None):
            _free(self._h)
            self._h = None


def prepare_phenotypes(cov: Covariates, Y: torch.Tensor, precision="split", stream=None) -> Panel:
    """Y: (N, P) float32/float64 CUDA tensor.  The library reads a column-major
    matrix (samples of a column contiguous, e.g. Y.t().contiguous().t()), which
    is passed through as it is; any other layout is first copied transposed."""
    _dev_check(Y)
    prec = _PREC[precision]
    fp64 = Y.dtype == torch.float64
    Yc = _colmajor(Y, torch.float64 if fp64 else torch.float32)
    ld = Yc.stride(1) if Yc.shape[1] > 1 else Yc.shape[0]
    h = ctypes.c_void_p()
    _check(_prep(cov.handle, Yc.shape[1], _ptr(Yc), int(fp64), ld, prec, _stream(stream), ctypes.byref(h)),
           "tgw_prepare_phenotypes")
    return Panel(h, cov, prec)


def tile_shape(idx: int):
    a, b, c = _i32(), _i32(), _i32()
    _check(_tile_shape(idx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "tgw_tile_shape")
    return a.value, b.value, c.value


def make_outputs(panel_sizes: Sequence[int], n_rows: int, names=OUTPUT_NAMES) -> List[Dict[str, torch.Tensor]]:
    return [{k: torch.empty((n_rows, p), dtype=torch.float32, device="cuda") for k in names} for p in panel_sizes]


def _outs_array(outs: Sequence[Dict[str, torch.Tensor]], panels, n_rows: int):
    arr = (Outputs * len(panels))()
    for j, (o, pan) in enumerate(zip(outs, panels)):
        ld = None
        for name in OUTPUT_NAMES:
            t = o.get(name) if o else None
            if t is None:
                continue
            _dev_check(t)
            if t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1:
                raise ValueError(f"output {name} must be a row-major float32 matrix")
            if t.shape[0] < n_rows or t.shape[1] < pan.n_pheno:
                raise ValueError(f"output {name} of panel {j} too small")
            if ld is not None and t.stride(0) != ld:
                raise ValueError("all outputs of one panel must share the row stride")
            ld = t.stride(0)
            setattr(arr[j], name, t.data_ptr())
        arr[j].ld = ld if ld is not None else pan.n_pheno
        b = o.get("best") if o else None
        if b is not None:
            _dev_check(b)
            if b.dtype != torch.int64 or b.dim() != 1 or not b.is_contiguous() or b.shape[0] < pan.n_pheno:
                raise ValueError(f"best of panel {j} must be a contiguous int64 vector of n_pheno entries")
            arr[j].best = b.data_ptr()
        tk = o.get("topk") if o else None
        if tk is not None:
            _dev_check(tk)
            if tk.dtype != torch.int64 or tk.dim() != 2 or not tk.is_contiguous() or tk.shape[0] < pan.n_pheno:
                raise ValueError(f"topk of panel {j} must be a contiguous int64 (n_pheno, k) matrix")
            arr[j].topk = tk.data_ptr()
            arr[j].topk_k = tk.shape[1]
    return arr


def make_best(panel_sizes: Sequence[int]) -> List[torch.Tensor]:
    """Zeroed per-phenotype best-test accumulators (one int64 per column)."""
    return [torch.zeros(p, dtype=torch.int64, device="cuda") for p in panel_sizes]


def unpack_best(best: torch.Tensor):
    """(max -log10 p, marker) per column from a best accumulator; marker -1 where none."""
    v = best.cpu().numpy().view("uint64")
    nl = (v >> 32).astype("uint32").view("float32")
    marker = (0xFFFFFFFF - (v & 0xFFFFFFFF)).astype("int64")
    marker[v == 0] = -1
    return nl, marker


def make_topk(panel_sizes: Sequence[int], k: int) -> List[torch.Tensor]:
    """Zeroed per-phenotype top-k lists ((n_pheno, k) int64 words per panel)."""
    return [torch.zeros((p, k), dtype=torch.int64, device="cuda") for p in panel_sizes]


def read_topk(panel: "Panel", words: torch.Tensor, stream=None):
    """-log10 p (FP64 from |t|, NaN for an empty slot) and marker (-1 empty) of a
    top-k list, as (n_pheno, k) float32 and int64 device tensors (tgw_topk_read)."""
    _dev_check(words)
    nl = torch.empty(words.shape, dtype=torch.float32, device="cuda")
    marker = torch.empty(words.shape, dtype=torch.int64, device="cuda")
    _check(_topk_read(panel.handle, _ptr(words), words.shape[1], _ptr(nl), _ptr(marker), _stream(stream)),
           "tgw_topk_read")
    return nl, marker


def make_hits(capacity: int):
    """Device hit list of `capacity` entries and its zeroed counter."""
    return (torch.zeros((capacity, HIT_DTYPE_BYTES // 4), dtype=torch.int32, device="cuda"),
            torch.zeros(1, dtype=torch.int64, device="cuda"))


def read_hits(hits: torch.Tensor, count: torch.Tensor):
    """Hit list as numpy arrays (marker, panel, pheno, nlog10p, r) and the raw count."""
    n = int(count.item())
    raw = hits[: min(n, hits.shape[0])].cpu().numpy()
    marker = raw[:, 0:2].copy().view("int64")[:, 0]
    return {"marker": marker, "panel": raw[:, 2].copy(), "pheno": raw[:, 3].copy(),
            "nlog10p": raw[:, 4].copy().view("float32"), "r": raw[:, 5].copy().view("float32"), "count": n}


class Plan:
    def __init__(self, panels: Sequence[Panel], block_markers: int = 0, tail_capacity: int = 0, tile: int = -1):
        self.panels = list(panels)
        hs = (ctypes.c_void_p * len(self.panels))(*[p.handle.value for p in self.panels])
        opts = PlanOptions(block_markers, tail_capacity, tile, 0)
        h = ctypes.c_void_p()
        _check(_plan_create(hs, len(self.panels), ctypes.byref(opts), ctypes.byref(h)), "tgw_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        t, n, b = _i32(), _i32(), _i64()
        _check(_plan_info(self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(b)), "tgw_plan_info")
        return {"tile": t.value, "n_tiles": n.value, "block_markers": b.value}

    def _args(self, geno: torch.Tensor, m_begin, m_end, code):
        _dev_check(geno)
        if geno.dtype != torch.uint8 or geno.dim() != 2 or not geno.is_contiguous():
            raise ValueError("geno must be a contiguous (n_markers, row_bytes) uint8 tensor")
        m_end = geno.shape[0] if m_end is None else m_end
        return _ptr(geno), geno.shape[0], geno.shape[1], code, m_begin, m_end

    def scan(self, geno, outs, m_begin=0, m_end=None, code=CODE_DOSAGE, stream=None):
        g, nm, rb, code, m0, m1 = self._args(geno, m_begin, m_end, code)
        arr = _outs_array(outs, self.panels, m1 - m0)
        _check(_scan(self._h, g, nm, rb, code, m0, m1, arr, _stream(stream)), "tgw_scan")

    def set_hits(self, hits: Optional[torch.Tensor], count: Optional[torch.Tensor] = None, threshold: float = 7.3):
        """Thresholded hit list for the following scans (make_hits); None turns it off."""
        if hits is None:
            _check(_plan_set_hits(self._h, None, 0, None, ctypes.c_float(0.0)), "tgw_plan_set_hits")
            self._hits = None
            return
        _dev_check(hits)
        _dev_check(count)
        if not hits.is_contiguous() or hits.element_size() * hits.shape[-1] != HIT_DTYPE_BYTES:
            raise ValueError("hits must come from make_hits")
        _check(_plan_set_hits(self._h, _ptr(hits), hits.shape[0], _ptr(count), ctypes.c_float(threshold)),
               "tgw_plan_set_hits")
        self._hits = (hits, count)  # keep the buffers alive while the plan refers to them

    def check(self, stream=None) -> int:
        n = _i64()
        _check(_plan_check(self._h, _stream(stream), ctypes.byref(n)), "tgw_plan_check")
        return n.value

    def autotune(self, geno, outs, m_begin=0, m_end=None, code=CODE_DOSAGE, stream=None) -> float:
        g, nm, rb, code, m0, m1 = self._args(geno, m_begin, m_end, code)
        arr = _outs_array(outs, self.panels, m1 - m0)
        ms = ctypes.c_double()
        _check(_autotune(self._h, g, nm, rb, code, m0, m1, arr, _stream(stream), ctypes.byref(ms)),
               "tgw_plan_autotune")
        return ms.value

    def profile(self, enable: bool = True):
        _check(_profile(self._h, int(enable)), "tgw_plan_profile")

    def profile_read(self, stream=None):
        ms, n = ctypes.c_double(), _i64()
        _check(_profile_read(self._h, _stream(stream), ctypes.byref(ms), ctypes.byref(n)), "tgw_plan_profile_read")
        return ms.value, n.value

    def graph(self, geno, outs, m_begin=0, m_end=None, code=CODE_DOSAGE) -> "Graph":
        g, nm, rb, code, m0, m1 = self._args(geno, m_begin, m_end, code)
        arr = _outs_array(outs, self.panels, m1 - m0)
        h = ctypes.c_void_p()
        _check(_graph_create(self._h, g, nm, rb, code, m0, m1, arr, ctypes.byref(h)), "tgw_graph_create")
        return Graph(h, self, geno, outs)

    def debug_contract(self, geno, m_begin=0, m_end=None, code=CODE_DOSAGE, stream=None) -> torch.Tensor:
        g, nm, rb, code, m0, m1 = self._args(geno, m_begin, m_end, code)
        P = self.panels[0].n_pheno
        S = torch.full((m1 - m0, P), float("nan"), dtype=torch.float32, device="cuda")
        _check(_dbg_contract(self._h, g, nm, rb, code, m0, m1, _ptr(S), P, _stream(stream)), "tgw_debug_contract")
        return S

    def debug_marker_stats(self, geno, m_begin=0, m_end=None, code=CODE_DOSAGE, stream=None):
        g, nm, rb, code, m0, m1 = self._args(geno, m_begin, m_end, code)
        shift = torch.empty(m1 - m0, dtype=torch.float64, device="cuda")
        mean = torch.empty(m1 - m0, dtype=torch.float64, device="cuda")
        scale = torch.empty(m1 - m0, dtype=torch.float64, device="cuda")
        _check(_dbg_stats(self._h, g, nm, rb, code, m0, m1, _ptr(shift), _ptr(mean), _ptr(scale), _stream(stream)),
               "tgw_debug_marker_stats")
        return shift, mean, scale

    def __del__(self, _free=_plan_free):  # bound early: module globals are gone at interpreter exit
        if getattr(self, "_h", None):
            _free(self._h)
            self._h = None


class Bed:
    """A variant-major PLINK 1 .bed file (tgw_bed_*); host-side calls need no GPU."""

    def __init__(self, path: str, n_samples: int):
        h = ctypes.c_void_p()
        _check(_bed_open(os.fsencode(path), n_samples, ctypes.byref(h)), "tgw_bed_open")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        a, b, c = _i64(), _i64(), _i64()
        _check(_bed_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "tgw_bed_info")
        return {"n_file_samples": a.value, "n_markers": b.value, "n_selected": c.value}

    def select(self, idx: Optional[Sequence[int]]):
        if idx is None:
            _check(_bed_select(self._h, None, 0), "tgw_bed_select")
            return
        arr = (_i64 * len(idx))(*[int(i) for i in idx])
        _check(_bed_select(self._h, arr, len(idx)), "tgw_bed_select")

    def read(self, m_begin: int, m_end: int, row_bytes: int):
        """Host rows [m_begin, m_end) with the selection applied, as a numpy uint8 array."""
        import numpy as np
        out = np.empty((m_end - m_begin, row_bytes), dtype=np.uint8)
        _check(_bed_read(self._h, m_begin, m_end, out.ctypes.data if out.size else None, row_bytes), "tgw_bed_read")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _bed_close(self._h)
            self._h = None

    def __del__(self, _free=_bed_close):  # bound early: module globals are gone at interpreter exit
        if getattr(self, "_h", None):
            _free(self._h)
            self._h = None


def fam_match(fam_path: str, ids: Sequence[str]):
    """File sample of each id (-1 if absent), the table's sample count and the number found."""
    arr = (ctypes.c_char_p * len(ids))(*[str(i).encode() for i in ids])
    idx = (_i64 * max(1, len(ids)))()
    nf, nfound = _i64(), _i64()
    _check(_fam_match(os.fsencode(fam_path), arr, len(ids), idx, ctypes.byref(nf), ctypes.byref(nfound)),
           "tgw_fam_match")
    return [idx[i] for i in range(len(ids))], nf.value, nfound.value


def scan_bed(plan: "Plan", bed: Bed, outs, m_begin=0, m_end=None, block_markers=0, n_threads=0, stream=None):
    """tgw_scan_bed: the scan streamed from a .bed file (output row m - m_begin)."""
    m_end = bed.info()["n_markers"] if m_end is None else m_end
    arr = _outs_array(outs, plan.panels, m_end - m_begin)
    _check(_scan_bed(plan.handle, bed.handle, m_begin, m_end, arr, block_markers, n_threads, _stream(stream)),
           "tgw_scan_bed")


class Graph:
    def __init__(self, handle, plan, geno, outs):
        self._h = handle
        self._keep = (plan, geno, outs)

    def launch(self, stream=None):
        _check(_graph_launch(self._h, _stream(stream)), "tgw_graph_launch")

    def __del__(self, _free=_graph_free):  # bound early: module globals are gone at interpreter exit
        if getattr(self, "_h", None):
            _free(self._h)
            self._h = None


def plan_create(panels, **kw) -> Plan:
    return Plan(panels, **kw)


def scan(plan: Plan, geno, outs=None, m_begin=0, m_end=None, code=CODE_DOSAGE, stream=None,
         names=OUTPUT_NAMES):
    """Run the scan; allocates outputs when `outs` is None and returns them."""
    m_end = geno.shape[0] if m_end is None else m_end
    if outs is None:
        outs = make_outputs([p.n_pheno for p in plan.panels], m_end - m_begin, names)
    plan.scan(geno, outs, m_begin, m_end, code, stream)
    return outs


def scan_static(panels: Sequence[Panel], geno, outs, m_begin=0, m_end=None, code=CODE_DOSAGE, tile=-1,
                n_tail: Optional[torch.Tensor] = None, stream=None):
    """tgw_scan_static: the scan without a plan, its workspace in the library's
    static device array (nothing allocated); n_tail (int64 device scalar, optional)
    receives the number of extreme-tail tests."""
    hs = (ctypes.c_void_p * len(panels))(*[p.handle.value for p in panels])
    _dev_check(geno)
    if geno.dtype != torch.uint8 or geno.dim() != 2 or not geno.is_contiguous():
        raise ValueError("geno must be a contiguous (n_markers, row_bytes) uint8 tensor")
    m_end = geno.shape[0] if m_end is None else m_end
    arr = _outs_array(outs, panels, m_end - m_begin)
    _check(_scan_static(hs, len(panels), _ptr(geno), geno.shape[0], geno.shape[1], code, m_begin, m_end, arr, tile,
                        _ptr(n_tail), _stream(stream)), "tgw_scan_static")
