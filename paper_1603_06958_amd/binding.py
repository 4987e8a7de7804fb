"""ctypes binding of libfamsa_lcs.so -- argument marshalling only.

Every step of the similarity computation runs in the HIP library; this
module converts numpy arrays to pointers, wraps Python callables as tile
callbacks and raises ``FamsaError`` on nonzero status.  It fails loudly when
the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Callable, Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfamsa_lcs.so")

OK, EINVAL, ENOMEM, EDEVICE, ECANCELED, EBUSY = 0, -1, -2, -3, -4, -5
PLAIN, DESCENDING, DEVICE_TILES, NO_GRAPH, NO_AUTOTUNE, ONE_STREAM = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
OUT_INDEL, OUT_SIM = 0x40, 0x80
PLAIN_ASYNC = 0x100
TWO_STREAMS = 0x200
LONG_SEGMENTED = 0x400
VALUES_LCS, VALUES_INDEL, VALUES_SIM = 0, 1, 2
MAX_LEN = 65535

_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ECANCELED: "ECANCELED", EBUSY: "EBUSY"}


class FamsaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("alphabet_size", ctypes.c_uint32),
                ("tile_rows", ctypes.c_uint32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("hbm_budget", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("cols_per_item", ctypes.c_uint32),
                ("step_values", ctypes.c_uint64), ("step_cells", ctypes.c_uint64)]


class Tile(ctypes.Structure):
    _fields_ = [("tile_index", ctypes.c_uint64), ("family", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("row_begin", ctypes.c_uint32), ("row_end", ctypes.c_uint32),
                ("lcs", ctypes.POINTER(ctypes.c_int32)), ("count", ctypes.c_uint64), ("stream", ctypes.c_void_p),
                ("values", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("ntiles", ctypes.c_uint64), ("nsteps", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("cells", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("pinned_bytes", ctypes.c_uint64),
                ("max_tile_values", ctypes.c_uint64), ("nfam", ctypes.c_uint32), ("max_len", ctypes.c_uint32),
                ("cols_per_item", ctypes.c_uint32), ("waves_per_group", ctypes.c_uint32 * 4)]


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double * 5), ("launches", ctypes.c_uint64 * 5),
                ("cells", ctypes.c_uint64 * 5), ("step_ms", ctypes.c_double), ("steps", ctypes.c_uint64),
                ("wall_ms", ctypes.c_double), ("tiles", ctypes.c_uint64)]


class PeakResult(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("lane_ops", ctypes.c_double), ("ops_per_s", ctypes.c_double),
                ("clock_ghz", ctypes.c_double), ("mean_loop_cycles", ctypes.c_double),
                ("lane_ops_per_clk_per_cu", ctypes.c_double), ("cus", ctypes.c_uint32)]


TILE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(Tile))

_lib = None


def lib():
    """Load libfamsa_lcs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FamsaError(EDEVICE, f"{LIB_PATH} is missing: build it with `python -m paper_1603_06958_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, u8p, u32p, u64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint32), \
            ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.famsa_lcs_default_options.argtypes = [ctypes.POINTER(Options)]
        L.famsa_lcs_default_options.restype = None
        L.famsa_lcs_plan.argtypes = [u8p, u64p, ctypes.c_uint32, u32p, ctypes.c_uint32, ctypes.POINTER(Options),
                                     ctypes.POINTER(vp)]
        L.famsa_lcs_plan.restype = ctypes.c_int
        L.famsa_lcs_tiles.argtypes = [vp, ctypes.c_uint64, TILE_FN, vp]
        L.famsa_lcs_tiles.restype = ctypes.c_int
        L.famsa_lcs_release.argtypes = [vp]
        L.famsa_lcs_release.restype = None
        L.famsa_lcs_last_error.argtypes = []
        L.famsa_lcs_last_error.restype = ctypes.c_char_p
        L.famsa_lcs_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.famsa_lcs_plan_get_info.restype = ctypes.c_int
        L.famsa_lcs_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.famsa_lcs_get_stats.restype = ctypes.c_int
        L.famsa_lcs_autotune.argtypes = [vp, ctypes.c_char_p]
        L.famsa_lcs_autotune.restype = ctypes.c_int
        L.famsa_slink_create.argtypes = [u32p, ctypes.c_uint32, ctypes.POINTER(vp)]
        L.famsa_slink_create.restype = ctypes.c_int
        L.famsa_slink_consume.argtypes = [vp, ctypes.POINTER(Tile)]
        L.famsa_slink_consume.restype = ctypes.c_int
        L.famsa_slink_result.argtypes = [vp, u32p, i64p, i64p]
        L.famsa_slink_result.restype = ctypes.c_int
        L.famsa_slink_rows_done.argtypes = [vp]
        L.famsa_slink_rows_done.restype = ctypes.c_uint32
        L.famsa_slink_destroy.argtypes = [vp]
        L.famsa_slink_destroy.restype = None
        L.famsa_mst_create.argtypes = [u32p, ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(vp)]
        L.famsa_mst_create.restype = ctypes.c_int
        L.famsa_mst_consume.argtypes = [vp, ctypes.POINTER(Tile)]
        L.famsa_mst_consume.restype = ctypes.c_int
        L.famsa_mst_result.argtypes = [vp, u32p, u32p, i64p, i64p, u32p]
        L.famsa_mst_result.restype = ctypes.c_int
        L.famsa_mst_get_stats.argtypes = [vp, u64p, u64p]
        L.famsa_mst_get_stats.restype = ctypes.c_int
        L.famsa_mst_destroy.argtypes = [vp]
        L.famsa_mst_destroy.restype = None
        L.famsa_mst_guide_tree.argtypes = [vp, u32p, u32p, i64p, i64p, u32p]
        L.famsa_mst_guide_tree.restype = ctypes.c_int
        L.famsa_slink_guide_tree.argtypes = [vp, u32p, u32p, i64p, i64p, u32p]
        L.famsa_slink_guide_tree.restype = ctypes.c_int
        L.famsa_guide_tree.argtypes = [ctypes.c_uint32, u32p, u32p, i64p, i64p, ctypes.c_uint32, u32p, u32p, i64p,
                                       i64p, u32p]
        L.famsa_guide_tree.restype = ctypes.c_int
        L.famsa_spanning_forest.argtypes = [ctypes.c_uint32, u32p, u32p, i64p, i64p, ctypes.c_uint64, u32p, u32p,
                                            i64p, i64p, u32p]
        L.famsa_spanning_forest.restype = ctypes.c_int
        L.famsa_guide_tree_leaf_order.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32, u32p, u32p, u32p]
        L.famsa_guide_tree_leaf_order.restype = ctypes.c_int
        L.famsa_guide_tree_newick.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32, ctypes.c_char_p,
                                              ctypes.c_uint64, u64p]
        L.famsa_guide_tree_newick.restype = ctypes.c_int
        L.famsa_gapped_create.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(vp)]
        L.famsa_gapped_create.restype = ctypes.c_int
        L.famsa_gapped_insert.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, ctypes.c_uint32]
        L.famsa_gapped_insert.restype = ctypes.c_int
        L.famsa_gapped_width.argtypes = [vp, u32p]
        L.famsa_gapped_width.restype = ctypes.c_int
        L.famsa_gapped_locate.argtypes = [vp, u32p, u32p, ctypes.c_uint32, u32p]
        L.famsa_gapped_locate.restype = ctypes.c_int
        L.famsa_gapped_decode.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, u8p, ctypes.c_uint64]
        L.famsa_gapped_decode.restype = ctypes.c_int
        L.famsa_gapped_state.argtypes = [vp, ctypes.c_uint32, u32p, u32p, u32p, u32p]
        L.famsa_gapped_state.restype = ctypes.c_int
        L.famsa_gapped_destroy.argtypes = [vp]
        L.famsa_gapped_destroy.restype = None
        L.famsa_lcs_server_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.famsa_lcs_server_create.restype = ctypes.c_int
        L.famsa_lcs_server_submit.argtypes = [vp, u8p, u64p, ctypes.c_uint32, u32p]
        L.famsa_lcs_server_submit.restype = ctypes.c_int
        L.famsa_lcs_server_step.argtypes = [vp, TILE_FN, vp, u32p]
        L.famsa_lcs_server_step.restype = ctypes.c_int
        L.famsa_lcs_server_job_state.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int)]
        L.famsa_lcs_server_job_state.restype = ctypes.c_int
        L.famsa_lcs_server_memory.argtypes = [vp, u64p, u64p]
        L.famsa_lcs_server_memory.restype = ctypes.c_int
        L.famsa_lcs_server_destroy.argtypes = [vp]
        L.famsa_lcs_server_destroy.restype = None
        L.famsa_valu_peak.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.POINTER(PeakResult)]
        L.famsa_valu_peak.restype = ctypes.c_int
        L.famsa_lcs_family_noalloc.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, vp, vp, ctypes.c_int, vp]
        L.famsa_lcs_family_noalloc.restype = ctypes.c_int
        L.famsa_profile_align.argtypes = [ctypes.c_uint32, u8p, u64p, u8p, u64p, u32p, u32p, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_int32), i64p, ctypes.c_int, i64p, u8p, u64p, u32p]
        L.famsa_profile_align.restype = ctypes.c_int
        L.famsa_profile_last_dp_ms.argtypes = []
        L.famsa_profile_last_dp_ms.restype = ctypes.c_double
        L.famsa_gap_costs_scaled.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                             ctypes.c_double, i64p]
        L.famsa_gap_costs_scaled.restype = ctypes.c_int
        _lib = L
    return _lib


def valu_peak(variant: int = 0, blocks_per_cu: int = 8, iters: int = 20000, device: int = 0) -> PeakResult:
    """Rate of register-only chains of the LCS step's VALU instructions
    (famsa_valu_peak): variant 0 the recurrence, 1 AND, 2 ADDC, 3 BITOP3."""
    r = PeakResult()
    check(lib().famsa_valu_peak(device, variant, blocks_per_cu, iters, ctypes.byref(r)))
    return r


NOALLOC_MAX_SEQ, NOALLOC_MAX_LEN, NOALLOC_MAX_LEN_S32 = 8192, 896, 512


def family_noalloc(codes_ptr: int, seq_off_ptr: int, nseq: int, out_ptr: int, status_ptr: Optional[int] = None,
                   alphabet_size: int = 20, device: int = 0, stream: Optional[int] = None) -> None:
    """famsa_lcs_family_noalloc on device buffers given by address (for
    example torch tensors' data_ptr()): codes uint8, seq_off uint64 (nseq + 1),
    out int32 (nseq (nseq - 1) / 2), status one int32 or None.  Queued on
    `stream`; returns without waiting."""
    check(lib().famsa_lcs_family_noalloc(codes_ptr or None, seq_off_ptr or None, nseq, alphabet_size,
                                         out_ptr or None, status_ptr or None, device, stream))


PROFILE_GAP = 0xFF
OP_M, OP_D, OP_I = 0, 1, 2


def profile_align(problems, subst, gap_costs, alphabet_size: Optional[int] = None, device: int = 0):
    """famsa_profile_align over a list of (sequence, rows) pairs: sequence
    uint8 codes, rows a K x n uint8 array (PROFILE_GAP for gaps).  Returns
    (scores int64 array, list of op arrays)."""
    S = np.ascontiguousarray(subst, dtype=np.int32)
    sigma = int(S.shape[0]) if alphabet_size is None else alphabet_size
    seqs = [np.ascontiguousarray(a, dtype=np.uint8).reshape(-1) for a, _ in problems]
    rows = [np.ascontiguousarray(r, dtype=np.uint8) for _, r in problems]
    n = len(seqs)
    seq_off = np.zeros(n + 1, np.uint64)
    np.cumsum([x.size for x in seqs], out=seq_off[1:])
    rows_off = np.zeros(n + 1, np.uint64)
    np.cumsum([r.size for r in rows], out=rows_off[1:])
    nrows = np.array([r.shape[0] for r in rows], np.uint32)
    width = np.array([r.shape[1] for r in rows], np.uint32)
    ops_off = np.zeros(n + 1, np.uint64)
    np.cumsum([x.size + r.shape[1] for x, r in zip(seqs, rows)], out=ops_off[1:])
    cat_s = np.concatenate(seqs) if n and int(seq_off[-1]) else np.zeros(1, np.uint8)
    cat_r = np.concatenate([r.reshape(-1) for r in rows]) if n and int(rows_off[-1]) else np.zeros(1, np.uint8)
    costs = np.ascontiguousarray(gap_costs, dtype=np.int64)
    score = np.zeros(max(n, 1), np.int64)
    ops = np.zeros(max(int(ops_off[-1]), 1), np.uint8)
    nops = np.zeros(max(n, 1), np.uint32)
    check(lib().famsa_profile_align(n, _ptr(cat_s, ctypes.c_uint8), _ptr(seq_off, ctypes.c_uint64),
                                    _ptr(cat_r, ctypes.c_uint8), _ptr(rows_off, ctypes.c_uint64),
                                    _ptr(nrows, ctypes.c_uint32), _ptr(width, ctypes.c_uint32), sigma,
                                    _ptr(S, ctypes.c_int32), _ptr(costs, ctypes.c_int64), device,
                                    _ptr(score, ctypes.c_int64), _ptr(ops, ctypes.c_uint8),
                                    _ptr(ops_off, ctypes.c_uint64), _ptr(nops, ctypes.c_uint32)))
    return score[:n], [ops[int(ops_off[p]):int(ops_off[p]) + int(nops[p])].copy() for p in range(n)]


def profile_last_dp_ms() -> float:
    return float(lib().famsa_profile_last_dp_ms())


def gap_costs_scaled(k: int, base, gl: float = 45.0, gd: float = 7.0) -> Tuple[int, int, int, int]:
    """(To, Te, Go, Ge) scaled by 1 + ln(k / gl) / gd and rounded (famsa_gap_costs_scaled)."""
    b = np.ascontiguousarray(base, dtype=np.float64)
    out = np.zeros(4, np.int64)
    check(lib().famsa_gap_costs_scaled(k, _ptr(b, ctypes.c_double), gl, gd, _ptr(out, ctypes.c_int64)))
    return tuple(int(x) for x in out)


def last_error() -> str:
    return (lib().famsa_lcs_last_error() or b"").decode()


def check(rc: int):
    if rc != OK:
        raise FamsaError(rc, last_error())
    return rc


def make_options(alphabet_size: int = 20, tile_rows: int = 1024, device: int = 0, stream: Optional[int] = None,
                 hbm_budget: int = 0, flags: int = 0, cols_per_item: int = 0, step_values: int = 0,
                 step_cells: int = 0) -> Options:
    o = Options()
    lib().famsa_lcs_default_options(ctypes.byref(o))
    o.alphabet_size = alphabet_size
    o.tile_rows = tile_rows
    o.device = device
    o.stream = stream
    o.hbm_budget = hbm_budget
    o.flags = flags
    o.cols_per_item = cols_per_item
    o.step_values = step_values
    o.step_cells = step_cells
    return o


def torch_stream_handle() -> Optional[int]:
    """hipStream_t of torch's current stream on the current device (None if torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class Plan:
    """A famsa_lcs plan over a batch of families (see include/famsa_lcs.h)."""

    def __init__(self, codes: np.ndarray, seq_off: np.ndarray, fam_off: Optional[np.ndarray] = None, **opts):
        self._codes = np.ascontiguousarray(codes, dtype=np.uint8)
        self._off = np.ascontiguousarray(seq_off, dtype=np.uint64)
        self._fam = None if fam_off is None else np.ascontiguousarray(fam_off, dtype=np.uint32)
        nseq = self._off.size - 1
        self.options = make_options(**opts)
        h = ctypes.c_void_p()
        cp = _ptr(self._codes, ctypes.c_uint8) if self._codes.size else None
        fp = _ptr(self._fam, ctypes.c_uint32) if self._fam is not None else None
        nfam = 0 if self._fam is None else self._fam.size - 1
        check(lib().famsa_lcs_plan(cp, _ptr(self._off, ctypes.c_uint64), nseq, fp, nfam,
                                   ctypes.byref(self.options), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_batch(cls, b, **opts) -> "Plan":
        return cls(b.codes, b.seq_off, b.fam_off, **opts)

    def close(self):
        if getattr(self, "handle", None):
            lib().famsa_lcs_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> PlanInfo:
        i = PlanInfo()
        check(lib().famsa_lcs_plan_get_info(self.handle, ctypes.byref(i)))
        return i

    def stats(self) -> Stats:
        s = Stats()
        check(lib().famsa_lcs_get_stats(self.handle, ctypes.byref(s)))
        return s

    def run(self, fn: Callable[[Tile], int], first_tile: int = 0) -> int:
        """Deliver tiles to fn(tile) (a ctypes Tile); fn returns 0 to continue."""
        err = []

        def cb(_user, tp):
            try:
                return int(fn(tp.contents) or 0)
            except BaseException as e:  # never let an exception cross the C frame
                err.append(e)
                return 1

        c = TILE_FN(cb)
        rc = lib().famsa_lcs_tiles(self.handle, first_tile, c, None)
        if err:
            raise err[0]
        return check(rc)

    def run_native(self, fn_ptr, user, first_tile: int = 0) -> int:
        """Deliver tiles to a C callback (e.g. famsa_slink_consume)."""
        return check(lib().famsa_lcs_tiles(self.handle, first_tile, fn_ptr, user))

    def collect(self, first_tile: int = 0) -> Dict[Tuple[int, int, int], np.ndarray]:
        """All host tiles as {(family, row_begin, row_end): array copy} (int32,
        or float32 similarities under OUT_SIM)."""
        out = {}

        def fn(t: Tile):
            out[(t.family, t.row_begin, t.row_end)] = tile_array(t).copy()
            return 0

        self.run(fn, first_tile)
        return out

    def autotune(self, cache_path: Optional[str] = None) -> int:
        return check(lib().famsa_lcs_autotune(self.handle, cache_path.encode() if cache_path else None))


def tile_array(t: Tile) -> np.ndarray:
    """View of a host tile's values (valid during the callback only): int32
    LCS or indel values, or float32 similarities under OUT_SIM."""
    dt = np.float32 if t.values == VALUES_SIM else np.int32
    if t.count == 0:
        return np.zeros(0, dt)
    a = np.ctypeslib.as_array(t.lcs, shape=(t.count,))
    return a.view(np.float32) if dt is np.float32 else a


def _merges(k, call):
    n = max(k - 1, 1)
    left, right = np.zeros(n, np.uint32), np.zeros(n, np.uint32)
    num, den = np.zeros(n, np.int64), np.zeros(n, np.int64)
    nm = ctypes.c_uint32()
    check(call(_ptr(left, ctypes.c_uint32), _ptr(right, ctypes.c_uint32), _ptr(num, ctypes.c_int64),
               _ptr(den, ctypes.c_int64), ctypes.byref(nm)))
    m = int(nm.value)
    return left[:m], right[:m], num[:m], den[:m]


def guide_tree(k: int, u, v, num, den):
    """famsa_guide_tree: single-linkage merges of a spanning forest's edges."""
    u, v = np.ascontiguousarray(u, np.uint32), np.ascontiguousarray(v, np.uint32)
    num, den = np.ascontiguousarray(num, np.int64), np.ascontiguousarray(den, np.int64)
    ne = u.size
    return _merges(k, lambda l, r, a, b, nm: lib().famsa_guide_tree(
        k, _ptr(u, ctypes.c_uint32) if ne else None, _ptr(v, ctypes.c_uint32) if ne else None,
        _ptr(num, ctypes.c_int64) if ne else None, _ptr(den, ctypes.c_int64) if ne else None, ne, l, r, a, b, nm))


def spanning_forest(k: int, u, v, num, den):
    """famsa_spanning_forest: (u, v, num, den) of the maximum spanning forest of the edges."""
    u, v = np.ascontiguousarray(u, np.uint32), np.ascontiguousarray(v, np.uint32)
    num, den = np.ascontiguousarray(num, np.int64), np.ascontiguousarray(den, np.int64)
    n = max(k - 1, 1)
    ou, ov = np.zeros(n, np.uint32), np.zeros(n, np.uint32)
    on, od = np.zeros(n, np.int64), np.zeros(n, np.int64)
    cnt = ctypes.c_uint32()
    ne = u.size
    check(lib().famsa_spanning_forest(k, _ptr(u, ctypes.c_uint32) if ne else None, _ptr(v, ctypes.c_uint32) if ne else None,
                                      _ptr(num, ctypes.c_int64) if ne else None, _ptr(den, ctypes.c_int64) if ne else None,
                                      ne, _ptr(ou, ctypes.c_uint32), _ptr(ov, ctypes.c_uint32), _ptr(on, ctypes.c_int64),
                                      _ptr(od, ctypes.c_int64), ctypes.byref(cnt)))
    m = int(cnt.value)
    return ou[:m], ov[:m], on[:m], od[:m]


def newick(left, right, k: int) -> str:
    """famsa_guide_tree_newick: the merge list in Newick form."""
    left = np.ascontiguousarray(left, np.uint32)
    right = np.ascontiguousarray(right, np.uint32)
    m = left.size
    lp = _ptr(left, ctypes.c_uint32) if m else None
    rp = _ptr(right, ctypes.c_uint32) if m else None
    need = ctypes.c_uint64()
    check(lib().famsa_guide_tree_newick(k, lp, rp, m, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(int(need.value))
    check(lib().famsa_guide_tree_newick(k, lp, rp, m, buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def leaf_order(left, right, k: int):
    """famsa_guide_tree_leaf_order: (order, first, size)."""
    left = np.ascontiguousarray(left, np.uint32)
    right = np.ascontiguousarray(right, np.uint32)
    m = left.size
    order = np.zeros(max(k, 1), np.uint32)
    first = np.zeros(max(k + m, 1), np.uint32)
    size = np.zeros(max(k + m, 1), np.uint32)
    check(lib().famsa_guide_tree_leaf_order(k, _ptr(left, ctypes.c_uint32) if m else None,
                                            _ptr(right, ctypes.c_uint32) if m else None, m,
                                            _ptr(order, ctypes.c_uint32), _ptr(first, ctypes.c_uint32),
                                            _ptr(size, ctypes.c_uint32)))
    return order[:k], first[:k + m], size[:k + m]


class Gapped:
    """Sequences in the gapped representation on the GPU (famsa_gapped_*)."""

    def __init__(self, codes: np.ndarray, seq_off: np.ndarray, device: int = 0):
        codes = np.ascontiguousarray(codes, np.uint8)
        off = np.ascontiguousarray(seq_off, np.uint64)
        h = ctypes.c_void_p()
        check(lib().famsa_gapped_create(_ptr(codes, ctypes.c_uint8) if codes.size else None,
                                        _ptr(off, ctypes.c_uint64), off.size - 1, device, ctypes.byref(h)))
        self.handle = h
        self.n = int(off.size - 1)

    def insert(self, cols, lens, first: int = 0, count: Optional[int] = None):
        cols = np.ascontiguousarray(cols, np.uint32)
        lens = np.ascontiguousarray(lens, np.uint32)
        count = self.n - first if count is None else count
        check(lib().famsa_gapped_insert(self.handle, first, count, _ptr(cols, ctypes.c_uint32) if cols.size else None,
                                        _ptr(lens, ctypes.c_uint32) if lens.size else None, cols.size))

    def width(self) -> np.ndarray:
        w = np.zeros(max(self.n, 1), np.uint32)
        check(lib().famsa_gapped_width(self.handle, _ptr(w, ctypes.c_uint32)))
        return w[:self.n]

    def locate(self, seq, col) -> np.ndarray:
        seq = np.ascontiguousarray(seq, np.uint32)
        col = np.ascontiguousarray(col, np.uint32)
        out = np.zeros(max(seq.size, 1), np.uint32)
        check(lib().famsa_gapped_locate(self.handle, _ptr(seq, ctypes.c_uint32), _ptr(col, ctypes.c_uint32), seq.size,
                                        _ptr(out, ctypes.c_uint32)))
        return out[:seq.size]

    def decode(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        """Rows of symbol codes, 0xFF for gaps (and for padding past a row's width)."""
        count = self.n - first if count is None else count
        w = self.width()[first:first + count]
        rb = int(w.max()) if w.size and w.max() > 0 else 1
        out = np.full((max(count, 1), rb), 0xFF, np.uint8)
        check(lib().famsa_gapped_decode(self.handle, first, count, _ptr(out, ctypes.c_uint8), rb))
        return out[:count]

    def state(self, s: int):
        n, p = ctypes.c_uint32(), ctypes.c_uint32()
        check(lib().famsa_gapped_state(self.handle, s, None, None, ctypes.byref(n), ctypes.byref(p)))
        gaps = np.zeros(n.value, np.uint32)
        dps = np.zeros(p.value, np.uint32)
        check(lib().famsa_gapped_state(self.handle, s, _ptr(gaps, ctypes.c_uint32), _ptr(dps, ctypes.c_uint32),
                                       None, None))
        return gaps, dps

    def close(self):
        if getattr(self, "handle", None):
            lib().famsa_gapped_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SLink:
    """Host single-linkage consumer (famsa_slink_*)."""

    def __init__(self, lengths: np.ndarray):
        self._len = np.ascontiguousarray(lengths, dtype=np.uint32)
        h = ctypes.c_void_p()
        check(lib().famsa_slink_create(_ptr(self._len, ctypes.c_uint32) if self._len.size else None,
                                       self._len.size, ctypes.byref(h)))
        self.handle = h
        self.k = int(self._len.size)

    # the C function pointer to hand to Plan.run_native
    @staticmethod
    def consume_fn():
        return ctypes.cast(lib().famsa_slink_consume, TILE_FN)

    def feed(self, t: Tile) -> int:
        return lib().famsa_slink_consume(self.handle, ctypes.byref(t))

    def rows_done(self) -> int:
        return int(lib().famsa_slink_rows_done(self.handle))

    def result(self):
        pi = np.zeros(self.k, np.uint32)
        num = np.zeros(self.k, np.int64)
        den = np.zeros(self.k, np.int64)
        check(lib().famsa_slink_result(self.handle, _ptr(pi, ctypes.c_uint32), _ptr(num, ctypes.c_int64),
                                       _ptr(den, ctypes.c_int64)))
        return pi, num, den

    def guide_tree(self):
        """(left, right, num, den) of the k-1 merges (famsa_slink_guide_tree)."""
        return _merges(self.k, lambda *a: lib().famsa_slink_guide_tree(self.handle, *a))

    def close(self):
        if getattr(self, "handle", None):
            lib().famsa_slink_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mst:
    """GPU single-linkage consumer (famsa_mst_*): feed device tiles."""

    def __init__(self, lengths: np.ndarray, device: int = 0):
        self._len = np.ascontiguousarray(lengths, dtype=np.uint32)
        h = ctypes.c_void_p()
        check(lib().famsa_mst_create(_ptr(self._len, ctypes.c_uint32) if self._len.size else None,
                                     self._len.size, device, ctypes.byref(h)))
        self.handle = h
        self.k = int(self._len.size)

    @staticmethod
    def consume_fn():
        return ctypes.cast(lib().famsa_mst_consume, TILE_FN)

    def result(self):
        n = max(self.k, 1)
        u = np.zeros(n, np.uint32)
        v = np.zeros(n, np.uint32)
        L = np.zeros(n, np.int64)
        D = np.zeros(n, np.int64)
        ne = ctypes.c_uint32()
        check(lib().famsa_mst_result(self.handle, _ptr(u, ctypes.c_uint32), _ptr(v, ctypes.c_uint32),
                                     _ptr(L, ctypes.c_int64), _ptr(D, ctypes.c_int64), ctypes.byref(ne)))
        m = int(ne.value)
        return u[:m], v[:m], L[:m], D[:m]

    def stats(self):
        t, r = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().famsa_mst_get_stats(self.handle, ctypes.byref(t), ctypes.byref(r)))
        return int(t.value), int(r.value)

    def guide_tree(self):
        """(left, right, lcs, indel2) of the k-1 merges (famsa_mst_guide_tree)."""
        return _merges(self.k, lambda *a: lib().famsa_mst_guide_tree(self.handle, *a))

    def close(self):
        if getattr(self, "handle", None):
            lib().famsa_mst_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
