"""ctypes binding of ``libalae.so`` (the C ABI in ``include/alae.h``).

Argument marshalling only: every step of a search runs in the library's HIP
kernels.  The library is loaded on import; a missing library raises
immediately (there is no fallback of any kind).  PyTorch is used only for
device buffers and streams in :meth:`Workspace.search_device`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libalae.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_0274_amd.build`")

# PyTorch-ROCm ships its own HIP runtime under a different file name.  Loading
# torch first makes libalae bind to that same runtime (matching soname), so
# device pointers and streams are shared and only one runtime owns the GPU.
try:  # pragma: no cover - torch is part of the supported environment
    import torch  # noqa: F401
except ImportError:  # ctypes-only use (index building, validation) still works
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

DNA, PROTEIN = 0, 1
ALPHABETS = {"dna": DNA, "protein": PROTEIN}
STATUS = {0: "ALAE_OK", 1: "ALAE_E_ARG", 2: "ALAE_E_ALPHABET", 3: "ALAE_E_SCORING", 4: "ALAE_E_TOO_LONG",
          5: "ALAE_E_NOMEM", 6: "ALAE_E_DEVICE", 7: "ALAE_E_ADMISSION", 8: "ALAE_E_INTERNAL", 9: "ALAE_E_IO",
          10: "ALAE_E_NOT_FOUND"}


class AlaeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.alae_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


class Scoring(ctypes.Structure):
    _fields_ = [("use_matrix", ctypes.c_int32), ("sa", ctypes.c_int32), ("sb", ctypes.c_int32),
                ("matrix", ctypes.POINTER(ctypes.c_int8)), ("sg", ctypes.c_int32), ("ss", ctypes.c_int32)]


class Hits(ctypes.Structure):
    _fields_ = [("query_end", ctypes.POINTER(ctypes.c_uint32)), ("text_end", ctypes.POINTER(ctypes.c_uint64)),
                ("score", ctypes.POINTER(ctypes.c_int32)), ("count", ctypes.c_size_t)]


class Stats(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_uint64), ("entries", ctypes.c_uint64), ("entries_diag", ctypes.c_uint64),
                ("entries_gap2", ctypes.c_uint64), ("entries_gap3", ctypes.c_uint64),
                ("dominated", ctypes.c_uint64), ("emitted", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("levels", ctypes.c_uint64), ("retries", ctypes.c_uint64), ("max_depth", ctypes.c_uint64),
                ("device_ms", ctypes.c_double), ("occ_reads", ctypes.c_uint64), ("sa_reads", ctypes.c_uint64),
                ("text_reads", ctypes.c_uint64), ("frontier_bytes", ctypes.c_uint64),
                ("level_launches", ctypes.c_uint64), ("level_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("general_ms", ctypes.c_double), ("wide_ms", ctypes.c_double), ("chain_steps", ctypes.c_uint64),
                ("wide_steps", ctypes.c_uint64), ("promoted", ctypes.c_uint64),
                ("dominated_gapped", ctypes.c_uint64), ("chain_bytes", ctypes.c_uint64),
                ("merge_ms", ctypes.c_double), ("reused", ctypes.c_uint64), ("replay_chains", ctypes.c_uint64),
                ("partitioned", ctypes.c_uint64), ("leftover", ctypes.c_uint64), ("order_ms", ctypes.c_double),
                ("level_lane_ms", ctypes.c_double), ("level_lane_launches", ctypes.c_uint64),
                ("tail_chains", ctypes.c_uint64), ("tail_depth", ctypes.c_uint64),
                ("wide_entries", ctypes.c_uint64), ("wide_max_steps", ctypes.c_uint64), ("live_ms", ctypes.c_double),
                ("wide_slowest_ms", ctypes.c_double), ("wide_slowest_rows", ctypes.c_uint64),
                ("dominated_qgram", ctypes.c_uint64), ("wide_slowest_start_ms", ctypes.c_double),
                ("device_levels", ctypes.c_uint64), ("graph_captures", ctypes.c_uint64)]

    def reusing_ratio(self) -> float:
        """Equation 6: reused entries over accessed (reused + computed) entries."""
        acc = self.reused + self.entries
        return self.reused / acc if acc else 0.0

    def level_alg_bytes(self) -> int:
        """Algorithmic bytes of the level kernels: one 64-byte granule per
        occurrence-block read plus the frontier records they read and write."""
        return 64 * self.occ_reads + self.frontier_bytes

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MLP_FEATURES = 10
MLP_HIDDEN = 32
MLP_PARAMS = MLP_HIDDEN * MLP_FEATURES + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1


class TraceStruct(ctypes.Structure):
    _fields_ = [("features", ctypes.POINTER(ctypes.c_float)), ("work", ctypes.POINTER(ctypes.c_float)),
                ("capacity", ctypes.c_size_t), ("count", ctypes.c_size_t), ("total", ctypes.c_size_t)]


class SearchOpts(ctypes.Structure):
    _fields_ = [("zero_floor_only", ctypes.c_int32), ("use_domination", ctypes.c_int32),
                ("use_score_filter", ctypes.c_int32), ("use_qprefix", ctypes.c_int32),
                ("use_reuse", ctypes.c_int32), ("order_queues", ctypes.c_int32),
                ("entry_capacity", ctypes.c_uint64), ("hit_capacity", ctypes.c_uint64),
                ("stats", ctypes.POINTER(Stats)), ("order_model", ctypes.c_void_p),
                ("trace", ctypes.POINTER(TraceStruct)), ("partition_threshold", ctypes.c_float),
                ("level_stage", ctypes.c_int32), ("wide_blocks_per_cu", ctypes.c_int32),
                ("lane_waves_per_cu", ctypes.c_int32), ("no_tail_split", ctypes.c_int32),
                ("batch_columns", ctypes.c_uint64), ("level_graph", ctypes.c_int32)]


class TuneTrial(ctypes.Structure):
    _fields_ = [("level_stage", ctypes.c_int32), ("wide_blocks_per_cu", ctypes.c_int32),
                ("lane_waves_per_cu", ctypes.c_int32), ("ms", ctypes.c_double), ("level_graph", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("default_ms", ctypes.c_double), ("best_ms", ctypes.c_double), ("trials", ctypes.c_int32),
                ("trial", TuneTrial * 16)]


class IndexOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("builder", ctypes.c_int32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("sigma", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("C", ctypes.c_uint64 * 21), ("dollar_row", ctypes.c_uint64), ("host_bytes", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("records", ctypes.c_uint64)]


_vp = ctypes.c_void_p
_u8p = ctypes.POINTER(ctypes.c_uint8)
_st = ctypes.c_int


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("alae_last_error", ctypes.c_char_p)
_sig("alae_version", ctypes.c_char_p)
_sig("alae_index_build", _st, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(IndexOpts),
     ctypes.POINTER(_vp))
_sig("alae_index_build_codes", _st, _u8p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(IndexOpts),
     ctypes.POINTER(_vp))
_sig("alae_index_save", _st, _vp, ctypes.c_char_p)
_sig("alae_index_load", _st, ctypes.c_char_p, ctypes.POINTER(IndexOpts), ctypes.POINTER(_vp))
_sig("alae_index_free", None, _vp)
_sig("alae_index_get_info", _st, _vp, ctypes.POINTER(IndexInfo))
_sig("alae_index_copy_sa", _st, _vp, ctypes.POINTER(ctypes.c_uint32))
_sig("alae_index_copy_bwt", _st, _vp, _u8p)
_sig("alae_index_range", _st, _vp, _u8p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64),
     ctypes.POINTER(ctypes.c_uint64))
_sig("alae_search", _st, _vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(SearchOpts), ctypes.POINTER(Hits))
_sig("alae_search_batch", _st, _vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t),
     ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32, ctypes.POINTER(SearchOpts), ctypes.POINTER(Hits))
_sig("alae_hits_free", None, ctypes.POINTER(Hits))
_sig("alae_workspace_create", _st, _vp, ctypes.POINTER(_vp))
_sig("alae_workspace_free", None, _vp)
_sig("alae_search_device", _st, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(SearchOpts), _vp, ctypes.POINTER(ctypes.c_size_t))
_sig("alae_search_device_batch", _st, _vp, _vp, ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t,
     ctypes.POINTER(Scoring), ctypes.c_int32, ctypes.POINTER(SearchOpts), _vp, ctypes.POINTER(ctypes.c_size_t))
_sig("alae_workspace_batch_offsets", _st, _vp, ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t)
_sig("alae_autotune", _st, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(SearchOpts), ctypes.c_int32, _vp, ctypes.POINTER(TuneReport))
class ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("mean_batch", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("span_s", ctypes.c_double)]


_sig("alae_server_create", _st, _vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp))
_sig("alae_server_submit", _st, _vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(ctypes.c_uint64))
_sig("alae_server_poll", _st, _vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(Hits))
_sig("alae_server_get_stats", _st, _vp, ctypes.POINTER(ServerStats))
_sig("alae_server_reset_stats", None, _vp)
_sig("alae_server_destroy", None, _vp)
_fp = ctypes.POINTER(ctypes.c_float)
_sig("alae_mlp_create", _st, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_vp))
_sig("alae_mlp_free", None, _vp)
_sig("alae_mlp_get_params", _st, _vp, _fp)
_sig("alae_mlp_set_params", _st, _vp, _fp)
_sig("alae_mlp_predict", _st, _vp, _fp, ctypes.c_size_t, _fp)
_sig("alae_mlp_loss_grad", _st, _vp, _fp, _fp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), _fp)
_sig("alae_mlp_train", _st, _vp, _fp, _fp, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_float,
     ctypes.c_uint64, ctypes.POINTER(ctypes.c_double))
_sig("alae_workspace_result", _st, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t))
_sig("alae_workspace_copy_result", _st, _vp, _vp, _vp, _vp)
_sig("alae_index_upload", _st, _vp)


class Alignment(ctypes.Structure):
    _fields_ = [("text_start", ctypes.c_uint64), ("query_start", ctypes.c_uint32), ("score", ctypes.c_int32),
                ("ops_offset", ctypes.c_uint64), ("ops_len", ctypes.c_uint32), ("status", ctypes.c_int32)]


class Alignments(ctypes.Structure):
    _fields_ = [("aln", ctypes.POINTER(Alignment)), ("count", ctypes.c_size_t), ("ops", ctypes.POINTER(ctypes.c_char)),
                ("ops_count", ctypes.c_uint64)]


_sig("alae_traceback", _st, _vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(Scoring),
     ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t,
     ctypes.POINTER(Alignments))
_sig("alae_alignments_free", None, ctypes.POINTER(Alignments))


class Karlin(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("K", ctypes.c_double), ("H", ctypes.c_double)]


_sig("alae_karlin_altschul", _st, ctypes.POINTER(Scoring), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(Karlin))
_sig("alae_evalue_threshold", _st, ctypes.POINTER(Karlin), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
     ctypes.POINTER(ctypes.c_int32))
_sig("alae_sharded_build", _st, _u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
     ctypes.POINTER(IndexOpts), ctypes.POINTER(_vp))
_sig("alae_sharded_free", None, _vp)
_sig("alae_sharded_search", _st, _vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(SearchOpts), ctypes.POINTER(Hits))
_sig("alae_index_build_records", _st, _u8p, ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t, ctypes.c_int,
     ctypes.POINTER(IndexOpts), ctypes.POINTER(_vp))
_sig("alae_index_record_of", _st, _vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64))
_sig("alae_search_device_noalloc", _st, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(Scoring), ctypes.c_int32,
     ctypes.POINTER(SearchOpts), _vp, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t))


def _check(status, where):
    if status != 0:
        raise AlaeError(status, where)


def version() -> str:
    return _lib.alae_version().decode()


def make_scoring(sa=1, sb=-3, sg=-5, ss=-2, matrix=None):
    """Scoring of Section 2.1; `matrix` (sigma x sigma, symmetric) switches to matrix mode."""
    sc = Scoring()
    sc.sa, sc.sb, sc.sg, sc.ss = int(sa), int(sb), int(sg), int(ss)
    if matrix is not None:
        arr = np.ascontiguousarray(np.asarray(matrix, dtype=np.int8))
        sc.use_matrix = 1
        sc.matrix = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        sc._keep = arr  # keep the buffer alive with the struct
    else:
        sc.use_matrix = 0
        sc.matrix = None
    return sc


def make_opts(stats: Stats | None = None, use_domination=True, use_score_filter=True, use_qprefix=True,
              entry_capacity=0, hit_capacity=0, zero_floor_only=False, use_reuse=False, order_model=None, trace=None,
              order_queues=0, partition_threshold=0.0, level_stage=0, wide_blocks_per_cu=0, lane_waves_per_cu=0,
              tail_split=True, batch_columns=0, level_graph=0):
    o = SearchOpts()
    o.batch_columns = int(batch_columns)
    o.level_graph = int(level_graph)
    o.no_tail_split = 0 if tail_split else 1
    o.level_stage = int(level_stage)
    o.wide_blocks_per_cu = int(wide_blocks_per_cu)
    o.lane_waves_per_cu = int(lane_waves_per_cu)
    o.partition_threshold = float(partition_threshold)
    o.order_queues = int(order_queues)
    o.use_reuse = 1 if use_reuse else 0
    o.order_model = order_model._h.value if order_model is not None else None
    o.trace = ctypes.pointer(trace._s) if trace is not None else None
    o.zero_floor_only = 1 if zero_floor_only else 0
    o.use_domination = 1 if use_domination else 0
    o.use_score_filter = 1 if use_score_filter else 0
    o.use_qprefix = 1 if use_qprefix else 0
    o.entry_capacity = int(entry_capacity)
    o.hit_capacity = int(hit_capacity)
    o.stats = ctypes.pointer(stats) if stats is not None else None
    return o


def _alpha(alphabet) -> int:
    if isinstance(alphabet, str):
        return ALPHABETS[alphabet.lower()]
    return int(alphabet)


def _decode_letters(alphabet: int) -> bytes:
    return b"ACGT" if alphabet == DNA else b"ARNDCQEGHILKMFPSTWYV"


def codes_to_bytes(codes: np.ndarray, alphabet) -> bytes:
    lut = np.frombuffer(_decode_letters(_alpha(alphabet)), dtype=np.uint8)
    return lut[np.asarray(codes, dtype=np.uint8)].tobytes()


class Index:
    """The FM-index of the reversed text (Section 5)."""

    def __init__(self, handle, alphabet: int):
        self._h = _vp(handle)
        self.alphabet = alphabet

    BUILDERS = {"auto": 0, "host": 1, "gpu": 2}

    @classmethod
    def build(cls, text, alphabet="dna", device: int = 0, builder: str = "auto"):
        """text: str/bytes of letters, or a uint8 array of codes.  builder: "host" (SA-IS),
        "gpu" (prefix doubling on the device) or "auto" (the GPU for texts of 2^22 or more)."""
        a = _alpha(alphabet)
        opts = IndexOpts(device, cls.BUILDERS[builder])
        h = _vp()
        if isinstance(text, np.ndarray):
            arr = np.ascontiguousarray(text, dtype=np.uint8)
            _check(_lib.alae_index_build_codes(arr.ctypes.data_as(_u8p), arr.shape[0], a, ctypes.byref(opts),
                                               ctypes.byref(h)), "alae_index_build_codes")
        else:
            b = text.encode() if isinstance(text, str) else bytes(text)
            _check(_lib.alae_index_build(b, len(b), a, ctypes.byref(opts), ctypes.byref(h)), "alae_index_build")
        return cls(h.value, a)

    @classmethod
    def build_records(cls, records, alphabet="dna", device: int = 0, builder: str = "auto"):
        """A database of records (uint8 code arrays), joined by a separator no alignment crosses;
        text positions count the separators (record r starts at sum of earlier lengths + r)."""
        a = _alpha(alphabet)
        arr = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.uint8) for r in records]))
        lens = (ctypes.c_size_t * len(records))(*[int(len(r)) for r in records])
        opts = IndexOpts(device, cls.BUILDERS[builder])
        h = _vp()
        _check(_lib.alae_index_build_records(arr.ctypes.data_as(_u8p), lens, len(records), a, ctypes.byref(opts),
                                             ctypes.byref(h)), "alae_index_build_records")
        return cls(h.value, a)

    def record_of(self, text_pos: int) -> tuple[int, int]:
        """(record, offset inside it) of a text position."""
        r, o = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.alae_index_record_of(self._h, int(text_pos), ctypes.byref(r), ctypes.byref(o)),
               "alae_index_record_of")
        return int(r.value), int(o.value)

    @classmethod
    def load(cls, path: str, device: int = 0):
        opts = IndexOpts(device, 0)
        h = _vp()
        _check(_lib.alae_index_load(path.encode(), ctypes.byref(opts), ctypes.byref(h)), "alae_index_load")
        idx = cls(h.value, 0)
        idx.alphabet = idx.info()["alphabet"]
        return idx

    def save(self, path: str):
        _check(_lib.alae_index_save(self._h, path.encode()), "alae_index_save")

    def info(self) -> dict:
        inf = IndexInfo()
        _check(_lib.alae_index_get_info(self._h, ctypes.byref(inf)), "alae_index_get_info")
        return {"n": inf.n, "sigma": inf.sigma, "alphabet": inf.alphabet, "C": list(inf.C)[:inf.sigma + 1],
                "dollar_row": inf.dollar_row, "host_bytes": inf.host_bytes, "device_bytes": inf.device_bytes,
                "records": inf.records}

    def sa_end(self) -> np.ndarray:
        n = self.info()["n"]
        out = np.empty(n + 1, dtype=np.uint32)
        _check(_lib.alae_index_copy_sa(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
               "alae_index_copy_sa")
        return out

    def bwt(self) -> np.ndarray:
        n = self.info()["n"]
        out = np.empty(n + 1, dtype=np.uint8)
        _check(_lib.alae_index_copy_bwt(self._h, out.ctypes.data_as(_u8p)), "alae_index_copy_bwt")
        return out

    def upload(self):
        """Put the index on its device now (alae_index_upload)."""
        _check(_lib.alae_index_upload(self._h), "alae_index_upload")

    def range(self, pattern_codes) -> tuple[int, int]:
        arr = np.ascontiguousarray(np.asarray(pattern_codes, dtype=np.uint8))
        lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.alae_index_range(self._h, arr.ctypes.data_as(_u8p), arr.shape[0], ctypes.byref(lo),
                                     ctypes.byref(hi)), "alae_index_range")
        return int(lo.value), int(hi.value)

    def free(self):
        if self._h:
            _lib.alae_index_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _hits_to_numpy(h: Hits):
    n = int(h.count)
    if n == 0:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64))
    j = np.ctypeslib.as_array(h.query_end, shape=(n,)).astype(np.int64)
    t = np.ctypeslib.as_array(h.text_end, shape=(n,)).astype(np.int64)
    s = np.ctypeslib.as_array(h.score, shape=(n,)).astype(np.int64)
    return j, t, s


def _query_bytes(query, alphabet: int) -> bytes:
    if isinstance(query, np.ndarray):
        return codes_to_bytes(query, alphabet)
    return query.encode() if isinstance(query, str) else bytes(query)


def search(index: Index, query, H: int, scoring: Scoring | None = None, stats: Stats | None = None, **opt):
    """One search; returns (query_end, text_end, score) int64 arrays sorted by (query_end, text_end)."""
    sc = scoring if scoring is not None else make_scoring()
    q = _query_bytes(query, index.alphabet)
    opts = make_opts(stats=stats, **opt)
    h = Hits()
    _check(_lib.alae_search(index._h, q, len(q), ctypes.byref(sc), int(H), ctypes.byref(opts), ctypes.byref(h)),
           "alae_search")
    try:
        return _hits_to_numpy(h)
    finally:
        _lib.alae_hits_free(ctypes.byref(h))


def search_batch(index: Index, queries, H: int, scoring: Scoring | None = None, stats: Stats | None = None, **opt):
    """k searches in one call; returns a list of (query_end, text_end, score) triples."""
    sc = scoring if scoring is not None else make_scoring()
    qs = [_query_bytes(q, index.alphabet) for q in queries]
    k = len(qs)
    arr = (ctypes.c_char_p * k)(*qs)
    lens = (ctypes.c_size_t * k)(*[len(q) for q in qs])
    outs = (Hits * k)()
    opts = make_opts(stats=stats, **opt)
    _check(_lib.alae_search_batch(index._h, arr, lens, k, ctypes.byref(sc), int(H), ctypes.byref(opts), outs),
           "alae_search_batch")
    res = []
    for i in range(k):
        res.append(_hits_to_numpy(outs[i]))
        _lib.alae_hits_free(ctypes.byref(outs[i]))
    return res


def search_device_noalloc(index: Index, d_query, H: int, d_keys, d_scores, scoring: Scoring | None = None,
                          stats: Stats | None = None, stream=None, **opt) -> int:
    """alae_search_device_noalloc: the search with every buffer in the library's fixed per-device
    array.  d_query (uint8 codes), d_keys (int64) and d_scores (int32) are torch tensors on the GPU;
    the capacity is d_keys.numel().  Returns the hit count (records written)."""
    sc = scoring if scoring is not None else make_scoring()
    opts = make_opts(stats=stats, **opt)
    cnt = ctypes.c_size_t()
    cap = int(d_keys.numel())
    if int(d_scores.numel()) < cap:
        raise ValueError("d_scores holds fewer records than d_keys")
    sptr = _vp(stream.cuda_stream) if stream is not None else None
    _check(_lib.alae_search_device_noalloc(index._h, _vp(d_query.data_ptr()), int(d_query.numel()), ctypes.byref(sc),
                                           int(H), ctypes.byref(opts), sptr, _vp(d_keys.data_ptr()),
                                           _vp(d_scores.data_ptr()), cap, ctypes.byref(cnt)),
           "alae_search_device_noalloc")
    return int(cnt.value)


class ShardedIndex:
    """A text cut into shards of `shard_len` text ends, each indexed from `overlap` characters
    before its first end (exact for queries whose L_max is at most overlap + 1)."""

    def __init__(self, text, alphabet="dna", shard_len=1 << 28, overlap=1 << 20, max_resident=0, device=0,
                 builder="auto"):
        a = _alpha(alphabet)
        arr = np.ascontiguousarray(np.asarray(text, dtype=np.uint8))
        opts = IndexOpts(device, Index.BUILDERS[builder])
        self._h = _vp()
        self.alphabet = a
        _check(_lib.alae_sharded_build(arr.ctypes.data_as(_u8p), arr.shape[0], a, int(shard_len), int(overlap),
                                       int(max_resident), ctypes.byref(opts), ctypes.byref(self._h)),
               "alae_sharded_build")

    def search(self, query, H: int, scoring: Scoring | None = None, stats: Stats | None = None, **opt):
        """(query_end, text_end, score) int64 arrays sorted by (query_end, text_end), text ends global."""
        sc = scoring if scoring is not None else make_scoring()
        q = _query_bytes(query, self.alphabet)
        opts = make_opts(stats=stats, **opt)
        h = Hits()
        _check(_lib.alae_sharded_search(self._h, q, len(q), ctypes.byref(sc), int(H), ctypes.byref(opts),
                                        ctypes.byref(h)), "alae_sharded_search")
        try:
            return _hits_to_numpy(h)
        finally:
            _lib.alae_hits_free(ctypes.byref(h))

    def free(self):
        if self._h:
            _lib.alae_sharded_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def traceback(index: Index, query, query_ends, text_ends, scores, scoring: Scoring | None = None):
    """Start and transcript of the optimal alignment (largest text start, then largest query
    start) of each cell; returns a list of dicts (text_start, query_start, score, ops, status)."""
    sc = scoring if scoring is not None else make_scoring()
    q = _query_bytes(query, index.alphabet)
    j = np.ascontiguousarray(np.asarray(query_ends, dtype=np.uint32))
    t = np.ascontiguousarray(np.asarray(text_ends, dtype=np.uint64))
    s = np.ascontiguousarray(np.asarray(scores, dtype=np.int32))
    out = Alignments()
    _check(_lib.alae_traceback(index._h, q, len(q), ctypes.byref(sc), j.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), j.shape[0], ctypes.byref(out)),
           "alae_traceback")
    try:
        ops = ctypes.string_at(out.ops, out.ops_count).decode() if out.ops_count else ""
        res = []
        for k in range(out.count):
            a = out.aln[k]
            res.append({"text_start": int(a.text_start), "query_start": int(a.query_start), "score": int(a.score),
                        "ops": ops[a.ops_offset:a.ops_offset + a.ops_len], "status": int(a.status)})
        return res
    finally:
        _lib.alae_alignments_free(ctypes.byref(out))


def karlin_altschul(scoring: Scoring | None = None, alphabet="dna", background=None) -> dict:
    """Ungapped Karlin-Altschul lambda, K and relative entropy H of a scoring scheme."""
    sc = scoring if scoring is not None else make_scoring()
    bg = None
    if background is not None:
        arr = np.ascontiguousarray(np.asarray(background, dtype=np.float64))
        bg = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    k = Karlin()
    _check(_lib.alae_karlin_altschul(ctypes.byref(sc), _alpha(alphabet), bg, ctypes.byref(k)), "alae_karlin_altschul")
    return {"lambda": k.lambda_, "K": k.K, "H": k.H}


def evalue_threshold(stats: dict, m: int, n: int, evalue: float) -> int:
    """H = ceil((ln(K m n) - ln E) / lambda) (Section 7), at least 1."""
    k = Karlin(stats["lambda"], stats["K"], stats["H"])
    h = ctypes.c_int32()
    _check(_lib.alae_evalue_threshold(ctypes.byref(k), int(m), int(n), float(evalue), ctypes.byref(h)),
           "alae_evalue_threshold")
    return int(h.value)


class Workspace:
    """Device buffers reused across searches; queries and results stay in device memory."""

    def __init__(self, index: Index):
        self.index = index
        self._h = _vp()
        _check(_lib.alae_workspace_create(index._h, ctypes.byref(self._h)), "alae_workspace_create")

    def search_device(self, d_query, H: int, scoring: Scoring | None = None, stats: Stats | None = None,
                      stream=None, **opt) -> int:
        """d_query: a torch uint8 tensor of codes on the GPU.  Returns the hit count."""
        sc = scoring if scoring is not None else make_scoring()
        opts = make_opts(stats=stats, **opt)
        cnt = ctypes.c_size_t()
        sptr = _vp(stream.cuda_stream) if stream is not None else None
        _check(_lib.alae_search_device(self._h, _vp(d_query.data_ptr()), int(d_query.numel()), ctypes.byref(sc),
                                       int(H), ctypes.byref(opts), sptr, ctypes.byref(cnt)), "alae_search_device")
        return int(cnt.value)

    def autotune(self, d_query, H: int, scoring: Scoring | None = None, reps: int = 2, stream=None, **opt):
        """Pick the launch shapes for this query (alae_autotune).  Returns (shapes, report): shapes is a
        dict of the four chosen options, to pass to search_device; report has the timings."""
        sc = scoring if scoring is not None else make_scoring()
        opts = make_opts(**opt)
        rep = TuneReport()
        sptr = _vp(stream.cuda_stream) if stream is not None else None
        _check(_lib.alae_autotune(self._h, _vp(d_query.data_ptr()), int(d_query.numel()), ctypes.byref(sc), int(H),
                                  ctypes.byref(opts), int(reps), sptr, ctypes.byref(rep)), "alae_autotune")
        shapes = {"level_stage": opts.level_stage, "wide_blocks_per_cu": opts.wide_blocks_per_cu,
                  "lane_waves_per_cu": opts.lane_waves_per_cu, "level_graph": opts.level_graph}
        trials = [{"level_stage": r.level_stage, "wide_blocks_per_cu": r.wide_blocks_per_cu,
                   "lane_waves_per_cu": r.lane_waves_per_cu, "level_graph": r.level_graph, "ms": r.ms}
                  for r in rep.trial[:rep.trials]]
        return shapes, {"default_ms": rep.default_ms, "best_ms": rep.best_ms, "trials": trials}

    def search_device_batch(self, d_queries, lens, H: int, scoring: Scoring | None = None,
                            stats: Stats | None = None, stream=None, **opt) -> int:
        """d_queries: the queries' codes end to end (torch uint8 on the GPU); lens: their lengths.
        Returns the total hit count; batch_offsets() splits the result by query."""
        sc = scoring if scoring is not None else make_scoring()
        opts = make_opts(stats=stats, **opt)
        k = len(lens)
        arr = (ctypes.c_size_t * k)(*[int(x) for x in lens])
        cnt = ctypes.c_size_t()
        sptr = _vp(stream.cuda_stream) if stream is not None else None
        _check(_lib.alae_search_device_batch(self._h, _vp(d_queries.data_ptr()), arr, k, ctypes.byref(sc), int(H),
                                             ctypes.byref(opts), sptr, ctypes.byref(cnt)), "alae_search_device_batch")
        self._k = k
        return int(cnt.value)

    def batch_offsets(self) -> np.ndarray:
        """Offsets (k+1) of each query's records in the last batch result."""
        k = self._k
        arr = (ctypes.c_size_t * (k + 1))()
        _check(_lib.alae_workspace_batch_offsets(self._h, arr, k), "alae_workspace_batch_offsets")
        return np.array(arr[:], dtype=np.int64)

    def result_torch(self, stream=None):
        """Copies of the sorted result as torch tensors on the device: (keys int64, scores int32)."""
        import torch

        k, s, n = _vp(), _vp(), ctypes.c_size_t()
        _check(_lib.alae_workspace_result(self._h, ctypes.byref(k), ctypes.byref(s), ctypes.byref(n)),
               "alae_workspace_result")
        cnt = int(n.value)
        keys = torch.empty(cnt, dtype=torch.int64, device="cuda")
        scores = torch.empty(cnt, dtype=torch.int32, device="cuda")
        if cnt:
            sptr = _vp(stream.cuda_stream) if stream is not None else None
            _check(_lib.alae_workspace_copy_result(self._h, _vp(keys.data_ptr()), _vp(scores.data_ptr()), sptr),
                   "alae_workspace_copy_result")
        return keys, scores

    def copy_result(self, keys, scores, stream=None) -> int:
        """Copy the sorted result into caller tensors (device, or pinned host memory) of at least the
        result's size: keys int64 ((query_end << 32) | text_end), scores int32.  Asynchronous on
        `stream`; returns the record count."""
        k, s, n = _vp(), _vp(), ctypes.c_size_t()
        _check(_lib.alae_workspace_result(self._h, ctypes.byref(k), ctypes.byref(s), ctypes.byref(n)),
               "alae_workspace_result")
        cnt = int(n.value)
        if keys.numel() < cnt or scores.numel() < cnt:
            raise ValueError(f"result of {cnt} records does not fit the buffers")
        if cnt:
            sptr = _vp(stream.cuda_stream) if stream is not None else None
            _check(_lib.alae_workspace_copy_result(self._h, _vp(keys.data_ptr()), _vp(scores.data_ptr()), sptr),
                   "alae_workspace_copy_result")
        return cnt

    def free(self):
        if self._h:
            _lib.alae_workspace_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Trace:
    """Per-chain-item (features, measured work) of one search, for training the work predictor."""

    def __init__(self, capacity: int = 1 << 20):
        self.features = np.zeros((capacity, MLP_FEATURES), dtype=np.float32)
        self.work = np.zeros(capacity, dtype=np.float32)
        self._s = TraceStruct()
        self._s.features = self.features.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._s.work = self.work.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._s.capacity = capacity

    @property
    def count(self) -> int:
        return int(self._s.count)

    @property
    def total(self) -> int:
        return int(self._s.total)

    def arrays(self):
        n = self.count
        return self.features[:n].copy(), self.work[:n].copy()


class MLP:
    """The work predictor: forward, backward and Adam run in the library's HIP kernels."""

    def __init__(self, seed: int = 0, device: int = 0):
        self._h = _vp()
        _check(_lib.alae_mlp_create(int(device), int(seed), ctypes.byref(self._h)), "alae_mlp_create")

    def get_params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_lib.alae_mlp_get_params(self._h, p.ctypes.data_as(_fp)), "alae_mlp_get_params")
        return p

    def set_params(self, p):
        arr, ptr = _f32(p)
        assert arr.shape == (MLP_PARAMS,)
        _check(_lib.alae_mlp_set_params(self._h, ptr), "alae_mlp_set_params")

    def predict(self, x) -> np.ndarray:
        arr, ptr = _f32(x)
        n = arr.shape[0]
        y = np.zeros(n, dtype=np.float32)
        _check(_lib.alae_mlp_predict(self._h, ptr, n, y.ctypes.data_as(_fp)), "alae_mlp_predict")
        return y

    def loss_grad(self, x, t):
        xa, xp = _f32(x)
        ta, tp = _f32(t)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_lib.alae_mlp_loss_grad(self._h, xp, tp, xa.shape[0], ctypes.byref(loss), g.ctypes.data_as(_fp)),
               "alae_mlp_loss_grad")
        return float(loss.value), g

    def train(self, x, t, epochs=20, batch=1024, lr=1e-3, seed=0) -> float:
        xa, xp = _f32(x)
        ta, tp = _f32(t)
        loss = ctypes.c_double()
        _check(_lib.alae_mlp_train(self._h, xp, tp, xa.shape[0], int(epochs), int(batch), float(lr), int(seed),
                                   ctypes.byref(loss)), "alae_mlp_train")
        return float(loss.value)

    def free(self):
        if self._h:
            _lib.alae_mlp_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over a resident index."""

    def __init__(self, index: Index, memory_budget: int = 0, slots: int = 0, max_batch: int = 0):
        self.index = index
        o = ServerOpts()
        o.memory_budget, o.max_inflight, o.max_batch = int(memory_budget), int(slots), int(max_batch)
        self._h = _vp()
        _check(_lib.alae_server_create(index._h, ctypes.byref(o), ctypes.byref(self._h)), "alae_server_create")
        self._scorings = {}

    def submit(self, query, H: int, scoring: Scoring | None = None) -> int:
        sc = scoring if scoring is not None else make_scoring()
        q = _query_bytes(query, self.index.alphabet)
        rid = ctypes.c_uint64()
        _check(_lib.alae_server_submit(self._h, q, len(q), ctypes.byref(sc), int(H), ctypes.byref(rid)),
               "alae_server_submit")
        return int(rid.value)

    def poll(self, rid: int, wait: bool = True):
        """The result as (query_end, text_end, score), or None while pending (wait=False)."""
        h = Hits()
        _check(_lib.alae_server_poll(self._h, int(rid), 1 if wait else 0, ctypes.byref(h)), "alae_server_poll")
        if h.count == ctypes.c_size_t(-1).value:
            return None
        try:
            return _hits_to_numpy(h)
        finally:
            _lib.alae_hits_free(ctypes.byref(h))

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.alae_server_get_stats(self._h, ctypes.byref(s)), "alae_server_get_stats")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def reset_stats(self):
        _lib.alae_server_reset_stats(self._h)

    def close(self):
        if self._h:
            _lib.alae_server_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
