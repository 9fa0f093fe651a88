"""ctypes binding of libllama_mi355x.so (declared in include/llama_mi355x.h).

Argument marshalling only: every step of the copy runs in the library's HIP
kernels.  Blobs are passed as device pointers plus sizes; torch tensors (any
dtype, contiguous, on the GPU) are accepted and only their data pointer and
byte size are used.  Streams are torch.cuda.Stream objects or raw hipStream_t
integers (the current torch stream by default).

There is no fallback: if the shared library has not been built, the first
call raises an error.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libllama_mi355x.so")

MAX_RANK = 8

AOS_PACKED, AOS_ALIGNED, SOA_SINGLE, SOA_MULTI, AOSOA, SPLIT, ONE, SOA_ALIGNED = 0, 1, 2, 3, 4, 5, 6, 7
KINDS = {"aos_packed": AOS_PACKED, "aos_aligned": AOS_ALIGNED, "soa_single": SOA_SINGLE,
         "soa_multi": SOA_MULTI, "aosoa": AOSOA, "split": SPLIT, "one": ONE, "soa_aligned": SOA_ALIGNED}

PATH_AUTO, PATH_STREAM, PATH_TILE, PATH_NAIVE, PATH_EMPTY, PATH_BOX = 0, 1, 2, 3, 4, 5
PATH_NAMES = {PATH_STREAM: "stream", PATH_TILE: "tile", PATH_NAIVE: "naive", PATH_EMPTY: "empty", PATH_BOX: "box"}
TILE_MODE_NAMES = {1: "staged", 2: "direct_store", 3: "direct_load", 4: "gather_store"}

OK = 0
E_INVALID_ARG, E_RECORD_MISMATCH, E_EXTENT_MISMATCH, E_BLOB_TOO_SMALL = -1, -2, -3, -4
E_OVERLAP, E_OVERFLOW, E_UNSUPPORTED, E_HIP, E_NO_BUDGET, E_BUSY = -6, -7, -8, -9, -10, -11

# elemental types of the neutral record form: (size, alignment)
TYPES = {"u8": (1, 1), "i8": (1, 1), "bool": (1, 1), "u16": (2, 2), "i16": (2, 2), "f16": (2, 2),
         "bf16": (2, 2), "u32": (4, 4), "i32": (4, 4), "f32": (4, 4), "u64": (8, 8), "i64": (8, 8),
         "f64": (8, 8)}


class LlamaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


class Field(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("align", ctypes.c_uint32), ("count", ctypes.c_uint32),
                ("children", ctypes.c_uint32)]


class RecordDesc(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_uint32), ("nodes", ctypes.POINTER(Field))]


class SplitDesc(ctypes.Structure):
    pass


SplitDesc._fields_ = [("first_leaf", ctypes.c_uint32), ("leaf_count", ctypes.c_uint32),
                      ("kind", ctypes.c_uint32 * 2), ("lanes", ctypes.c_uint32 * 2),
                      ("split", ctypes.POINTER(SplitDesc) * 2)]


def _split_desc(spec, keep):
    """A SplitDesc for (first, count, part, part); a part is (kind, lanes) or
    ("split", spec) for a nested split.  Every descriptor made goes to `keep`."""
    first, count, p0, p1 = spec
    sd = SplitDesc()
    sd.first_leaf, sd.leaf_count = int(first), int(count)
    for k, (kind, arg) in enumerate((p0, p1)):
        sd.kind[k] = KINDS[kind] if isinstance(kind, str) else int(kind)
        if sd.kind[k] == SPLIT:
            sd.split[k] = ctypes.pointer(_split_desc(arg, keep))
        else:
            sd.lanes[k] = int(arg)
    keep.append(sd)
    return sd


LINEARIZERS = {"row": 0, "col": 1, "morton": 2}


class MappingDesc(ctypes.Structure):
    _fields_ = [("record", ctypes.POINTER(RecordDesc)), ("kind", ctypes.c_uint32), ("rank", ctypes.c_uint32),
                ("extents", ctypes.c_uint64 * MAX_RANK), ("lanes", ctypes.c_uint32),
                ("linearizer", ctypes.c_uint32), ("split", ctypes.POINTER(SplitDesc))]


class Blob(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("size", ctypes.c_uint64)]


class CopyOptions(ctypes.Structure):
    _fields_ = [("path", ctypes.c_uint32), ("tile_records", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_uint32), ("tile_records", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("workgroups", ctypes.c_uint64), ("runs", ctypes.c_uint32),
                ("wg_per_cu", ctypes.c_uint32), ("tiles", ctypes.c_uint64), ("read_bytes", ctypes.c_uint64),
                ("write_bytes", ctypes.c_uint64), ("tile_mode", ctypes.c_uint32), ("cache_hints", ctypes.c_uint32),
                ("plan_flags", ctypes.c_uint32), ("source_chunks", ctypes.c_uint32)]


class CopyItem(ctypes.Structure):
    _fields_ = [("src", ctypes.POINTER(MappingDesc)), ("src_blobs", ctypes.POINTER(Blob)),
                ("dst", ctypes.POINTER(MappingDesc)), ("dst_blobs", ctypes.POINTER(Blob))]


class BatchInfo(ctypes.Structure):
    _fields_ = [("items", ctypes.c_uint64), ("tile_items", ctypes.c_uint64), ("stream_items", ctypes.c_uint64),
                ("work_units", ctypes.c_uint64), ("read_bytes", ctypes.c_uint64), ("write_bytes", ctypes.c_uint64),
                ("threads", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32), ("workgroups", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("launches", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class HeatmapDesc(ctypes.Structure):
    _fields_ = [("src_reads", ctypes.POINTER(ctypes.c_void_p)), ("dst_writes", ctypes.POINTER(ctypes.c_void_p)),
                ("dst_reads", ctypes.POINTER(ctypes.c_void_p))]


_lib = None

# name -> (restype, argtypes) of every entry point the binding uses
_SIGNATURES = {
    "llama_last_error": (ctypes.c_char_p, []),
    "llama_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "llama_record_info": (ctypes.c_int, [ctypes.POINTER(RecordDesc), ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "llama_record_leaf": (ctypes.c_int, [ctypes.POINTER(RecordDesc), ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "llama_mapping_blob_count": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(ctypes.c_uint32)]),
    "llama_mapping_blob_size": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_uint64)]),
    "llama_mapping_offset": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(ctypes.c_uint64),
                                            ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "llama_plan": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(MappingDesc),
                                  ctypes.POINTER(CopyOptions), ctypes.POINTER(PlanInfo)]),
    "llama_plan_copy": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(MappingDesc),
                                       ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(CopyOptions),
                                       ctypes.POINTER(PlanInfo), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "llama_copy": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(MappingDesc),
                                  ctypes.POINTER(Blob), ctypes.c_void_p]),
    "llama_copy_naive": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob),
                                        ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.c_void_p]),
    "llama_copy_ex": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(MappingDesc),
                                     ctypes.POINTER(Blob), ctypes.POINTER(CopyOptions), ctypes.c_void_p]),
    "llama_copy_leaves": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(MappingDesc),
                                         ctypes.POINTER(Blob), ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(CopyOptions), ctypes.c_void_p]),
    "llama_autotune": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(MappingDesc),
                                      ctypes.POINTER(Blob), ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.POINTER(CopyOptions), ctypes.POINTER(ctypes.c_double)]),
    "llama_tune_lookup": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(MappingDesc),
                                         ctypes.POINTER(CopyOptions), ctypes.POINTER(ctypes.c_int)]),
    "llama_tune_clear": (ctypes.c_int, []),
    "llama_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "llama_tune_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32)]),
    "llama_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "llama_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CopyItem), ctypes.POINTER(ctypes.c_uint64)]),
    "llama_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "llama_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]),
    "llama_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "llama_server_reset_stats": (ctypes.c_int, [ctypes.c_void_p]),
    "llama_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "llama_server_create_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "llama_batch_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(CopyItem), ctypes.POINTER(CopyOptions),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "llama_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "llama_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                            ctypes.POINTER(ctypes.c_double)]),
    "llama_batch_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchInfo)]),
    "llama_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "llama_copy_batch": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(CopyItem), ctypes.c_void_p]),
    "llama_copy_batch_noalloc": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(CopyItem), ctypes.c_void_p]),
    "llama_copy_transfer": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.c_uint32,
                                           ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_void_p]),
    "llama_copy_box": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(CopyOptions), ctypes.c_void_p]),
    "llama_copy_heatmap": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob),
                                          ctypes.POINTER(MappingDesc), ctypes.POINTER(Blob),
                                          ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(CopyOptions),
                                          ctypes.POINTER(HeatmapDesc), ctypes.c_void_p]),
    "llama_heatmap_begin": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "llama_heatmap_end": (ctypes.c_int, []),
    "llama_trace_leaves": (ctypes.c_int, [ctypes.POINTER(MappingDesc), ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_04284_amd.build` "
                               "(the copy has no other implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().llama_status_string(status).decode()


def check(status: int) -> None:
    if status != OK:
        raise LlamaError(status, lib().llama_last_error().decode())


# --------------------------------------------------------------------------
# records and mappings
# --------------------------------------------------------------------------

class Record:
    """A record dimension in the library's pre-order node form, built from the
    neutral nested form (see paper_2106_04284_amd.workloads)."""

    def __init__(self, record):
        nodes = []

        def emit(m, count=1):
            if isinstance(m, tuple):  # static array: a nested count multiplies
                inner, c = m
                emit(inner, count * int(c))
                return
            if isinstance(m, list):
                nodes.append((0, 0, count, len(m)))
                for x in m:
                    emit(x)
                return
            size, align = TYPES[m]
            nodes.append((size, align, count, 0))

        for member in record:
            emit(member)
        self.nodes = (Field * len(nodes))(*[Field(*n) for n in nodes])
        self.desc = RecordDesc(len(nodes), ctypes.cast(self.nodes, ctypes.POINTER(Field)))
        self.source = record

    def info(self):
        n, s, r = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().llama_record_info(ctypes.byref(self.desc), ctypes.byref(n), ctypes.byref(s), ctypes.byref(r)))
        return int(n.value), int(s.value), int(r.value)

    @property
    def leaf_count(self):
        return self.info()[0]

    @property
    def packed_size(self):
        return self.info()[1]

    @property
    def aligned_size(self):
        return self.info()[2]

    def leaf(self, f: int):
        size, align = ctypes.c_uint32(), ctypes.c_uint32()
        po, ao = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().llama_record_leaf(ctypes.byref(self.desc), f, ctypes.byref(size), ctypes.byref(align),
                                      ctypes.byref(po), ctypes.byref(ao)))
        return {"size": size.value, "align": align.value, "packed_offset": po.value, "aligned_offset": ao.value}


class Mapping:
    """A mapping of `record` over `extents`.  kind "split" takes
    split=(first_leaf, leaf_count, part, part): the selected leaf range through
    the first part's mapping, the other leaves through the second's (sec. 3.7
    Split); a part is (kind, lanes), or ("split", (first, count, part, part))
    to split that part's leaves again."""

    def __init__(self, record: Record, kind: str, extents, lanes: int = 0, split=None, linearizer="row"):
        ext = [int(e) for e in (extents if isinstance(extents, (list, tuple)) else [extents])]
        self.record = record
        self.kind = kind
        self.extents = ext
        self.lanes = int(lanes)
        self.split = split
        self.linearizer = linearizer
        self._split = None
        self.desc = MappingDesc()
        self.desc.record = ctypes.pointer(record.desc)
        self.desc.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        self.desc.rank = len(ext)
        for d, e in enumerate(ext[:MAX_RANK]):
            self.desc.extents[d] = e
        self.desc.lanes = self.lanes
        self.desc.linearizer = LINEARIZERS[linearizer] if isinstance(linearizer, str) else int(linearizer)
        if split is not None:
            self._split = []  # the descriptors, kept alive with the one that points at them
            self.desc.split = ctypes.pointer(_split_desc(split, self._split))

    @property
    def blob_count(self) -> int:
        n = ctypes.c_uint32()
        check(lib().llama_mapping_blob_count(ctypes.byref(self.desc), ctypes.byref(n)))
        return int(n.value)

    def blob_size(self, b: int) -> int:
        s = ctypes.c_uint64()
        check(lib().llama_mapping_blob_size(ctypes.byref(self.desc), b, ctypes.byref(s)))
        return int(s.value)

    def blob_sizes(self):
        return [self.blob_size(b) for b in range(self.blob_count)]

    def offset(self, coord, leaf: int):
        c = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in coord])
        b, o = ctypes.c_uint32(), ctypes.c_uint64()
        check(lib().llama_mapping_offset(ctypes.byref(self.desc), c, leaf, ctypes.byref(b), ctypes.byref(o)))
        return int(b.value), int(o.value)

    def alloc(self, device="cuda", fill=None):
        """Allocates the mapping's blobs as uint8 torch tensors (allocation is
        the caller's business; this is a convenience)."""
        import torch
        out = []
        for s in self.blob_sizes():
            t = torch.empty(s, dtype=torch.uint8, device=device)
            if fill is not None:
                t.fill_(fill)
            out.append(t)
        return out


def _blobs(blobs):
    arr = (Blob * max(len(blobs), 1))()
    for k, b in enumerate(blobs):
        if isinstance(b, tuple):
            ptr, size = b
        else:  # a torch tensor
            if not b.is_contiguous():
                raise ValueError("blob tensors must be contiguous")
            ptr, size = b.data_ptr(), b.numel() * b.element_size()
        arr[k] = Blob(ptr, size)
    return arr


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


COPY_NO_DIRECT = 1
COPY_NO_SPLIT = 2
COPY_PRESERVE_PADDING = 4
COPY_NO_GATHER = 8


def _options(path=PATH_AUTO, tile_records=0, threads=0, wg_per_cu=0, flags=0):
    if isinstance(path, str):
        path = {"auto": PATH_AUTO, "stream": PATH_STREAM, "tile": PATH_TILE, "naive": PATH_NAIVE, "box": PATH_BOX}[path]
    return CopyOptions(path, tile_records, threads, wg_per_cu, flags)


def copy(src: Mapping, src_blobs, dst: Mapping, dst_blobs, stream=None, path=PATH_AUTO, tile_records=0,
         threads=0, wg_per_cu=0, flags=0):
    """llama_copy / llama_copy_ex: enqueues the copy on `stream`."""
    sb, db = _blobs(src_blobs), _blobs(dst_blobs)
    if path == PATH_AUTO and not tile_records and not threads and not wg_per_cu and not flags:
        check(lib().llama_copy(ctypes.byref(src.desc), sb, ctypes.byref(dst.desc), db, _stream(stream)))
    else:
        o = _options(path, tile_records, threads, wg_per_cu, flags)
        check(lib().llama_copy_ex(ctypes.byref(src.desc), sb, ctypes.byref(dst.desc), db, ctypes.byref(o),
                                  _stream(stream)))


NO_LEAF = 0xFFFFFFFF


MEMORY_DEVICE, MEMORY_HOST = 0, 1


def copy_transfer(src: Mapping, src_blobs, dst: Mapping, dst_blobs, src_on_host: bool, chunk_bytes=0, stream=None):
    """llama_copy_transfer: a copy between host and device memory that
    changes the layout on the way, chunk by chunk.  src_on_host: the source
    blobs are host tensors (the destination's on the device), else the
    reverse."""
    sm, dm = (MEMORY_HOST, MEMORY_DEVICE) if src_on_host else (MEMORY_DEVICE, MEMORY_HOST)
    check(lib().llama_copy_transfer(ctypes.byref(src.desc), _blobs(src_blobs), sm, ctypes.byref(dst.desc),
                                    _blobs(dst_blobs), dm, int(chunk_bytes), _stream(stream)))


def copy_box(src: Mapping, src_blobs, src_offset, dst: Mapping, dst_blobs, dst_offset, box, stream=None,
             path=PATH_AUTO, tile_records=0, threads=0, flags=0):
    """llama_copy_box: the records of a box of the array dimensions, from
    src_offset + c in the source to dst_offset + c in the destination."""
    r = len(box)
    so = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in src_offset])
    do = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in dst_offset])
    bx = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in box])
    if len(src_offset) != r or len(dst_offset) != r:
        raise ValueError("offsets and box need one entry per dimension")
    o = _options(path, tile_records, threads, 0, flags)
    check(lib().llama_copy_box(ctypes.byref(src.desc), _blobs(src_blobs), so, ctypes.byref(dst.desc),
                               _blobs(dst_blobs), do, bx, ctypes.byref(o), _stream(stream)))


def copy_leaves(src: Mapping, src_blobs, dst: Mapping, dst_blobs, source_leaf, stream=None, path=PATH_AUTO,
                tile_records=0, threads=0, wg_per_cu=0, flags=0):
    """llama_copy_leaves: destination leaf k takes source leaf source_leaf[k]
    (None: the leaf keeps its bytes); the records may differ."""
    arr = (ctypes.c_uint32 * max(len(source_leaf), 1))(*[NO_LEAF if x is None else int(x) for x in source_leaf])
    o = _options(path, tile_records, threads, wg_per_cu, flags)
    check(lib().llama_copy_leaves(ctypes.byref(src.desc), _blobs(src_blobs), ctypes.byref(dst.desc),
                                  _blobs(dst_blobs), arr, ctypes.byref(o), _stream(stream)))


def _counter_array(tensors):
    if tensors is None:
        return None
    arr = (ctypes.c_void_p * max(len(tensors), 1))()
    for k, t in enumerate(tensors):
        arr[k] = None if t is None else t.data_ptr()
    return arr


def copy_heatmap(src: Mapping, src_blobs, dst: Mapping, dst_blobs, source_leaf=None, stream=None,
                 src_reads=None, dst_writes=None, dst_reads=None, path=PATH_AUTO, tile_records=0, threads=0,
                 wg_per_cu=0, flags=0):
    """llama_copy_heatmap: the copy (llama_copy_ex, or llama_copy_leaves with
    source_leaf) in its counted kernel variants.  src_reads / dst_writes /
    dst_reads are lists of int32 device tensors, one per blob (blob size
    elements each), that the copy adds its per-byte access counts to."""
    arr = None
    if source_leaf is not None:
        arr = (ctypes.c_uint32 * max(len(source_leaf), 1))(*[NO_LEAF if x is None else int(x) for x in source_leaf])
    o = _options(path, tile_records, threads, wg_per_cu, flags)
    keep = [_counter_array(x) for x in (src_reads, dst_writes, dst_reads)]
    h = HeatmapDesc(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p)) if a is not None else None for a in keep])
    check(lib().llama_copy_heatmap(ctypes.byref(src.desc), _blobs(src_blobs), ctypes.byref(dst.desc),
                                   _blobs(dst_blobs), arr, ctypes.byref(o), ctypes.byref(h), _stream(stream)))


class CountRange(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("size", ctypes.c_uint64), ("counters", ctypes.c_void_p)]


class heatmap:
    """Context manager around llama_heatmap_begin / llama_heatmap_end: the
    copies made inside it on this thread run in their counted variants.
    reads / writes: lists of (blob tensor, int32 counter tensor) pairs."""

    def __init__(self, reads=(), writes=(), stream=None):
        def arr(pairs):
            a = (CountRange * max(len(pairs), 1))()
            for k, (blob, cnt) in enumerate(pairs):
                a[k] = CountRange(blob.data_ptr(), blob.numel() * blob.element_size(), cnt.data_ptr())
            return a
        self._r, self._w = arr(list(reads)), arr(list(writes))
        self._nr, self._nw = len(reads), len(writes)
        self._stream = stream

    def __enter__(self):
        check(lib().llama_heatmap_begin(self._nr, self._r, self._nw, self._w, _stream(self._stream)))
        return self

    def __exit__(self, *exc):
        check(lib().llama_heatmap_end())
        return False


def trace_leaves(m: Mapping, counters, stream=None):
    """llama_trace_leaves: per-leaf sums of a view's per-byte counters, then
    the sum over the bytes no leaf owns (a list of F + 1 integers)."""
    f = m.record.leaf_count
    out = (ctypes.c_uint64 * (f + 1))()
    arr = _counter_array(counters)
    check(lib().llama_trace_leaves(ctypes.byref(m.desc), ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), out,
                                   _stream(stream)))
    return [int(x) for x in out]


def copy_naive(src: Mapping, src_blobs, dst: Mapping, dst_blobs, stream=None):
    """llama_copy_naive: the element-wise baseline kernel."""
    check(lib().llama_copy_naive(ctypes.byref(src.desc), _blobs(src_blobs), ctypes.byref(dst.desc),
                                 _blobs(dst_blobs), _stream(stream)))


PLAN_GATHERED_SOURCE = 1
PLAN_KEEPS_DESTINATION = 2
PLAN_SCATTERED_DESTINATION = 4


def _info_dict(info: PlanInfo) -> dict:
    return {"path": PATH_NAMES.get(info.path, "?"), "tile_records": info.tile_records, "threads": info.threads,
            "lds_bytes": info.lds_bytes, "workgroups": info.workgroups, "runs": info.runs,
            "wg_per_cu": info.wg_per_cu, "tiles": info.tiles,
            "read_bytes": info.read_bytes, "write_bytes": info.write_bytes,
            "tile_mode": TILE_MODE_NAMES.get(info.tile_mode), "stream_loads": bool(info.cache_hints & 1),
            "stream_stores": bool(info.cache_hints & 2),
            "gathered_source": bool(info.plan_flags & PLAN_GATHERED_SOURCE),
            "keeps_destination": bool(info.plan_flags & PLAN_KEEPS_DESTINATION),
            "scattered_destination": bool(info.plan_flags & PLAN_SCATTERED_DESTINATION),
            "source_chunks": info.source_chunks}


def plan(src: Mapping, dst: Mapping, path=PATH_AUTO, tile_records=0, threads=0, wg_per_cu=0, flags=0) -> dict:
    """llama_plan: what a copy of this pair would launch."""
    info = PlanInfo()
    o = _options(path, tile_records, threads, wg_per_cu, flags)
    check(lib().llama_plan(ctypes.byref(src.desc), ctypes.byref(dst.desc), ctypes.byref(o), ctypes.byref(info)))
    return _info_dict(info)


def plan_copy(src: Mapping, dst: Mapping, src_leaf=None, path=PATH_AUTO, tile_records=0, threads=0, wg_per_cu=0,
              flags=0, capacity=64) -> list:
    """llama_plan_copy: every launch of llama_copy_ex (or, with `src_leaf`,
    llama_copy_leaves) for this pair, in order."""
    infos = (PlanInfo * capacity)()
    count = ctypes.c_uint32()
    o = _options(path, tile_records, threads, wg_per_cu, flags)
    leaf = None
    if src_leaf is not None:
        leaf = (ctypes.c_uint32 * len(src_leaf))(*[NO_LEAF if x is None else int(x) for x in src_leaf])
    check(lib().llama_plan_copy(ctypes.byref(src.desc), ctypes.byref(dst.desc), leaf, ctypes.byref(o), infos,
                                capacity, ctypes.byref(count)))
    return [_info_dict(infos[k]) for k in range(count.value)]


# --------------------------------------------------------------------------
# autotuning
# --------------------------------------------------------------------------

def _opt_dict(o: CopyOptions) -> dict:
    return {"path": PATH_NAMES.get(o.path, "auto"), "tile_records": o.tile_records, "threads": o.threads,
            "wg_per_cu": o.wg_per_cu}


def autotune(src: Mapping, src_blobs, dst: Mapping, dst_blobs, stream=None, reps=3):
    """llama_autotune: returns (best options, best GB/s) and caches them."""
    o, g = CopyOptions(), ctypes.c_double()
    check(lib().llama_autotune(ctypes.byref(src.desc), _blobs(src_blobs), ctypes.byref(dst.desc), _blobs(dst_blobs),
                               _stream(stream), reps, ctypes.byref(o), ctypes.byref(g)))
    return _opt_dict(o), g.value


def tune_lookup(src: Mapping, dst: Mapping):
    o, found = CopyOptions(), ctypes.c_int()
    check(lib().llama_tune_lookup(ctypes.byref(src.desc), ctypes.byref(dst.desc), ctypes.byref(o), ctypes.byref(found)))
    return _opt_dict(o) if found.value else None


def tune_clear():
    check(lib().llama_tune_clear())


def tune_save(path: str):
    check(lib().llama_tune_save(path.encode()))


def tune_load(path: str) -> int:
    n = ctypes.c_uint32()
    check(lib().llama_tune_load(path.encode(), ctypes.byref(n)))
    return n.value


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------

class _Items:
    """A CopyItem array plus every object it points into."""

    def __init__(self, items):
        self.keep = []
        self.arr = (CopyItem * max(len(items), 1))()
        for k, (src, sblobs, dst, dblobs) in enumerate(items):
            sb, db = _blobs(sblobs), _blobs(dblobs)
            self.keep += [src, dst, sb, db, sblobs, dblobs]  # the blob tensors live as long as the items
            self.arr[k] = CopyItem(ctypes.pointer(src.desc), ctypes.cast(sb, ctypes.POINTER(Blob)),
                                   ctypes.pointer(dst.desc), ctypes.cast(db, ctypes.POINTER(Blob)))
        self.n = len(items)


class Batch:
    """llama_batch_*: a prepared batch of copies, launched as one persistent
    kernel (captured into a hipGraph on its first launch on a stream).
    `items` is a list of (src_mapping, src_blobs, dst_mapping, dst_blobs)."""

    def __init__(self, items, tile_records=0, threads=0, wg_per_cu=0, flags=0):
        self._items = _Items(items)
        self._h = ctypes.c_void_p()
        o = _options(PATH_AUTO, tile_records, threads, wg_per_cu, flags)
        check(lib().llama_batch_create(self._items.n, self._items.arr, ctypes.byref(o), ctypes.byref(self._h)))

    def launch(self, stream=None):
        check(lib().llama_batch_launch(self._h, _stream(stream)))

    def autotune(self, stream=None, reps=3) -> float:
        """llama_batch_autotune: re-plans the batch with the fastest measured
        LDS budget, threads and grid; returns its GB/s."""
        g = ctypes.c_double()
        check(lib().llama_batch_autotune(self._h, _stream(stream), int(reps), ctypes.byref(g)))
        return g.value

    def info(self) -> dict:
        i = BatchInfo()
        check(lib().llama_batch_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in BatchInfo._fields_}

    def close(self):
        if self._h:
            check(lib().llama_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_batch(items, stream=None):
    """llama_copy_batch: one-shot batch launched on `stream`."""
    it = _Items(items)
    check(lib().llama_copy_batch(it.n, it.arr, _stream(stream)))


def copy_batch_noalloc(items, stream=None):
    """llama_copy_batch_noalloc: the one-shot batch with its work table in the
    library's static device buffer (no device allocation)."""
    it = _Items(items)
    check(lib().llama_copy_batch_noalloc(it.n, it.arr, _stream(stream)))


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

SERVE_BATCHED, SERVE_NAIVE, SERVE_PER_REQUEST = 0, 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("group_bytes", ctypes.c_uint64),
                ("stream_bytes", ctypes.c_uint64), ("streams", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("queue_capacity", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("policy", ctypes.c_uint32)]


EXEC_START = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.POINTER(CopyItem))
EXEC_POLL = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64)


class Executor(ctypes.Structure):
    _fields_ = [("context", ctypes.c_void_p), ("start", EXEC_START), ("poll", EXEC_POLL)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("bytes_done", ctypes.c_uint64),
                ("max_inflight_bytes", ctypes.c_uint64), ("mean_batch", ctypes.c_double),
                ("p50_latency", ctypes.c_double), ("p99_latency", ctypes.c_double), ("max_latency", ctypes.c_double),
                ("window", ctypes.c_double)]


class Server:
    """llama_server_*: requests admitted within an HBM budget and run with
    continuous batching.  submit() keeps the request's mappings and blobs
    alive until its ticket has been waited for or polled done."""

    def __init__(self, budget_bytes, streams=0, max_batch=0, queue_capacity=0, threads=0, policy=SERVE_BATCHED,
                 group_bytes=0, depth=0, stream_bytes=0, executor=None):
        """`executor` (llama_server_create_ex): an object with start(launch,
        items) and poll(launch) methods returning the C statuses; `items` is a
        list of CopyItem structures.  It runs on the server's engine thread
        and must not call the server."""
        cfg = ServerConfig(int(budget_bytes), int(group_bytes), int(stream_bytes), streams, depth, max_batch,
                           queue_capacity, threads, policy)
        self._h = ctypes.c_void_p()
        self._keep = {}
        self._exec = None
        if executor is None:
            check(lib().llama_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
            return

        def start(_ctx, launch, n, items):
            try:
                return int(executor.start(int(launch), [items[k] for k in range(n)]))
            except Exception:  # an exception cannot cross the C boundary: fail the launch
                import traceback
                traceback.print_exc()
                return E_INVALID_ARG

        def poll(_ctx, launch):
            try:
                return int(executor.poll(int(launch)))
            except Exception:
                import traceback
                traceback.print_exc()
                return E_INVALID_ARG

        self._exec = Executor(None, EXEC_START(start), EXEC_POLL(poll))  # kept alive with the server
        check(lib().llama_server_create_ex(ctypes.byref(cfg), ctypes.byref(self._exec), ctypes.byref(self._h)))

    def submit(self, src: Mapping, src_blobs, dst: Mapping, dst_blobs) -> int:
        return self.submit_prepared(Server.prepare(src, src_blobs, dst, dst_blobs))

    @staticmethod
    def prepare(src: Mapping, src_blobs, dst: Mapping, dst_blobs):
        """The request's C structures, built once: submit_prepared then only
        calls llama_server_submit (a client that replays many requests keeps
        their marshalling out of its timing)."""
        return _Items([(src, src_blobs, dst, dst_blobs)])

    def submit_prepared(self, prepared) -> int:
        t = ctypes.c_uint64()
        check(lib().llama_server_submit(self._h, prepared.arr, ctypes.byref(t)))
        self._keep[t.value] = prepared
        return t.value

    def poll(self, ticket):
        done, st, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib().llama_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(lat)))
        if done.value:
            self._keep.pop(ticket, None)
            return st.value, lat.value
        return None

    def wait(self, ticket):
        st, lat = ctypes.c_int(), ctypes.c_double()
        check(lib().llama_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(lat)))
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().llama_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def reset_stats(self):
        check(lib().llama_server_reset_stats(self._h))

    def close(self):
        if self._h:
            check(lib().llama_server_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
