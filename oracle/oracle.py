"""Python access to the CPU oracle of the layout-aware copy.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the library itself never imports it.

The arithmetic lives in ``llama_oracle.c`` (plain C, its own record parser and
mapping formulas, written from the LLAMA paper's sec. 3.3 "Describing a data
structure", sec. 3.7 "Mappings", sec. 3.9 "Copying between views" and the naive
copy of sec. 4.2).  This module only marshals numpy buffers and compiles the C
file when its shared object is missing.

Records are given in the neutral nested form used by the workload definitions:
a record is a list of members; a member is an elemental type name, a nested
list (a nested record), or a ``(member, count)`` pair for a static array.
Mappings are ``(kind, extents, lanes)`` with kind one of ``aos_packed``,
``aos_aligned``, ``soa_single``, ``soa_multi``, ``soa_aligned`` (single-blob
SoA whose sub-arrays start at multiples of ``lanes`` bytes, 0 meaning 256),
``aosoa``, ``one`` (every coordinate at the same single packed record), or
``split`` with
``split=(first, count, (kind, lanes), (kind, lanes))``: leaves
``[first, first + count)`` mapped by the first plain mapping, the others by the
second (sec. 3.7 Split).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "llama_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

MAX_RANK = 8
MAX_LEAVES = 4096

LINEARIZERS = {"row": 0, "col": 1, "morton": 2}
KINDS = {"aos_packed": 0, "aos_aligned": 1, "soa_single": 2, "soa_multi": 3, "aosoa": 4, "split": 5, "one": 6,
         "soa_aligned": 7}


class _Record(ctypes.Structure):
    _fields_ = [("nleaves", ctypes.c_int32),
                ("size", ctypes.POINTER(ctypes.c_uint64)),
                ("align", ctypes.POINTER(ctypes.c_uint64))]


class _Mapping(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("extents", ctypes.c_uint64 * MAX_RANK), ("lanes", ctypes.c_uint64),
                ("first", ctypes.c_int32), ("count", ctypes.c_int32),
                ("part_kind", ctypes.c_int32 * 2), ("part_lanes", ctypes.c_uint64 * 2),
                ("part_split", ctypes.c_void_p * 2), ("linearizer", ctypes.c_int32)]


def build(force: bool = False) -> str:
    """Compiles llama_oracle.c into liborc.so with gcc -O2 -fopenmp (OpenMP
    serves only the threaded copy used to time the oracle on all cores).

    LLAMA_ORACLE_LIB names another build of the oracle to load instead; the
    test suite uses it to run the pins against deliberately broken copies of
    the oracle, which must fail them."""
    override = os.environ.get("LLAMA_ORACLE_LIB")
    if override and not force:
        return override
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u64, i32, i64 = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
        RP, MP = ctypes.POINTER(_Record), ctypes.POINTER(_Mapping)
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.orc_parse_record.argtypes = [ctypes.c_char_p, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.c_int]
        L.orc_parse_record.restype = ctypes.c_int
        for name in ("orc_packed_offset", "orc_aligned_offset"):
            getattr(L, name).argtypes = [RP, ctypes.c_int]
            getattr(L, name).restype = u64
        for name in ("orc_packed_size", "orc_aligned_size"):
            getattr(L, name).argtypes = [RP]
            getattr(L, name).restype = u64
        L.orc_record_count.argtypes = [MP]
        L.orc_record_count.restype = u64
        L.orc_linearize.argtypes = [MP, ctypes.POINTER(u64)]
        L.orc_linearize.restype = u64
        L.orc_blob_count.argtypes = [MP, RP]
        L.orc_blob_count.restype = ctypes.c_int
        L.orc_blob_size.argtypes = [MP, RP, ctypes.c_int]
        L.orc_blob_size.restype = u64
        L.orc_blob_nr_and_offset.argtypes = [MP, RP, ctypes.POINTER(u64), ctypes.c_int,
                                             ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.orc_blob_nr_and_offset.restype = ctypes.c_int
        L.orc_copy.argtypes = [RP, MP, PP, MP, PP]
        L.orc_copy.restype = ctypes.c_int
        L.orc_copy_keep.argtypes = [RP, MP, PP, MP, PP]
        L.orc_copy_keep.restype = ctypes.c_int
        L.orc_linear_size.argtypes = [MP]
        L.orc_linear_size.restype = u64
        L.orc_copy_box.argtypes = [RP, MP, PP, ctypes.POINTER(u64), MP, PP, ctypes.POINTER(u64),
                                   ctypes.POINTER(u64), ctypes.c_int]
        L.orc_copy_box.restype = ctypes.c_int
        L.orc_copy_threads.argtypes = [RP, MP, PP, MP, PP, ctypes.c_int, ctypes.c_int]
        L.orc_copy_threads.restype = ctypes.c_int
        L.orc_memcpy_threads.argtypes = [ctypes.c_void_p, ctypes.c_void_p, u64, ctypes.c_int]
        L.orc_memcpy_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_write_counts.argtypes = [RP, MP, PP]
        L.orc_write_counts.restype = ctypes.c_int
        L.orc_copy_writes.argtypes = [RP, MP, ctypes.POINTER(i32), ctypes.c_int, PP]
        L.orc_copy_writes.restype = ctypes.c_int
        L.orc_check_samples.argtypes = [RP, MP, PP, MP, PP, ctypes.POINTER(u64), ctypes.POINTER(i32),
                                        i64, ctypes.POINTER(i64)]
        L.orc_check_samples.restype = i64
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# records
# --------------------------------------------------------------------------

def record_spec(record) -> str:
    """Renders the neutral nested record form as the oracle's spec string."""
    def member(m):
        if isinstance(m, tuple):
            inner, count = m
            return f"{member(inner)}[{int(count)}]"
        if isinstance(m, list):
            return "{" + ",".join(member(x) for x in m) + "}"
        return str(m)
    return member(list(record))


class Record:
    """A flattened record as the oracle sees it."""

    def __init__(self, record):
        spec = record if isinstance(record, str) else record_spec(record)
        size = (ctypes.c_uint64 * MAX_LEAVES)()
        align = (ctypes.c_uint64 * MAX_LEAVES)()
        n = lib().orc_parse_record(spec.encode(), size, align, MAX_LEAVES)
        if n < 0:
            raise ValueError(f"oracle cannot parse record {spec!r} (code {n})")
        self.spec = spec
        self.sizes = [int(size[k]) for k in range(n)]
        self.aligns = [int(align[k]) for k in range(n)]
        self._size = (ctypes.c_uint64 * max(n, 1))(*self.sizes)
        self._align = (ctypes.c_uint64 * max(n, 1))(*self.aligns)
        self.c = _Record(n, self._size, self._align)

    @property
    def nleaves(self) -> int:
        return len(self.sizes)

    def packed_offset(self, f: int) -> int:
        return int(lib().orc_packed_offset(ctypes.byref(self.c), f))

    def aligned_offset(self, f: int) -> int:
        return int(lib().orc_aligned_offset(ctypes.byref(self.c), f))

    @property
    def packed_size(self) -> int:
        return int(lib().orc_packed_size(ctypes.byref(self.c)))

    @property
    def aligned_size(self) -> int:
        return int(lib().orc_aligned_size(ctypes.byref(self.c)))


# --------------------------------------------------------------------------
# mappings
# --------------------------------------------------------------------------

def _mapping(kind: str, extents, lanes: int = 0, split=None, linearizer: str = "row") -> _Mapping:
    ext = [int(e) for e in (extents if isinstance(extents, (list, tuple)) else [extents])]
    if not 1 <= len(ext) <= MAX_RANK:
        raise ValueError("rank must be 1..8")
    m = _Mapping()
    m.kind = KINDS[kind]
    m.rank = len(ext)
    for d, e in enumerate(ext):
        m.extents[d] = e
    m.lanes = int(lanes)
    m.linearizer = LINEARIZERS[linearizer]
    if kind == "split":
        first, count, p0, p1 = split
        m.first, m.count = int(first), int(count)
        m._nested = []  # keeps nested splits alive while m is
        for k, (pk, pa) in enumerate((p0, p1)):
            m.part_kind[k] = KINDS[pk]
            if pk == "split":  # pa is the nested split over the part's leaves
                inner = _mapping("split", ext, 0, pa, linearizer)
                m._nested.append(inner)
                m.part_split[k] = ctypes.addressof(inner)
            else:
                m.part_lanes[k] = int(pa)
    return m


class Mapping:
    def __init__(self, record: Record, kind: str, extents, lanes: int = 0, split=None, linearizer: str = "row"):
        self.record = record
        self.kind = kind
        self.extents = [int(e) for e in (extents if isinstance(extents, (list, tuple)) else [extents])]
        self.lanes = int(lanes)
        self.split = split
        self.linearizer = linearizer
        if kind == "split":
            first, count = int(split[0]), int(split[1])
            if not (first >= 0 and count >= 1 and first + count <= record.nleaves and count < record.nleaves):
                raise ValueError("split: the selected leaves must be a proper, non-empty range")
        self.c = _mapping(kind, self.extents, lanes, split, linearizer)

    @property
    def count(self) -> int:
        return int(lib().orc_record_count(ctypes.byref(self.c)))

    @property
    def linear_size(self) -> int:
        """Linear indices the mapping lays out (Morton order: holes included)."""
        return int(lib().orc_linear_size(ctypes.byref(self.c)))

    @property
    def blob_count(self) -> int:
        return int(lib().orc_blob_count(ctypes.byref(self.c), ctypes.byref(self.record.c)))

    def blob_size(self, b: int) -> int:
        return int(lib().orc_blob_size(ctypes.byref(self.c), ctypes.byref(self.record.c), b))

    def blob_sizes(self):
        return [self.blob_size(b) for b in range(self.blob_count)]

    def linearize(self, coord) -> int:
        c = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in coord])
        return int(lib().orc_linearize(ctypes.byref(self.c), c))

    def blob_nr_and_offset(self, coord, leaf: int):
        c = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in coord])
        b, o = ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().orc_blob_nr_and_offset(ctypes.byref(self.c), ctypes.byref(self.record.c), c, int(leaf),
                                          ctypes.byref(b), ctypes.byref(o))
        if rc != 0:
            raise ValueError(f"blob_nr_and_offset failed ({rc})")
        return int(b.value), int(o.value)

    def alloc(self, fill: int = 0):
        return [np.full(s, fill, dtype=np.uint8) for s in self.blob_sizes()]


def _ptrs(blobs):
    arr = (ctypes.c_void_p * max(len(blobs), 1))()
    for k, b in enumerate(blobs):
        if not (isinstance(b, np.ndarray) and b.dtype == np.uint8 and b.flags.c_contiguous):
            raise TypeError("blobs must be contiguous uint8 numpy arrays")
        arr[k] = b.ctypes.data
    return arr


def copy(src: Mapping, src_blobs, dst: Mapping, dst_blobs=None, keep_padding=False):
    """The naive field-wise copy; returns the destination blobs.  By default
    the destination's padding becomes zero; with keep_padding, `dst_blobs`
    (required) are updated in place and their padding keeps its bytes."""
    if keep_padding and dst_blobs is None:
        raise ValueError("keep_padding needs the destination blobs")
    if dst_blobs is None:
        dst_blobs = dst.alloc()
    for b, s in zip(src_blobs, src.blob_sizes()):
        if b.size < s:
            raise ValueError("source blob too small")
    for b, s in zip(dst_blobs, dst.blob_sizes()):
        if b.size < s:
            raise ValueError("destination blob too small")
    fn = lib().orc_copy_keep if keep_padding else lib().orc_copy
    rc = fn(ctypes.byref(src.record.c), ctypes.byref(src.c), _ptrs(src_blobs), ctypes.byref(dst.c),
            _ptrs(dst_blobs))
    if rc != 0:
        raise ValueError(f"oracle copy failed ({rc})")
    return dst_blobs


def copy_threads(src: Mapping, src_blobs, dst: Mapping, dst_blobs=None, keep_padding=False, threads=0):
    """copy() run on `threads` host threads (0: the OpenMP default), each over
    a contiguous piece of the coordinate order; the same bytes as copy()."""
    if keep_padding and dst_blobs is None:
        raise ValueError("keep_padding needs the destination blobs")
    if dst_blobs is None:
        dst_blobs = [np.empty(s, dtype=np.uint8) for s in dst.blob_sizes()]
    for b, s in zip(src_blobs, src.blob_sizes()):
        if b.size < s:
            raise ValueError("source blob too small")
    for b, s in zip(dst_blobs, dst.blob_sizes()):
        if b.size < s:
            raise ValueError("destination blob too small")
    rc = lib().orc_copy_threads(ctypes.byref(src.record.c), ctypes.byref(src.c), _ptrs(src_blobs),
                                ctypes.byref(dst.c), _ptrs(dst_blobs), 1 if keep_padding else 0, int(threads))
    if rc != 0:
        raise ValueError(f"oracle copy failed ({rc})")
    return dst_blobs


def memcpy_threads(dst: np.ndarray, src: np.ndarray, threads=0) -> int:
    """Host memcpy of src into dst on `threads` threads (0: the OpenMP
    default); returns the threads used."""
    if dst.nbytes < src.nbytes:
        raise ValueError("destination too small")
    return int(lib().orc_memcpy_threads(dst.ctypes.data, src.ctypes.data, src.nbytes, int(threads)))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def copy_box(src: Mapping, src_blobs, src_offset, dst: Mapping, dst_blobs, dst_offset, box, keep_padding=False):
    """The copy of a box of the array dimensions: the values at src_offset + c
    go to dst_offset + c for every coordinate c of `box`.  Updates and
    returns `dst_blobs`."""
    r = len(src.extents)
    so = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in src_offset])
    do = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in dst_offset])
    bx = (ctypes.c_uint64 * MAX_RANK)(*[int(x) for x in box])
    if not (len(src_offset) == len(dst_offset) == len(box) == r):
        raise ValueError("offsets and box need one entry per dimension")
    rc = lib().orc_copy_box(ctypes.byref(src.record.c), ctypes.byref(src.c), _ptrs(src_blobs), so,
                            ctypes.byref(dst.c), _ptrs(dst_blobs), do, bx, 1 if keep_padding else 0)
    if rc != 0:
        raise ValueError(f"oracle copy_box failed ({rc})")
    return dst_blobs


def copy_leaves(src: Mapping, src_blobs, dst: Mapping, dst_blobs, source_leaf, keep_padding=False):
    """The copy between differing records: destination leaf k takes source
    leaf source_leaf[k] (None: the leaf keeps its bytes).  Updates and returns
    `dst_blobs`."""
    frm = (ctypes.c_int32 * max(dst.record.nleaves, 1))(*[-1 if x is None else int(x) for x in source_leaf])
    rc = lib().orc_copy_leaves(ctypes.byref(src.record.c), ctypes.byref(src.c), _ptrs(src_blobs),
                               ctypes.byref(dst.record.c), ctypes.byref(dst.c), _ptrs(dst_blobs), frm,
                               1 if keep_padding else 0)
    if rc != 0:
        raise ValueError(f"oracle copy_leaves failed ({rc})")
    return dst_blobs


def write_counts(m: Mapping):
    """Per-byte count of how many (coordinate, leaf) values map to each byte."""
    counts = [np.zeros(s, dtype=np.uint32) for s in m.blob_sizes()]
    arr = (ctypes.c_void_p * max(len(counts), 1))()
    for k, c in enumerate(counts):
        arr[k] = c.ctypes.data
    rc = lib().orc_write_counts(ctypes.byref(m.record.c), ctypes.byref(m.c), arr)
    if rc != 0:
        raise ValueError("write_counts failed")
    return counts


def copy_writes(dst: Mapping, source_leaf=None, keep_padding=False):
    """Per-byte count of the writes the copy's definition makes into `dst`:
    one per byte a value goes to, one per byte of the zero fill (none with
    keep_padding).  source_leaf: as in copy_leaves (None entries keep their
    bytes); None: the plain copy."""
    counts = [np.zeros(s, dtype=np.uint32) for s in dst.blob_sizes()]
    arr = (ctypes.c_void_p * max(len(counts), 1))()
    for k, c in enumerate(counts):
        arr[k] = c.ctypes.data
    frm = None
    if source_leaf is not None:
        frm = (ctypes.c_int32 * max(dst.record.nleaves, 1))(*[-1 if x is None else int(x) for x in source_leaf])
    rc = lib().orc_copy_writes(ctypes.byref(dst.record.c), ctypes.byref(dst.c), frm, 1 if keep_padding else 0, arr)
    if rc != 0:
        raise ValueError("copy_writes failed")
    return counts


def check_samples(src: Mapping, src_blobs, dst: Mapping, dst_blobs, idx, leaf):
    """Counts sampled (linear index, leaf) values whose destination bytes differ
    from their source bytes.  Returns (mismatches, first mismatching sample)."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    leaf = np.ascontiguousarray(leaf, dtype=np.int32)
    first = ctypes.c_int64()
    bad = lib().orc_check_samples(
        ctypes.byref(src.record.c), ctypes.byref(src.c), _ptrs(src_blobs), ctypes.byref(dst.c),
        _ptrs(dst_blobs), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        leaf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(idx.size), ctypes.byref(first))
    if bad < 0:
        raise ValueError("check_samples failed")
    return int(bad), int(first.value)


def padding_masks(m: Mapping):
    """Per blob, a boolean mask of the bytes no value maps to (padding)."""
    return [c == 0 for c in write_counts(m)]
