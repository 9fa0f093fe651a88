"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test compares the oracle with something it does not share code with: the
C compiler's struct layout (ctypes), numpy structured dtypes and reshapes, a
constructive byte-by-byte serialiser written from the paper's prose definitions
of the mappings (LLAMA sec. 3.7), the iteration order the paper prints
(sec. 3.6, Listing 7), equivalences the paper states (sec. 4.2: SoA is AoSoA
with L equal to the record count; sec. 3.9: identical mappings copy as memcpy),
and invariants of a byte permutation (round trip, composition, exactly-once
coverage).
"""
import ctypes
import os
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from paper_2106_04284_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KINDS = ["aos_packed", "aos_aligned", "soa_single", "soa_multi", "soa_aligned", "aosoa"]
SIZES = {"u8": 1, "i8": 1, "bool": 1, "u16": 2, "i16": 2, "u32": 4, "i32": 4, "f32": 4,
         "u64": 8, "i64": 8, "f64": 8}


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _layouts(lanes=(1, 2, 4, 8, 32, 64)):
    out = [(k, 0) for k in KINDS if k != "aosoa"]  # aligned SoA: 0 means sub-arrays 256-byte aligned
    out += [("soa_aligned", 16)]
    out += [("aosoa", L) for L in lanes]
    return out


def _unique_leaf_values(types, n, seed):
    """Per-leaf arrays whose bytes are random; records stay distinguishable."""
    return W.typed_random_values(types, n, seed)


def _soa_multi_blobs(values):
    return [np.ascontiguousarray(v).view(np.uint8).reshape(-1).copy() for v in values]


def _build(orc, rec, kind, extents, lanes, values):
    """A source blob set of the given layout holding `values` (per leaf), built
    by the oracle from the multi-blob SoA form (whose blobs are the per-leaf
    arrays by definition)."""
    r = orc.Record(rec)
    mb = orc.Mapping(r, "soa_multi", extents)
    m = orc.Mapping(r, kind, extents, lanes)
    return orc.copy(mb, _soa_multi_blobs(values), m)


# --------------------------------------------------------------------------
# Serialiser written from the paper's prose (sec. 3.7 "Mappings"), building
# each layout by appending bytes; it computes no offsets.
# --------------------------------------------------------------------------

def _serialise(types, values, kind, n, lanes):
    leaf_bytes = [np.ascontiguousarray(v).view(np.uint8).reshape(n, -1) if n else None for v in values]
    maxa = max(SIZES[t] for t in types)

    def val(i, f):
        return bytes(leaf_bytes[f][i]) if n else b""

    if kind in ("aos_packed", "aos_aligned"):
        out = bytearray()
        for i in range(n):
            start = len(out)
            for f, t in enumerate(types):
                if kind == "aos_aligned":
                    while (len(out) - start) % SIZES[t]:
                        out.append(0)
                out += val(i, f)
            if kind == "aos_aligned":
                while (len(out) - start) % maxa:
                    out.append(0)
        return [bytes(out)]
    if kind == "soa_single":
        out = bytearray()
        for f in range(len(types)):
            for i in range(n):
                out += val(i, f)
        return [bytes(out)]
    if kind == "soa_aligned":
        # one blob; before every sub-array but the first, zeros up to the
        # next multiple of the alignment (lanes, 0 meaning 256)
        a = lanes or 256
        out = bytearray()
        for f in range(len(types)):
            while f and len(out) % a:
                out.append(0)
            for i in range(n):
                out += val(i, f)
        return [bytes(out)]
    if kind == "soa_multi":
        blobs = []
        for f in range(len(types)):
            b = bytearray()
            for i in range(n):
                b += val(i, f)
            blobs.append(bytes(b))
        return blobs
    if kind == "aosoa":
        out = bytearray()
        i0 = 0
        while i0 < n:
            for f, t in enumerate(types):
                for lane in range(lanes):
                    i = i0 + lane
                    out += val(i, f) if i < n else bytes(SIZES[t])
            i0 += lanes
        return [bytes(out)]
    raise ValueError(kind)


# --------------------------------------------------------------------------
# record flattening (sec. 3.3, Listings 1-2)
# --------------------------------------------------------------------------

def test_listing1_leaf_order_and_sizes(orc):
    rows = _golden("listing1_particle.txt")
    r = orc.Record(W.LISTING1)
    assert r.nleaves == len(rows)
    assert r.sizes == [int(row[2]) for row in rows]
    assert W.leaf_types(W.LISTING1) == [row[1] for row in rows]


def test_listing2_c_struct_equals_aligned_aos(orc):
    """Listing 2's ParticleCpp, laid out by the C compiler's rules (ctypes),
    must equal the aligned AoS record of Listing 1: leaf offsets and stride."""
    class VecCpp(ctypes.Structure):
        _fields_ = [("x", ctypes.c_float), ("y", ctypes.c_float)]

    class ParticleCpp(ctypes.Structure):
        _fields_ = [("id", ctypes.c_uint16), ("pos", VecCpp), ("mass", ctypes.c_double),
                    ("flags", ctypes.c_bool * 3)]

    c_offsets = [ParticleCpp.id.offset, ParticleCpp.pos.offset + VecCpp.x.offset,
                 ParticleCpp.pos.offset + VecCpp.y.offset, ParticleCpp.mass.offset,
                 ParticleCpp.flags.offset, ParticleCpp.flags.offset + 1, ParticleCpp.flags.offset + 2]
    r = orc.Record(W.LISTING1)
    assert [r.aligned_offset(f) for f in range(r.nleaves)] == c_offsets
    assert r.aligned_size == ctypes.sizeof(ParticleCpp)
    assert r.packed_size == sum(ctypes.sizeof(t) for t in
                                (ctypes.c_uint16, ctypes.c_float, ctypes.c_float, ctypes.c_double)) + 3


@pytest.mark.parametrize("name", ["particle", "lbm", "mixed", "listing1"])
def test_record_sizes_against_numpy_dtypes(orc, name):
    """Packed offsets/size equal a numpy packed structured dtype; aligned ones
    equal numpy's align=True (C rule) dtype of the flattened leaves."""
    types = W.leaf_types(W.RECORDS[name])
    r = orc.Record(W.RECORDS[name])
    fields = [(f"f{k}", W.NP_DTYPES[t]) for k, t in enumerate(types)]
    packed = np.dtype(fields, align=False)
    aligned = np.dtype(fields, align=True)
    assert [r.packed_offset(f) for f in range(r.nleaves)] == [packed.fields[f"f{k}"][1] for k in range(len(types))]
    assert r.packed_size == packed.itemsize
    assert [r.aligned_offset(f) for f in range(r.nleaves)] == [aligned.fields[f"f{k}"][1] for k in range(len(types))]
    assert r.aligned_size == aligned.itemsize


def test_config_record_figures(orc):
    """Sizes of the workload records, each also fixed by a numpy dtype above."""
    p, l, m = (orc.Record(W.RECORDS[k]) for k in ("particle", "lbm", "mixed"))
    assert (p.nleaves, p.packed_size, p.aligned_size) == (7, 28, 28)
    assert (l.nleaves, l.packed_size, l.aligned_size) == (20, 156, 160)
    assert (m.nleaves, m.packed_size, m.aligned_size) == (10, 49, 56)
    assert [m.aligned_offset(f) for f in range(10)] == [0, 8, 16, 24, 28, 32, 36, 40, 44, 48]


def test_nested_static_arrays_flatten(orc):
    r = orc.Record([(["u8", "f64"], 2), ("u16", 3)])
    assert r.sizes == [1, 8, 1, 8, 2, 2, 2]
    with pytest.raises(ValueError):
        orc.Record("{f32,}")
    with pytest.raises(ValueError):
        orc.Record("{f33}")
    with pytest.raises(ValueError):
        orc.Record("{f32[0]}")


# --------------------------------------------------------------------------
# array dimensions (sec. 3.6 Listing 7; Listing 4)
# --------------------------------------------------------------------------

def test_index_range_order_matches_paper(orc):
    rows = _golden("index_range_3x3.txt")
    m = orc.Mapping(orc.Record(W.PARTICLE), "aos_packed", [3, 3])
    assert [m.linearize([int(a), int(b)]) for a, b in rows] == list(range(9))


@pytest.mark.parametrize("extents", [[5, 7], [2, 3, 4], [4, 1, 6, 3], [128, 256, 32]])
def test_linearize_equals_numpy_ravel(orc, extents):
    m = orc.Mapping(orc.Record(W.PARTICLE), "aos_packed", extents)
    g = np.random.default_rng(7)
    for _ in range(50):
        c = [int(g.integers(0, e)) for e in extents]
        assert m.linearize(c) == int(np.ravel_multi_index(c, extents))


def test_copy_visits_coordinates_row_major(orc):
    """A rank-3 copy AoS -> SoA equals a rank-1 copy of the same record count:
    both mappings linearise the same way, so only the linear index matters."""
    rec = W.PARTICLE
    types = W.leaf_types(rec)
    ext = [3, 5, 7]
    vals = _unique_leaf_values(types, 105, 11)
    a3 = _build(orc, rec, "aos_packed", ext, 0, vals)
    a1 = _build(orc, rec, "aos_packed", [105], 0, vals)
    assert all(np.array_equal(x, y) for x, y in zip(a3, a1))
    # and the AoS of a rank-3 view equals numpy's C-order structured array
    st_dt = np.dtype([(f"f{k}", W.NP_DTYPES[t]) for k, t in enumerate(types)])
    arr = np.zeros(ext, dtype=st_dt)
    for k in range(len(types)):
        arr[f"f{k}"] = vals[k].reshape(ext)
    assert np.array_equal(a3[0], arr.view(np.uint8).reshape(-1))


# --------------------------------------------------------------------------
# mappings against library routines and the constructive serialiser
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["particle", "mixed", "listing1", "lbm"])
@pytest.mark.parametrize("n", [0, 1, 5, 64, 67])
def test_layouts_equal_serialiser(orc, name, n):
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    vals = _unique_leaf_values(types, n, 100 + n)
    for kind, lanes in _layouts():
        got = _build(orc, rec, kind, [n], lanes, vals)
        want = _serialise(types, vals, kind, n, lanes)
        assert [bytes(b) for b in got] == want, (kind, lanes)


@pytest.mark.parametrize("name", ["particle", "mixed"])
def test_aos_equals_numpy_structured_array(orc, name):
    types = W.leaf_types(W.RECORDS[name])
    n = 257
    vals = _unique_leaf_values(types, n, 3)
    for align, kind in ((False, "aos_packed"), (True, "aos_aligned")):
        dt = np.dtype([(f"f{k}", W.NP_DTYPES[t]) for k, t in enumerate(types)], align=align)
        arr = np.zeros(n, dtype=dt)
        for k in range(len(types)):
            arr[f"f{k}"] = vals[k]
        got = _build(orc, W.RECORDS[name], kind, [n], 0, vals)
        assert np.array_equal(got[0], arr.view(np.uint8).reshape(-1)), kind


@pytest.mark.parametrize("lanes", [1, 4, 8, 32, 64])
@pytest.mark.parametrize("n", [64, 100, 257])
def test_aosoa_equals_numpy_reshape_transpose(orc, lanes, n):
    """For a record of equal-size leaves, AoSoA_L is the (F, N) value matrix,
    tail-padded to whole blocks, reshaped (F, B, L) and transposed (B, F, L)."""
    types = ["f32"] * 7
    vals = [v.view(np.uint32) for v in _unique_leaf_values(types, n, 5)]
    blocks = -(-n // lanes)
    mat = np.zeros((7, blocks * lanes), dtype=np.uint32)
    mat[:, :n] = np.stack(vals)
    want = mat.reshape(7, blocks, lanes).transpose(1, 0, 2).copy().view(np.uint8).reshape(-1)
    got = _build(orc, W.PARTICLE, "aosoa", [n], lanes, vals)
    assert np.array_equal(got[0], want)


def test_soa_blobs_equal_concatenation(orc):
    types = W.leaf_types(W.MIXED)
    n = 1001
    vals = _unique_leaf_values(types, n, 9)
    mb = _build(orc, W.MIXED, "soa_multi", [n], 0, vals)
    sb = _build(orc, W.MIXED, "soa_single", [n], 0, vals)
    for blob, v in zip(mb, vals):
        assert np.array_equal(blob, v.view(np.uint8))
    # no padding between the sub-arrays: SoA single-blob is the concatenation
    assert np.array_equal(sb[0], np.concatenate(mb))


# --------------------------------------------------------------------------
# equivalences the paper states or implies
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("n", [1, 7, 64, 300])
@pytest.mark.parametrize("align", [1, 4, 16, 256, 4096])
def test_aligned_soa_against_numpy_padding(orc, name, n, align):
    """SoA with aligned sub-arrays (the padded SoA of sec. 4.4 and sec. 3.9):
    the per-leaf arrays, each zero-padded by numpy to a multiple of the
    alignment except the last, concatenated; with alignment 1 it is the
    single-blob SoA, and every sub-array start is a multiple of the
    alignment."""
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    vals = _unique_leaf_values(types, n, 5 + n)
    arrays = [np.ascontiguousarray(v).view(np.uint8).reshape(-1) for v in vals]
    parts = [np.pad(a, (0, (-a.size) % align)) for a in arrays[:-1]] + [arrays[-1]]
    want = np.concatenate(parts)
    got = _build(orc, rec, "soa_aligned", [n], align, vals)
    assert len(got) == 1 and np.array_equal(got[0], want)
    if align == 1:
        single = _build(orc, rec, "soa_single", [n], 0, vals)
        assert np.array_equal(got[0], single[0])
    r = orc.Record(rec)
    m = orc.Mapping(r, "soa_aligned", [n], align)
    starts = np.cumsum([0] + [p.size for p in parts[:-1]])
    for f in range(r.nleaves):
        assert m.blob_nr_and_offset([0], f) == (0, int(starts[f])) and starts[f] % align == 0
        assert m.blob_nr_and_offset([n - 1], f) == (0, int(starts[f]) + (n - 1) * r.sizes[f])


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm"])
@pytest.mark.parametrize("n", [1, 7, 64, 300])
def test_soa_is_aosoa_with_n_lanes(orc, name, n):
    """Sec. 4.2: SoA can be seen as AoSoA with L equal to the record count."""
    types = W.leaf_types(W.RECORDS[name])
    vals = _unique_leaf_values(types, n, n)
    sb = _build(orc, W.RECORDS[name], "soa_single", [n], 0, vals)
    ao = _build(orc, W.RECORDS[name], "aosoa", [n], n, vals)
    assert np.array_equal(sb[0], ao[0])


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm"])
def test_packed_aos_is_aosoa_1(orc, name):
    types = W.leaf_types(W.RECORDS[name])
    vals = _unique_leaf_values(types, 77, 1)
    a = _build(orc, W.RECORDS[name], "aos_packed", [77], 0, vals)
    b = _build(orc, W.RECORDS[name], "aosoa", [77], 1, vals)
    assert np.array_equal(a[0], b[0])


def test_particle_packed_equals_aligned(orc):
    vals = _unique_leaf_values(["f32"] * 7, 500, 2)
    a = _build(orc, W.PARTICLE, "aos_packed", [500], 0, vals)
    b = _build(orc, W.PARTICLE, "aos_aligned", [500], 0, vals)
    assert np.array_equal(a[0], b[0])


def test_identical_mappings_copy_is_memcpy(orc):
    """Sec. 3.9: with identical mappings a raw copy of the blobs is correct;
    with different mappings it is not."""
    r = orc.Record(W.MIXED)
    for kind, lanes in _layouts():
        m = orc.Mapping(r, kind, [333], lanes)
        vals = _unique_leaf_values(W.leaf_types(W.MIXED), 333, 4)
        src = _build(orc, W.MIXED, kind, [333], lanes, vals)
        out = orc.copy(m, src, orc.Mapping(r, kind, [333], lanes))
        assert all(np.array_equal(x, y) for x, y in zip(out, src))
    src = _build(orc, W.MIXED, "aos_packed", [333], 0, _unique_leaf_values(W.leaf_types(W.MIXED), 333, 4))
    out = orc.copy(orc.Mapping(r, "aos_packed", [333]), src, orc.Mapping(r, "soa_single", [333]))
    assert not np.array_equal(out[0], src[0])


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
def test_exactly_once_and_padding_complement(orc, name):
    """Every value byte lands on a distinct, in-bounds destination byte; the
    bytes nobody writes are exactly the layout's padding, and they are the
    only bytes the serialiser fills with zeros on its own."""
    r = orc.Record(W.RECORDS[name])
    n = 45
    data_bytes = n * r.packed_size
    for kind, lanes in _layouts():
        m = orc.Mapping(r, kind, [n], lanes)
        for i in range(n):
            for f in range(r.nleaves):
                b, o = m.blob_nr_and_offset([i], f)
                assert o + r.sizes[f] <= m.blob_size(b)
        counts = orc.write_counts(m)
        assert all(int(c.max(initial=0)) <= 1 for c in counts), (kind, lanes)
        assert sum(int(c.sum()) for c in counts) == data_bytes
        # aligned SoA: the zeros the serialiser appends between sub-arrays
        soa_pad = len(_serialise(W.leaf_types(W.RECORDS[name]), _unique_leaf_values(W.leaf_types(W.RECORDS[name]), n, 1),
                                 "soa_aligned", n, lanes)[0]) - data_bytes
        pad_expected = {"aos_packed": 0, "soa_single": 0, "soa_multi": 0, "soa_aligned": soa_pad,
                        "aos_aligned": n * (r.aligned_size - r.packed_size),
                        "aosoa": (-(-n // max(lanes, 1)) * max(lanes, 1) - n) * r.packed_size}[kind]
        assert sum(int((c == 0).sum()) for c in counts) == pad_expected


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
def test_padding_is_zero_and_round_trip(orc, name):
    """Random source bytes, padding included: the destination's padding is zero
    whatever the source padding holds, and A -> B -> A restores every value
    byte (and every byte when the source padding was zero)."""
    r = orc.Record(W.RECORDS[name])
    n = 131
    lay = _layouts(lanes=(1, 8, 32))
    for ka, la in lay:
        a = orc.Mapping(r, ka, [n], la)
        src = [W.random_bytes(s, 17 + k) for k, s in enumerate(a.blob_sizes())]
        pad_a = orc.padding_masks(a)
        for kb, lb in lay:
            b = orc.Mapping(r, kb, [n], lb)
            mid = orc.copy(a, src, b, b.alloc(fill=0xCD))
            for blob, pad in zip(mid, orc.padding_masks(b)):
                assert not blob[pad].any()
            back = orc.copy(b, mid, a)
            for x, y, pad in zip(back, src, pad_a):
                assert np.array_equal(x[~pad], y[~pad])
                assert not x[pad].any()


@pytest.mark.parametrize("name", ["particle", "mixed", "listing1", "lbm"])
@pytest.mark.parametrize("n", [1, 5, 67])
def test_keep_padding_copy_against_serialiser(orc, name, n):
    """The other padding reading (the library's opt-in): the destination's
    padding keeps its old bytes and every value is written.  Value bytes equal
    the serialiser's layout; the padding is where the serialiser leaves zeros
    even when every value byte is 0xFF, and there the old bytes remain."""
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    vals = _unique_leaf_values(types, n, 300 + n)
    ones = [np.full(n * np.dtype(W.NP_DTYPES[t]).itemsize, 0xFF, np.uint8).view(W.NP_DTYPES[t]) for t in types]
    r = orc.Record(rec)
    lay = _layouts(lanes=(1, 8, 32))
    for ka, la in lay:
        src = _build(orc, rec, ka, [n], la, vals)
        a = orc.Mapping(r, ka, [n], la)
        for kb, lb in lay:
            b = orc.Mapping(r, kb, [n], lb)
            want = [np.frombuffer(x, np.uint8) for x in _serialise(types, vals, kb, n, lb)]
            pad = [np.frombuffer(x, np.uint8) == 0 for x in _serialise(types, ones, kb, n, lb)]
            init = [W.random_bytes(s, 7 + k) for k, s in enumerate(b.blob_sizes())]
            got = orc.copy(a, src, b, [x.copy() for x in init], keep_padding=True)
            for g, w, p, i in zip(got, want, pad, init):
                assert np.array_equal(g[~p], w[~p]), (ka, la, kb, lb)
                assert np.array_equal(g[p], i[p]), (ka, la, kb, lb)


def test_composition(orc):
    """A -> B -> C equals A -> C for every triple of layouts."""
    r = orc.Record(W.MIXED)
    n = 70
    lay = _layouts(lanes=(8, 32))
    first = orc.Mapping(r, lay[0][0], [n], lay[0][1])
    vals = _unique_leaf_values(W.leaf_types(W.MIXED), n, 21)
    base = _build(orc, W.MIXED, lay[0][0], [n], lay[0][1], vals)
    g = random.Random(5)
    for _ in range(30):
        (ka, la), (kb, lb), (kc, lc) = (g.choice(lay) for _ in range(3))
        A = orc.Mapping(r, ka, [n], la)
        B = orc.Mapping(r, kb, [n], lb)
        C = orc.Mapping(r, kc, [n], lc)
        a = orc.copy(first, base, A)
        ac = orc.copy(A, a, C)
        abc = orc.copy(B, orc.copy(A, a, B), C)
        assert all(np.array_equal(x, y) for x, y in zip(ac, abc))


def test_check_samples_detects_a_wrong_byte(orc):
    r = orc.Record(W.PARTICLE)
    n = 200
    a = orc.Mapping(r, "aos_packed", [n])
    b = orc.Mapping(r, "aosoa", [n], 8)
    src = [W.random_bytes(n * 28, 1)]
    dst = orc.copy(a, src, b)
    idx = np.repeat(np.arange(n), 7)
    leaf = np.tile(np.arange(7), n)
    assert orc.check_samples(a, src, b, dst, idx, leaf) == (0, -1)
    dst[0][8 * 4 * 3 + 5 * 4] ^= 1  # record 5, leaf 3 in AoSoA8
    bad, first = orc.check_samples(a, src, b, dst, idx, leaf)
    assert bad == 1 and (idx[first], leaf[first]) == (5, 3)


# --------------------------------------------------------------------------
# random records (hypothesis) against the serialiser
# --------------------------------------------------------------------------

_TYPES = ["u8", "u16", "u32", "f64", "i64", "bool", "f32"]


@st.composite
def _records(draw, depth=0):
    members = []
    for _ in range(draw(st.integers(1, 4))):
        choice = draw(st.integers(0, 9 if depth < 2 else 6))
        if choice <= 5:
            m = draw(st.sampled_from(_TYPES))
        else:
            m = draw(_records(depth=depth + 1))
        if draw(st.integers(0, 4)) == 0:
            m = (m, draw(st.integers(1, 3)))
        members.append(m)
    return members


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(rec=_records(), n=st.integers(0, 40), lanes=st.sampled_from([1, 2, 4, 8, 16, 32, 64]),
       kind=st.sampled_from(KINDS), seed=st.integers(0, 2**31))
def test_random_records_against_serialiser(orc, rec, n, lanes, kind, seed):
    types = W.leaf_types(rec)
    if len(types) > 24:
        return
    vals = _unique_leaf_values(types, n, seed)
    got = _build(orc, rec, kind, [n], lanes if kind in ("aosoa", "soa_aligned") else 0, vals)
    want = _serialise(types, vals, kind, n, lanes)
    assert [bytes(b) for b in got] == want


# --------------------------------------------------------------------------
# Split (sec. 3.7): the selected leaves through one mapping, the others through
# another, each part over its own sub-record and in its own blobs
# --------------------------------------------------------------------------

def _split_ranges(F):
    out = {(0, 1), (0, F - 1), (1, F - 1), (F // 2, 1), (1, max(F - 2, 1))}
    return sorted((a, c) for a, c in out if c >= 1 and c < F and a + c <= F)


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("n", [0, 1, 5, 67])
def test_split_equals_serialised_parts(orc, name, n):
    """A Split layout is the prose serialiser's layout of the selected leaves
    (as a record of their own) followed by its layout of the other leaves."""
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    F = len(types)
    vals = _unique_leaf_values(types, n, 40 + n)
    r = orc.Record(rec)
    src = orc.Mapping(r, "soa_multi", [n])
    rng = random.Random(F * 100 + n)
    parts = _layouts(lanes=(1, 4, 32))
    for first, count in _split_ranges(F):
        sel = list(range(first, first + count))
        rest = [f for f in range(F) if f not in sel]
        for p0 in parts:
            p1 = rng.choice(parts)
            m = orc.Mapping(r, "split", [n], split=(first, count, p0, p1))
            got = orc.copy(src, _soa_multi_blobs(vals), m)
            want = (_serialise([types[f] for f in sel], [vals[f] for f in sel], p0[0], n, p0[1]) +
                    _serialise([types[f] for f in rest], [vals[f] for f in rest], p1[0], n, p1[1]))
            assert [bytes(b) for b in got] == want, (first, count, p0, p1)


def test_split_of_multi_blob_soa_permutes_its_blobs(orc):
    """Splitting multi-blob SoA into two multi-blob SoA parts only reorders the
    blobs: the selected leaves' blobs first, then the others in leaf order."""
    types = W.leaf_types(W.MIXED)
    F, n = len(types), 333
    vals = _unique_leaf_values(types, n, 12)
    r = orc.Record(W.MIXED)
    mb = orc.Mapping(r, "soa_multi", [n])
    whole = _soa_multi_blobs(vals)
    for first, count in _split_ranges(F):
        m = orc.Mapping(r, "split", [n], split=(first, count, ("soa_multi", 0), ("soa_multi", 0)))
        got = orc.copy(mb, whole, m)
        order = list(range(first, first + count)) + [f for f in range(F) if not first <= f < first + count]
        assert len(got) == F
        for b, f in enumerate(order):
            assert np.array_equal(got[b], whole[f]), (first, count, b)


@pytest.mark.parametrize("name", ["particle", "mixed"])
def test_split_exactly_once_and_round_trip(orc, name):
    """Every value byte of a Split layout is written exactly once, its only
    unwritten bytes are its parts' padding, and AoS -> Split -> AoS is the
    identity."""
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    F, n = len(types), 45
    r = orc.Record(rec)
    S = sum(SIZES[t] for t in types)
    for first, count in _split_ranges(F):
        for p0, p1 in ((("aos_aligned", 0), ("aosoa", 8)), (("aosoa", 4), ("soa_single", 0)),
                       (("soa_multi", 0), ("aos_packed", 0))):
            m = orc.Mapping(r, "split", [n], split=(first, count, p0, p1))
            counts = orc.write_counts(m)
            assert all(int(c.max(initial=0)) <= 1 for c in counts)
            assert sum(int(c.sum()) for c in counts) == n * S
            aos = orc.Mapping(r, "aos_aligned", [n])
            start = _build(orc, rec, "aos_aligned", [n], 0, _unique_leaf_values(types, n, first + count))
            back = orc.copy(m, orc.copy(aos, start, m), aos)
            assert np.array_equal(back[0], start[0])


# --------------------------------------------------------------------------
# One (sec. 3.7): the array dimensions collapse to a single record
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("ext", [[1], [37], [4, 9]])
def test_one_broadcasts_a_single_packed_record(orc, name, ext):
    """One holds one packed record whatever the extents; copied into packed
    AoS it is that record repeated (numpy tile), and every value byte of it
    is read by every coordinate."""
    rec = W.RECORDS[name]
    types = W.leaf_types(rec)
    r = orc.Record(rec)
    one = orc.Mapping(r, "one", ext)
    S = sum(SIZES[t] for t in types)
    n = int(np.prod(ext))
    assert one.blob_sizes() == [S]
    blob = [np.frombuffer(bytes(random.Random(n).randrange(256) for _ in range(S)), np.uint8).copy()]
    aos = orc.copy(one, blob, orc.Mapping(r, "aos_packed", ext))
    assert np.array_equal(aos[0], np.tile(blob[0], n))
    assert [int(c.min()) for c in orc.write_counts(one)] == [n]


def test_split_with_one_part_reads_a_shared_value(orc):
    """Split of the particle with mass through One (the nesting of sec. 3.7's
    listing, one level deep): into multi-blob SoA, every record gets the same
    mass and its own position and velocity."""
    n = 50
    r = orc.Record(W.PARTICLE)
    m = orc.Mapping(r, "split", [n], split=(6, 1, ("one", 0), ("soa_multi", 0)))
    assert m.blob_sizes() == [4] + [4 * n] * 6
    rng = np.random.default_rng(3)
    src = [rng.integers(0, 256, s, dtype=np.uint8) for s in m.blob_sizes()]
    out = orc.copy(m, src, orc.Mapping(r, "soa_multi", [n]))
    for f in range(6):
        assert np.array_equal(out[f], src[1 + f])
    assert np.array_equal(out[6], np.tile(src[0], n))


@pytest.mark.parametrize("n", [1, 9, 70])
def test_nested_split_equals_serialised_parts(orc, n):
    """A Split whose rest is itself a Split (the nesting in sec. 3.7's mapping
    listing): the blobs are the prose serialiser's layouts of the three parts,
    in order: the selected leaves, then the inner split's selected leaves,
    then the remaining ones."""
    types = W.leaf_types(W.PARTICLE)
    vals = _unique_leaf_values(types, n, 77 + n)
    r = orc.Record(W.PARTICLE)
    for inner0, inner1 in ((("aosoa", 4), ("aos_aligned", 0)), (("soa_single", 0), ("aos_packed", 0))):
        m = orc.Mapping(r, "split", [n], split=(3, 3, ("soa_multi", 0), ("split", (3, 1, inner0, inner1))))
        got = orc.copy(orc.Mapping(r, "soa_multi", [n]), _soa_multi_blobs(vals), m)
        want = (_serialise(types[3:6], vals[3:6], "soa_multi", n, 0) +
                _serialise(types[6:7], vals[6:7], inner0[0], n, inner0[1]) +
                _serialise(types[0:3], vals[0:3], inner1[0], n, inner1[1]))
        assert [bytes(b) for b in got] == want, (inner0, inner1)
    # the listing's own shape: velocities as SoA, mass through One, positions as aligned AoS
    c = orc.Mapping(r, "split", [n], split=(3, 3, ("soa_multi", 0), ("split", (3, 1, ("one", 0), ("aos_aligned", 0)))))
    assert c.blob_sizes() == [4 * n] * 3 + [4, 12 * n]
    src = [np.random.default_rng(n).integers(0, 256, s, dtype=np.uint8) for s in c.blob_sizes()]
    aos = orc.copy(c, src, orc.Mapping(r, "aos_packed", [n]))[0].reshape(n, 28)
    assert (aos[:, 24:28] == src[3]).all()
    assert np.array_equal(aos[:, 0:12].reshape(-1), src[4])


# --------------------------------------------------------------------------
# copies between differing records (sec. 3.9: a field missing on one side)
# --------------------------------------------------------------------------

PARTICLE_NO_MASS = [["f32", "f32", "f32"], ["f32", "f32", "f32"]]


@pytest.mark.parametrize("kind", _layouts(lanes=(4, 32)))
@pytest.mark.parametrize("n", [1, 45])
def test_copy_leaves_field_missing_on_either_side(orc, kind, n):
    """Into a record without mass: the serialiser's layout of the six common
    leaves.  Into a record with mass from one without: the mass keeps its
    bytes (unused AoSoA lanes included), everything else as the serialiser."""
    types7, types6 = W.leaf_types(W.PARTICLE), W.leaf_types(PARTICLE_NO_MASS)
    vals = _unique_leaf_values(types7, n, 5 + n)
    r7, r6 = orc.Record(W.PARTICLE), orc.Record(PARTICLE_NO_MASS)
    src7 = orc.copy(orc.Mapping(r7, "soa_multi", [n]), _soa_multi_blobs(vals), orc.Mapping(r7, "aos_packed", [n]))
    m6 = orc.Mapping(r6, kind[0], [n], kind[1])
    got = orc.copy_leaves(orc.Mapping(r7, "aos_packed", [n]), src7, m6, m6.alloc(fill=0xEE), list(range(6)))
    assert [bytes(b) for b in got] == _serialise(types6, vals[:6], kind[0], n, kind[1])
    # the other way: mass has no source and keeps its canary, lanes past N included
    src6 = orc.copy(orc.Mapping(r6, "soa_multi", [n]), _soa_multi_blobs(vals[:6]), orc.Mapping(r6, "aos_packed", [n]))
    m7 = orc.Mapping(r7, kind[0], [n], kind[1])
    got = orc.copy_leaves(orc.Mapping(r6, "aos_packed", [n]), src6, m7, m7.alloc(fill=0xEE),
                          list(range(6)) + [None])
    canary = [np.frombuffer(bytes([0xEE]) * 4 * n, np.float32)]
    full = _serialise(types7, vals[:6] + canary, kind[0], n, kind[1])
    if kind[0] == "aosoa":  # unused lanes of the mass chunk keep the canary too
        L_, S = kind[1], 28
        blocks = -(-n // L_)
        want = bytearray(full[0])
        for i in range(n, blocks * L_):
            o = (i // L_) * L_ * S + L_ * 24 + (i % L_) * 4
            want[o:o + 4] = b"\xee" * 4
        full = [bytes(want)]
    assert [bytes(b) for b in got] == full


def test_copy_leaves_identity_and_permutation(orc):
    """The identity leaf map is the plain copy; a map that swaps two
    equal-size leaves equals the copy of the swapped values."""
    types = W.leaf_types(W.MIXED)
    n = 77
    vals = _unique_leaf_values(types, n, 8)
    r = orc.Record(W.MIXED)
    mb = orc.Mapping(r, "soa_multi", [n])
    for kind in _layouts(lanes=(8,)):
        m = orc.Mapping(r, kind[0], [n], kind[1])
        plain = orc.copy(mb, _soa_multi_blobs(vals), m)
        got = orc.copy_leaves(mb, _soa_multi_blobs(vals), m, m.alloc(fill=0x5A), list(range(len(types))))
        assert all(np.array_equal(a, b) for a, b in zip(plain, got)), kind
        # leaves 3 and 4 are both f32: swap them
        perm = list(range(len(types)))
        perm[3], perm[4] = 4, 3
        sw = list(vals)
        sw[3], sw[4] = vals[4], vals[3]
        got = orc.copy_leaves(mb, _soa_multi_blobs(vals), m, m.alloc(fill=0x5A), perm)
        want = orc.copy(mb, _soa_multi_blobs(sw), m)
        assert all(np.array_equal(a, b) for a, b in zip(want, got)), kind


# --------------------------------------------------------------------------
# the threaded copy used to time the oracle on all host cores (sec. 4 runs one
# thread per physical core): the same bytes as the serial copy
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("ext", [[1], [67], [1000], [3, 5, 7]])
def test_threaded_copy_equals_serial_copy(orc, name, ext):
    rec = W.RECORDS[name]
    r = orc.Record(rec)
    n = int(np.prod(ext))
    layouts = _layouts(lanes=(1, 8, 32))
    g = random.Random(hash((name, n)) & 0xFFFF)
    for a, b in g.sample([(a, b) for a in layouts for b in layouts], 12) + [(("aos_packed", 0), ("aosoa", 8))]:
        ms, md = orc.Mapping(r, a[0], ext, a[1]), orc.Mapping(r, b[0], ext, b[1])
        src = [W.random_bytes(s, 5 + k) for k, s in enumerate(ms.blob_sizes())]
        want = orc.copy(ms, src, md)
        for threads in (1, 3, 8):
            got = orc.copy_threads(ms, src, md, [W.random_bytes(s, 9) for s in md.blob_sizes()], threads=threads)
            assert all(np.array_equal(x, y) for x, y in zip(got, want)), (a, b, threads)
            kept = [W.random_bytes(s, 11) for s in md.blob_sizes()]
            want_k = orc.copy(ms, src, md, [x.copy() for x in kept], keep_padding=True)
            got_k = orc.copy_threads(ms, src, md, kept, keep_padding=True, threads=threads)
            assert all(np.array_equal(x, y) for x, y in zip(got_k, want_k)), (a, b, threads, "keep")


def test_threaded_copy_splits_and_one(orc):
    r = orc.Record(W.PARTICLE)
    n = 777
    S = ("split", (0, 3, ("aosoa", 8), ("soa_multi", 0)))
    cases = [(S, ("aos_aligned", 0)), (("aos_packed", 0), S), (("one", 0), ("soa_single", 0)),
             (("aos_packed", 0), ("split", (3, 4, ("one", 0), ("aos_packed", 0))))]
    for a, b in cases:
        ms = orc.Mapping(r, a[0], [n], split=a[1]) if a[0] == "split" else orc.Mapping(r, a[0], [n], a[1])
        md = orc.Mapping(r, b[0], [n], split=b[1]) if b[0] == "split" else orc.Mapping(r, b[0], [n], b[1])
        src = [W.random_bytes(s, 21 + k) for k, s in enumerate(ms.blob_sizes())]
        want = orc.copy(ms, src, md)
        got = orc.copy_threads(ms, src, md, threads=8)
        assert all(np.array_equal(x, y) for x, y in zip(got, want)), (a, b)


def test_memcpy_threads_copies_every_byte(orc):
    src = W.random_bytes(1 << 20 | 13, 3)
    for threads in (1, 5, 8):
        dst = np.zeros(src.size + 7, dtype=np.uint8)
        used = orc.memcpy_threads(dst, src, threads)
        assert 1 <= used <= threads
        assert np.array_equal(dst[:src.size], src) and not dst[src.size:].any()


# --------------------------------------------------------------------------
# linearizers (sec. 3.7 lists the linearizer among a mapping's building
# blocks; sec. 2 points to other storage orders and space-filling curves)
# --------------------------------------------------------------------------

def _coords(ext):
    return [tuple(int(x) for x in c) for c in np.ndindex(*ext)]


@pytest.mark.parametrize("ext", [[7], [5, 7], [2, 3, 4], [4, 1, 6, 3]])
def test_column_major_equals_numpy_fortran_order(orc, ext):
    r = orc.Record(W.PARTICLE)
    m = orc.Mapping(r, "aos_packed", ext, linearizer="col")
    assert m.linear_size == int(np.prod(ext))
    for c in _coords(ext):
        assert m.linearize(c) == int(np.ravel_multi_index(c, ext, order="F"))


def test_morton_4x4_golden(orc):
    want = [[int(x) for x in row] for row in _golden("morton_4x4.txt")]
    m = orc.Mapping(orc.Record(W.PARTICLE), "aos_packed", [4, 4], linearizer="morton")
    assert [[m.linearize([y, x]) for x in range(4)] for y in range(4)] == want


def _z_recursive(c, k):
    """Z-order index of coordinate c in a grid of side 2^k, built by recursion
    on quadrants: the quadrant of c's top bits (first dimension most
    significant) times the cells per quadrant, plus c's index inside it."""
    if k == 0:
        return 0
    half = 1 << (k - 1)
    quadrant = 0
    for x in c:
        quadrant = quadrant * 2 + (1 if x >= half else 0)
    return quadrant * half ** len(c) + _z_recursive([x % half for x in c], k - 1)


@pytest.mark.parametrize("ext", [[8, 8], [4, 4, 4], [2, 2, 2, 2], [16, 16]])
def test_morton_equals_recursive_quadrants(orc, ext):
    m = orc.Mapping(orc.Record(W.PARTICLE), "aos_packed", ext, linearizer="morton")
    k = int(ext[0]).bit_length() - 1
    idx = [m.linearize(c) for c in _coords(ext)]
    assert idx == [_z_recursive(list(c), k) for c in _coords(ext)]
    assert sorted(idx) == list(range(int(np.prod(ext))))  # a bijection when every extent is 2^k
    assert m.linear_size == int(np.prod(ext))


@pytest.mark.parametrize("ext", [[3, 5], [5, 3], [6, 2, 3], [9], [1, 7]])
def test_morton_ragged_extents(orc, ext):
    """Extents that are not one power of two: the Z index of the coordinate in
    the enclosing grid of side 2^k, injective, growing along every dimension;
    the mapping lays out up to the last coordinate's index."""
    m = orc.Mapping(orc.Record(W.PARTICLE), "aos_packed", ext, linearizer="morton")
    k = max(int(e - 1).bit_length() for e in ext)
    idx = {c: m.linearize(c) for c in _coords(ext)}
    assert all(idx[c] == _z_recursive(list(c), k) for c in idx)
    assert len(set(idx.values())) == len(idx)
    assert m.linear_size == max(idx.values()) + 1
    assert m.blob_sizes() == [m.linear_size * 28]


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm"])
@pytest.mark.parametrize("lin", ["col", "morton"])
def test_linearizer_layouts(orc, name, lin):
    """Multi-blob SoA under a linearizer holds each leaf's values at their
    linear index (numpy fancy indexing): column-major is numpy's Fortran
    order; Morton slots no coordinate reaches are zero.  Every other layout
    round-trips through it, and exactly-once coverage holds with the holes as
    padding."""
    ext = [5, 6] if lin == "morton" else [3, 4, 5]
    rec = W.RECORDS[name]
    r = orc.Record(rec)
    types = W.leaf_types(rec)
    n = int(np.prod(ext))
    vals = _unique_leaf_values(types, n, 17)
    src_m = orc.Mapping(r, "soa_multi", ext)
    src = _soa_multi_blobs(vals)
    dst_m = orc.Mapping(r, "soa_multi", ext, linearizer=lin)
    got = orc.copy(src_m, src, dst_m)
    if lin == "col":
        want = [np.ascontiguousarray(np.asarray(v).reshape(ext).ravel(order="F")).view(np.uint8) for v in vals]
    else:
        k = max(int(e - 1).bit_length() for e in ext)
        z = np.array([_z_recursive(list(c), k) for c in _coords(ext)])
        want = []
        for v in vals:
            w = np.zeros(dst_m.linear_size, dtype=v.dtype)
            w[z] = v
            want.append(w.view(np.uint8))
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_, w_)
    for kind, lanes in _layouts(lanes=(4, 8)):
        m = orc.Mapping(r, kind, ext, lanes, linearizer=lin)
        there = orc.copy(src_m, src, m)
        back = orc.copy(m, there, src_m)
        assert all(np.array_equal(x, y) for x, y in zip(back, src)), kind
        counts = orc.write_counts(m)
        assert all(c.max() <= 1 for c in counts)
        assert sum(int(c.sum()) for c in counts) == n * r.packed_size
        for blob, pad in zip(there, orc.padding_masks(m)):
            assert not blob[pad].any()


def test_copy_between_linearizers_commutes(orc):
    r = orc.Record(W.MIXED)
    ext = [5, 3, 4]
    vals = _unique_leaf_values(W.leaf_types(W.MIXED), 60, 3)
    a = orc.Mapping(r, "soa_multi", ext)
    src = _soa_multi_blobs(vals)
    b = orc.Mapping(r, "aosoa", ext, 8, linearizer="morton")
    c = orc.Mapping(r, "aos_aligned", ext, linearizer="col")
    via_b = orc.copy(b, orc.copy(a, src, b), c)
    direct = orc.copy(a, src, c)
    assert all(np.array_equal(x, y) for x, y in zip(via_b, direct))


# --------------------------------------------------------------------------
# box copies (sec. 3.2 VirtualView onto a sub-box; sec. 3.9 copies between
# views of different size or shape)
# --------------------------------------------------------------------------

BOX_CASES = [([9], [13], [2], [5], [6]), ([5, 7], [6, 4], [1, 2], [3, 0], [2, 4]),
             ([4, 5, 6], [6, 5, 4], [1, 0, 2], [2, 1, 0], [3, 4, 3]), ([4, 4], [4, 4], [0, 0], [0, 0], [4, 4]),
             ([3, 3], [3, 3], [1, 1], [0, 0], [0, 2])]


@pytest.mark.parametrize("case", BOX_CASES, ids=[str(c[4]) for c in BOX_CASES])
@pytest.mark.parametrize("name", ["particle", "mixed", "listing1"])
def test_box_copy_equals_numpy_slicing(orc, case, name):
    se, de, so, do, box = case
    rec = W.RECORDS[name]
    r = orc.Record(rec)
    types = W.leaf_types(rec)
    V = _unique_leaf_values(types, int(np.prod(se)), 5)
    Wv = _unique_leaf_values(types, int(np.prod(de)), 6)
    sl_s = tuple(slice(o, o + b) for o, b in zip(so, box))
    sl_d = tuple(slice(o, o + b) for o, b in zip(do, box))
    expect_vals = []
    for v, w in zip(V, Wv):
        w2 = np.array(w).reshape(de).copy()
        w2[sl_d] = np.array(v).reshape(se)[sl_s]
        expect_vals.append(w2.reshape(-1))
    g = random.Random(hash((name, tuple(box))) & 0xFFFF)
    for a, b in g.sample([(a, b) for a in _layouts((4, 8)) for b in _layouts((4, 8))], 10):
        for lin in ("row", "morton"):
            ms = orc.Mapping(r, a[0], se, a[1], linearizer=lin)
            md = orc.Mapping(r, b[0], de, b[1], linearizer="row" if lin == "morton" else "col")
            src = orc.copy(orc.Mapping(r, "soa_multi", se), _soa_multi_blobs(V), ms)
            dst = orc.copy(orc.Mapping(r, "soa_multi", de), _soa_multi_blobs(Wv), md)
            orc.copy_box(ms, src, so, md, dst, do, box)
            want = orc.copy(orc.Mapping(r, "soa_multi", de), _soa_multi_blobs(expect_vals), md)
            assert all(np.array_equal(x, y) for x, y in zip(dst, want)), (a, b, lin)


def test_box_copy_touches_only_the_box(orc):
    """Brute force over every destination byte: bytes of the box's values hold
    the source's values, the box records' alignment gaps are zero (or keep
    their bytes), every other byte keeps its value."""
    rec = W.MIXED
    r = orc.Record(rec)
    se, de, so, do, box = [4, 6], [5, 5], [1, 2], [2, 0], [3, 4]
    ms = orc.Mapping(r, "aosoa", se, 4)
    md = orc.Mapping(r, "aos_aligned", de)
    src = [W.random_bytes(s, 1) for s in ms.blob_sizes()]
    before = [W.random_bytes(s, 2) for s in md.blob_sizes()]
    R = r.aligned_size
    for keep in (False, True):
        dst = orc.copy_box(ms, src, so, md, [x.copy() for x in before], do, box, keep_padding=keep)
        value_bytes, box_records = {}, set()
        for c in _coords(box):
            sc = [o + x for o, x in zip(so, c)]
            dc = [o + x for o, x in zip(do, c)]
            box_records.add(int(np.ravel_multi_index(dc, de)))
            for f in range(r.nleaves):
                bs, os_ = ms.blob_nr_and_offset(sc, f)
                bd, od = md.blob_nr_and_offset(dc, f)
                for k in range(r.sizes[f]):
                    value_bytes[od + k] = src[bs][os_ + k]
        for o in range(md.blob_size(0)):
            if o in value_bytes:
                assert dst[0][o] == value_bytes[o]
            elif o // R in box_records and not keep:
                assert dst[0][o] == 0
            else:
                assert dst[0][o] == before[0][o]


def test_box_copy_of_everything_is_the_copy(orc):
    r = orc.Record(W.LBM)
    ext = [3, 4, 5]
    for a, b in [(("aos_aligned", 0), ("aosoa", 8)), (("soa_single", 0), ("aos_aligned", 0))]:
        ms, md = orc.Mapping(r, a[0], ext, a[1]), orc.Mapping(r, b[0], ext, b[1])
        src = [W.random_bytes(s, 4) for s in ms.blob_sizes()]
        got = orc.copy_box(ms, src, [0, 0, 0], md, md.alloc(), [0, 0, 0], ext)
        assert all(np.array_equal(x, y) for x, y in zip(got, orc.copy(ms, src, md)))


def test_box_copy_rejects_boxes_outside_a_view(orc):
    r = orc.Record(W.PARTICLE)
    ms, md = orc.Mapping(r, "aos_packed", [4, 4]), orc.Mapping(r, "soa_multi", [3, 5])
    src, dst = ms.alloc(), md.alloc()
    with pytest.raises(ValueError):
        orc.copy_box(ms, src, [1, 0], md, dst, [0, 0], [4, 1])
    with pytest.raises(ValueError):
        orc.copy_box(ms, src, [0, 0], md, dst, [0, 2], [1, 4])


# --------------------------------------------------------------------------
# the writes of the definition (Heatmap of the copy, sec. 3.7)
# --------------------------------------------------------------------------

def _written_by_two_fills(run, sizes):
    """Which destination bytes a copy writes, found by running it on a
    destination of 0x00 bytes and on one of 0xFF bytes: a written byte holds
    the same value both times, an untouched one its fill."""
    a = run([np.zeros(s, np.uint8) for s in sizes])
    b = run([np.full(s, 0xFF, np.uint8) for s in sizes])
    return [(x == y).astype(np.uint32) for x, y in zip(a, b)]


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
def test_copy_writes_match_two_fill_coverage(orc, name):
    """copy_writes, the per-byte writes of the definition, is at most one per
    byte and equals the bytes the oracle's copies change, for the plain copy
    (every byte: values, and zeros on padding), the copy that keeps padding,
    and copies between differing records (leaves without a source keep their
    bytes, their unused AoSoA lanes included)."""
    import random
    r = orc.Record(W.RECORDS[name])
    g = random.Random(7)
    for n in (1, 13, 45):
        for kind, lanes in _layouts():
            md = orc.Mapping(r, kind, [n], lanes)
            ms = orc.Mapping(r, "aos_packed", [n])
            src = [W.random_bytes(s, 11) for s in ms.blob_sizes()]
            sizes = md.blob_sizes()
            plain = orc.copy_writes(md)
            assert all(bool((c == 1).all()) for c in plain), (kind, lanes, n)
            keep = orc.copy_writes(md, keep_padding=True)
            want = _written_by_two_fills(lambda d: orc.copy(ms, src, md, d, keep_padding=True), sizes)
            assert all(np.array_equal(x, y) for x, y in zip(keep, want)), (kind, lanes, n)
            for keep_padding in (False, True):
                frm = [None if g.random() < 0.4 else f for f in range(r.nleaves)]
                if all(x is None for x in frm):
                    frm[0] = 0
                got = orc.copy_writes(md, source_leaf=frm, keep_padding=keep_padding)
                want = _written_by_two_fills(
                    lambda d: orc.copy_leaves(ms, src, md, d, frm, keep_padding=keep_padding), sizes)
                assert all(np.array_equal(x, y) for x, y in zip(got, want)), (kind, lanes, n, frm, keep_padding)

