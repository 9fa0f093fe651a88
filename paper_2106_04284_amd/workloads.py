"""Seeded synthetic inputs shaped like the LLAMA paper's workloads.

This module is shared by the library's tests, the benchmark and the oracle
checks.  It holds only record shapes and random values: no offsets, no blob
sizes, no layout arithmetic.  Each caller lays the values out with its own code.

Records use a neutral nested form: a record is a list of members; a member is
an elemental type name, a nested list (a nested record), or ``(member, count)``
for a static array (LLAMA sec. 3.3 turns ``T[n]`` into a record of n fields).

Workloads:
  * particle -- the n-body particle of sec. 4.1: pos{x,y,z}, vel{x,y,z}, mass,
    all float32;
  * lbm      -- a lattice-Boltzmann cell: 19 float64 distributions plus one
    32-bit flag word (sec. 4.3 describes 20 doubles per cell, one used as a bit
    set; the flag word stands in for it);
  * mixed    -- {f64[3], f32[4], i32[2], u8}, a heterogeneous record standing
    in for the 100-field HEP event record of sec. 4.2, whose definition the
    paper does not print;
  * listing1 -- the Particle of Listing 1 ({u16, {f32, f32}, f64, bool[3]}).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2106_04284

PARTICLE = [["f32", "f32", "f32"], ["f32", "f32", "f32"], "f32"]
LBM = [("f64", 19), "u32"]
MIXED = [("f64", 3), ("f32", 4), ("i32", 2), "u8"]
LISTING1 = ["u16", ["f32", "f32"], "f64", ("bool", 3)]

RECORDS = {"particle": PARTICLE, "lbm": LBM, "mixed": MIXED, "listing1": LISTING1}

# the seven layouts of the particle benchmark: (kind, AoSoA lanes)
LAYOUTS = [("aos_packed", 0), ("aos_aligned", 0), ("soa_single", 0), ("soa_multi", 0),
           ("aosoa", 8), ("aosoa", 32), ("aosoa", 64)]

# bit patterns planted into raw 32-bit inputs: signalling NaN, quiet NaN,
# negative NaN with payload, -0, smallest subnormal, +inf, -inf
SPECIAL_U32 = np.array([0x7F800001, 0x7FC00000, 0xFFA5A5A5, 0x80000000, 0x00000001,
                        0x7F800000, 0xFF800000], dtype=np.uint32)

NP_DTYPES = {"u8": np.uint8, "i8": np.int8, "bool": np.uint8, "u16": np.uint16, "i16": np.int16,
             "f16": np.float16, "bf16": np.uint16, "u32": np.uint32, "i32": np.int32,
             "f32": np.float32, "u64": np.uint64, "i64": np.int64, "f64": np.float64}


def leaf_types(record):
    """Elemental type names in depth-first declaration order."""
    out = []

    def walk(m):
        if isinstance(m, tuple):
            inner, count = m
            for _ in range(int(count)):
                walk(inner)
        elif isinstance(m, list):
            for x in m:
                walk(x)
        else:
            out.append(m)
    walk(list(record))
    return out


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_bytes(nbytes: int, seed: int) -> np.ndarray:
    """Uniform random bytes (raw bit patterns, any value allowed)."""
    g = rng(seed)
    words = g.integers(0, 2**32, size=(nbytes + 3) // 4, dtype=np.uint32)
    return words.view(np.uint8)[:nbytes].copy()


def particle_values(n: int, seed: int):
    """Per-leaf arrays of the n-body particle: pos, vel ~ U[-1, 1], mass ~ U[0.1, 1]."""
    g = rng(seed)
    pos = [g.uniform(-1.0, 1.0, n).astype(np.float32) for _ in range(3)]
    vel = [g.uniform(-1.0, 1.0, n).astype(np.float32) for _ in range(3)]
    mass = g.uniform(0.1, 1.0, n).astype(np.float32)
    return pos + vel + [mass]


def raw_u32_values(nleaves: int, n: int, seed: int):
    """Per-leaf arrays of raw random 32-bit patterns (NaN payloads included),
    with the special patterns planted at fixed records of every leaf."""
    g = rng(seed)
    out = []
    for f in range(nleaves):
        a = g.integers(0, 2**32, size=n, dtype=np.uint32)
        for k, v in enumerate(SPECIAL_U32):
            for pos in (k, n // 2 + k, n - 1 - k):
                if 0 <= pos < n:
                    a[(pos + f) % n] = v
        out.append(a)
    return out


def lbm_values(n: int, seed: int):
    """Per-leaf arrays of a lattice-Boltzmann cell: 19 f64 ~ U[0, 0.1] and a
    32-bit word of random flag bits."""
    g = rng(seed)
    dist = [g.uniform(0.0, 0.1, n).astype(np.float64) for _ in range(19)]
    flags = g.integers(0, 2**32, size=n, dtype=np.uint32)
    return dist + [flags]


def typed_random_values(types, n: int, seed: int):
    """Per-leaf arrays of raw random bits, one array per leaf type."""
    g = rng(seed)
    out = []
    for t in types:
        dt = np.dtype(NP_DTYPES[t])
        raw = g.integers(0, 256, size=n * dt.itemsize, dtype=np.uint8)
        out.append(raw.view(dt))
    return out


def batch_items(seed: int = BASE_SEED + 4, count: int = 1000, nmin: float = 1e3, nmax: float = 1e7):
    """The batching workload: record counts log-uniform in [nmin, nmax), record
    type particle or mixed with probability 1/2 each, and a (source, destination)
    layout pair drawn uniformly from the 42 ordered pairs of distinct layouts."""
    g = rng(seed)
    pairs = [(a, b) for a in LAYOUTS for b in LAYOUTS if a != b]
    items = []
    for _ in range(count):
        n = int(math.floor(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        rec = "particle" if g.random() < 0.5 else "mixed"
        src, dst = pairs[int(g.integers(0, len(pairs)))]
        items.append({"record": rec, "n": n, "src": src, "dst": dst})
    return items


def poisson_trace(seed: int, rate_per_s: float, count: int, pmin: float = 64e3, pmax: float = 1e9):
    """The serving workload: Poisson arrivals at `rate_per_s`, payload
    log-uniform in [pmin, pmax) bytes, record type and layout pair as in the
    batching workload.  Each request carries its payload in bytes; the caller
    turns it into a record count with its own record size."""
    g = rng(seed)
    pairs = [(a, b) for a in LAYOUTS for b in LAYOUTS if a != b]
    t = 0.0
    reqs = []
    for _ in range(count):
        t += g.exponential(1.0 / rate_per_s)
        payload = math.exp(g.uniform(math.log(pmin), math.log(pmax)))
        rec = "particle" if g.random() < 0.5 else "mixed"
        src, dst = pairs[int(g.integers(0, len(pairs)))]
        reqs.append({"t": t, "payload": payload, "record": rec, "src": src, "dst": dst})
    return reqs
