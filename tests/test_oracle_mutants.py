"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong index, a wrong operand) in
a copy of the oracle's C source, builds it on the CPU, and runs the pin suite
against that build in a subprocess.  The pin suite must fail for every mutant.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "llama_oracle.c")

MUTANTS = {
    "aligned_offset_no_rounding": ("off = round_up(off, r->align[g]);", "off = off;"),
    "aligned_stride_no_tail_rounding": ("return round_up(end, max_align);", "return end;"),
    "packed_offset_drops_a_leaf": ("for (int g = 0; g < f; g++)", "for (int g = 1; g < f; g++)"),
    "linearize_wrong_extent": ("for (int d = 0; d < m->rank; d++)\n        i = i * m->extents[d] + coord[d];",
                               "for (int d = 0; d < m->rank; d++)\n        i = i * m->extents[0] + coord[d];"),
    "column_major_is_row_major": ("for (int d = m->rank - 1; d >= 0; d--)\n            i = i * m->extents[d] + coord[d];",
                                  "for (int d = 0; d < m->rank; d++)\n            i = i * m->extents[d] + coord[d];"),
    "morton_first_dimension_lowest": ("i += (uint64_t)1 << (j * m->rank + (m->rank - 1 - d));",
                                      "i += (uint64_t)1 << (j * m->rank + d);"),
    "morton_size_is_record_count": ("    if (m->linearizer != ORC_MORTON || n == 0)\n        return n;",
                                    "    if (1)\n        return n;"),
    "box_source_offset_dropped": ("sc[d] = src_offset[d] + c[d];", "sc[d] = c[d];"),
    "box_destination_uses_source_offset": ("dc[d] = dst_offset[d] + c[d];", "dc[d] = src_offset[d] + c[d];"),
    "box_gaps_not_zeroed": ("memset(dst_blobs[0] + orc_linearize(dst, dc) * R, 0, (size_t)R);", "(void)R;"),
    "soa_single_wrong_element_size": ("*offset = n * orc_packed_offset(r, f) + i * r->size[f];",
                                      "*offset = n * orc_packed_offset(r, f) + i * r->size[0];"),
    "soa_single_base_uses_index": ("*offset = n * orc_packed_offset(r, f) + i * r->size[f];",
                                   "*offset = i * orc_packed_offset(r, f) + i * r->size[f];"),
    "soa_multi_one_blob": ("*blob = (uint64_t)f;", "*blob = 0;"),
    "aosoa_lane_stride": ("lane * r->size[f];", "lane * r->size[0];"),
    "aosoa_block_stride_aligned": ("block * (L * orc_packed_size(r))", "block * (L * orc_aligned_size(r))"),
    "aosoa_swapped_split": ("uint64_t block = i / L;\n        uint64_t lane = i % L;",
                            "uint64_t block = i % L;\n        uint64_t lane = i / L;"),
    "aosoa_blob_size_no_tail": ("return blocks * m->lanes * orc_packed_size(r);", "return n * orc_packed_size(r);"),
    "padding_not_zeroed": ("memset(dst_blobs[b], 0, (size_t)orc_blob_size(dst, r, b));", "(void)0;"),
    "keep_mode_zeroes_padding": ("                  const orc_mapping* dst, uint8_t* const* dst_blobs)\n{\n",
                                 "                  const orc_mapping* dst, uint8_t* const* dst_blobs)\n{\n"
                                 "    for (int b = 0; b < orc_blob_count(dst, r); b++)\n"
                                 "        memset(dst_blobs[b], 0, (size_t)orc_blob_size(dst, r, b));\n"),
    "split_rest_index_off": ("return f < m->first ? f : f - m->count;", "return f < m->first ? f : f - m->first;"),
    "split_rest_blobs_overlap": ("first_blob = (uint64_t)orc_blob_count(&p.m, &p.r);", "first_blob = 0;"),
    "split_selection_one_long": ("return f >= m->first && f < m->first + m->count;",
                                 "return f >= m->first && f <= m->first + m->count;"),
    "one_offset_uses_index": ("        (void)i;\n        *blob = 0;\n        *offset = orc_packed_offset(r, f);",
                              "        *blob = 0;\n        *offset = i * orc_packed_size(r) + orc_packed_offset(r, f);"),
    "copy_leaves_zeroes_kept_lanes": ("                    if (from[k] < 0)\n                        memset(owned[0]",
                                      "                    if (from[k] < -1)\n                        memset(owned[0]"),
    "copy_leaves_reads_own_index": ("orc_blob_nr_and_offset(src, rs, coord, from[k], &bs, &os);",
                                    "orc_blob_nr_and_offset(src, rs, coord, k, &bs, &os);"),
    "static_array_one_short": ("for (uint64_t c = 1; c < count; c++)", "for (uint64_t c = 2; c < count; c++)"),
    "aos_aligned_uses_packed_stride": ("*offset = i * orc_aligned_size(r) + orc_aligned_offset(r, f);",
                                       "*offset = i * orc_packed_size(r) + orc_aligned_offset(r, f);"),
    "copy_writes_no_zero_fill": ("            for (uint64_t o = 0; o < sz; o++)\n                if (!owned[b][o])\n                    counts[b][o]++;",
                                 "            for (uint64_t o = 0; o < sz; o++)\n                if (!owned[b][o])\n                    (void)0;"),
    "copy_writes_counts_kept_leaves": ("                    if (!from || from[f] >= 0)\n                        counts[b][o + k]++;",
                                       "                    counts[b][o + k]++;"),
    "soa_aligned_no_rounding": ("start = round_up(start + n * r->size[g - 1], a);",
                                "start = start + n * r->size[g - 1];"),
    "soa_aligned_rounds_to_leaf_size": ("start = round_up(start + n * r->size[g - 1], a);",
                                        "start = round_up(start + n * r->size[g - 1], r->size[g - 1]);"),
    "soa_aligned_default_alignment": ("uint64_t a = m->lanes ? m->lanes : 256;", "uint64_t a = m->lanes ? m->lanes : 128;"),
    "threaded_piece_starts_at_origin": ("delinearize(src, lo, coord);", "(void)lo;"),
    "threaded_last_piece_drops_tail": ("uint64_t hi = k + 1 == pieces ? n : n / (uint64_t)pieces * (uint64_t)(k + 1);",
                                       "uint64_t hi = n / (uint64_t)pieces * (uint64_t)(k + 1);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", str(mutant_c), "-o", str(lib)])
    env = dict(os.environ, LLAMA_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
