"""Each plausible mistake planted in a copy of the oracle source must make at
least one pin fail (CPU only; the real oracle is never modified)."""
import os

import pytest

import oracle
from pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "numarck_oracle.c")

# (name, original text, planted mistake) -- each original occurs exactly once
MUTANTS = [
    ("ratio_sign", "double r = (q - p) / p;", "double r = (p - q) / p;"),
    ("ratio_denominator", "double r = (q - p) / p;", "double r = (q - p) / q;"),
    ("cap_dropped", "isfinite(r) && fabs(r) <= cap;", "isfinite(r);"),
    ("lo_is_max", "if (precedes(d[j], tmn)) tmn = d[j];", "if (precedes(tmn, d[j])) tmn = d[j];"),
    ("zero_order", "return a == b && signbit(a) && !signbit(b);", "return 0;"),
    ("bin_width_E", "double width = 2.0 * E;", "double width = E;"),
    ("bin_round", "(int64_t)floor((d[j] - lo) / width)", "(int64_t)round((d[j] - lo) / width)"),
    ("bin_anchor", "(int64_t)floor((d[j] - lo) / width)", "(int64_t)floor(d[j] / width)"),
    ("count_init", "counts[nb] = 1;", "counts[nb] = 0;"),
    ("M_off_by_one", "M = (int64_t)floor((hi - lo) / (2.0 * E)) + 1;",
     "M = (int64_t)floor((hi - lo) / (2.0 * E));"),
    ("topk_ascending", "return x->count > y->count ? -1 : 1;", "return x->count < y->count ? -1 : 1;"),
    ("tie_higher_id", "return (x->id > y->id) - (x->id < y->id);",
     "return (x->id < y->id) - (x->id > y->id);"),
    ("centre_lower_edge", "(double)(2 * sel[i] + 1) * E", "(double)(2 * sel[i]) * E"),
    ("centre_upper_edge", "(double)(2 * sel[i] + 1) * E", "(double)(2 * sel[i] + 2) * E"),
    ("recon_sign", "rounded_to_type(dtype, p * (1.0 + c));", "rounded_to_type(dtype, p * (1.0 - c));"),
    ("recon_unrounded", "double r = rounded_to_type(dtype, p * (1.0 + c));", "double r = p * (1.0 + c);"),
    ("verify_dropped", "if (fabs(r - q) <= E * fabs(p)) {", "if (1) {"),
    ("verify_wrong_base", "if (fabs(r - q) <= E * fabs(p)) {", "if (fabs(r - q) <= E * fabs(q)) {"),
    ("escape_stores_prev", "copy_elem(incomp, n_inc, curr, j, dtype);",
     "copy_elem(incomp, n_inc, prev, j, dtype);"),
    ("pack_msb_first", "if ((idx >> b) & 1u) packed[bit >> 5]",
     "if ((idx >> (B - 1 - b)) & 1u) packed[bit >> 5]"),
    ("block_size_bytes", "uint64_t epb = (8 * block_bytes) / B;", "uint64_t epb = block_bytes / B;"),
    ("block_offset_inclusive",
     "if (j % epb == 0 && block_inc_off) block_inc_off[j / epb] = (int64_t)seen;\n"
     "      if (idx[j] == esc) seen++;",
     "if (idx[j] == esc) seen++;\n"
     "      if (j % epb == 0 && block_inc_off) block_inc_off[j / epb] = (int64_t)seen;"),
    ("size_words_as_bytes", "+ words * 4 + n_inc * L;", "+ words + n_inc * L;"),
    ("decode_sign", "store_rounded(out, dtype, oj, p * (1.0 + c));",
     "store_rounded(out, dtype, oj, p * (1.0 - c));"),
    ("range_rank_from_zero", "uint64_t rank = (uint64_t)block_inc_off[blk];", "uint64_t rank = 0;"),
    ("bad_index_unflagged", "if (code >= info->k_used) *flags |= ORC_FLAG_BAD_INDEX;", "if (0) {}"),
    ("chooseB_k_is_2B", "const int64_t k = ((int64_t)1 << B) - 1;", "const int64_t k = (int64_t)1 << B;"),
    ("chooseB_invalid_ignored", "const uint64_t incompressible = n - covered;",
     "const uint64_t incompressible = n_valid - covered;"),
    ("chooseB_index_bytes", "+ n * (uint64_t)B +", "+ n * (uint64_t)B / 8 +"),
    ("chooseB_ties_to_larger", "if (bestB == 0 || bits[B] < best) {", "if (bestB == 0 || bits[B] <= best) {"),
    ("chooseB_counts_ascending", "return (x < y) - (x > y);", "return (x > y) - (x < y);"),
    ("ew_k_plus_one_chunks", "const double w = (hi - lo) / (double)k;",
     "const double w = (hi - lo) / (double)(k + 1);"),
    ("ew_centre_lower_edge", "lo + ((double)i + 0.5) * w", "lo + (double)i * w"),
    ("ew_no_clamp", "i = t < (double)(k - 1) ? (int64_t)t : (int64_t)(k - 1);", "i = (int64_t)t;"),
    ("ew_anchor_zero", "floor((d[j] - lo) / w)", "floor(d[j] / w)"),
    ("ew_zero_width_divides", "if (w > 0.0) {", "if (1) {"),
    ("za_anchor_plus_E", "lo = -E;\n    hi = 0.0;\n  }", "lo = E;\n    hi = 0.0;\n  }"),
    ("za_anchor_zero", "lo = -E;\n    hi = 0.0;\n  }", "lo = 0.0;\n    hi = 0.0;\n  }"),
    ("za_keeps_range", "if (zero_anchor) {  /* no range", "if (0) {  /* no range"),
    ("ll_rank_ties_higher", "return (x->code > y->code) - (x->code < y->code);",
     "return (x->code < y->code) - (x->code > y->code);"),
    ("ll_rank_rare_first",
     "if (x->count != y->count) return (x->count < y->count) - (x->count > y->count);",
     "if (x->count != y->count) return (x->count > y->count) - (x->count < y->count);"),
    ("ll_length_plus_one", "return 2 * floor_log2_u64(v + ((uint64_t)1 << k)) - k + 1;",
     "return 2 * floor_log2_u64(v + ((uint64_t)1 << k)) - k + 2;"),
    ("ll_k_ties_larger", "if (kk == 0 || bits < best) {", "if (kk == 0 || bits <= best) {"),
    ("ll_no_padding", "sub_off[s + 1] = sub_off[s] + (bits + 31) / 32 * 32;",
     "sub_off[s + 1] = sub_off[s] + bits;"),
    ("ll_msb_first", "put_bit(stream, pos++, (uint32_t)(x >> b) & 1u);",
     "put_bit(stream, pos++, (uint32_t)(x >> (nb - 1 - b)) & 1u);"),
    ("ll_group_offset_absolute", "put_u16(stream, sub_off[s] + 16 * g, (uint32_t)(pos - sub_off[s]));",
     "put_u16(stream, sub_off[s] + 16 * g, (uint32_t)pos);"),
    ("ll_no_group_table", "uint64_t bits = ORC_SUB_HEAD_BITS;", "uint64_t bits = 0;"),
    ("ll_group_half_size",
     "uint64_t j0 = s * ORC_SUB + (uint64_t)g * ORC_GROUP;\n      uint64_t j1 = j0 + ORC_GROUP;\n"
     "      j0 = j0 < n ? j0 : n;\n      j1 = j1 < n ? j1 : n;\n      for (uint64_t j = j0; j < j1; j++) {\n"
     "        const uint64_t x",
     "uint64_t j0 = s * ORC_SUB + (uint64_t)g * (ORC_GROUP / 2);\n      uint64_t j1 = j0 + ORC_GROUP;\n"
     "      j0 = j0 < n ? j0 : n;\n      j1 = j1 < n ? j1 : n;\n      for (uint64_t j = j0; j < j1; j++) {\n"
     "        const uint64_t x"),
    ("ll_group_end_unchecked", "if (g + 1 < ORC_GROUPS && pos != gend) return ORC_EINVAL;", ""),
]


def test_mutants_are_listed_uniquely():
    src = open(SRC).read()
    for name, old, _ in MUTANTS:
        assert src.count(old) == 1, name


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read().replace(old, new)
    path = tmp_path / "mutant.c"
    path.write_text(src)
    import shutil
    shutil.copy(os.path.join(os.path.dirname(SRC), "numarck_oracle.h"), tmp_path / "numarck_oracle.h")
    lib = oracle.build(str(path), str(tmp_path / "libmutant.so"))
    o = oracle.Oracle(lib)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError) as e:  # ValueError: status from the library
            failed.append(pin.__name__)
            break
    assert failed, f"mutant {name} survived every pin"
