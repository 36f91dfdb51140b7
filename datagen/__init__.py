"""Seeded synthetic input generators for the KPA grouping path.

This package holds only random-number generation and row packing: no step of
the grouping method (extract, partition, sort, reduce, merge, join) is computed
here.  Both the CPU oracle and the GPU path consume the bytes it produces.
"""
from .rows import (  # noqa: F401
    splitmix64, uniform_int, uniform_u64, zipf_ranks, zipf_cdf_table,
    key_table, pack_rows16, pack_rows32, gen_c1, gen_c2, gen_c3, gen_c4_window,
    gen_c4, c4_window_sizes, c4_zipf_s, RowLayout, LAYOUT16, LAYOUT32,
    gen_ysb, ysb_tables, YSB_VIEW, YSB_COLS, LAYOUT_YSB,
)
