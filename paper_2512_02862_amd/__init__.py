"""MI355X-native per-GPU relational hot path (filter, hash partition, hash join,
group-by SUM) behind a C ABI.  See include/pyst.h; the Python binding is
paper_2512_02862_amd.pyst."""
