"""The autotuner's table writer emits entries in the field order of the
library's Tuning struct."""
import os
import re

from paper_2012_13548_amd.autotune import write_table

ROW = re.compile(r"^\{(\d+), ([\d.]+), ([\d.]+), (\d+), (\d+), ([12]), ([01]), (\d+), "
                 r"([\d.]+), ([\d.]+), (\d+), (-?[\d.]+)\},$")


def test_table_format(tmp_path):
    entries = [dict(scale=26, alpha=28, beta=24, lane_scan=4, bu_blocks_per_cu=8, vertices_per_lane=2,
                    packed=1, lds_kb=140, lds_density=0.3, batch_alpha=14, batch_blocks_per_cu=8,
                    gamma=1.4),
               dict(scale=20, alpha=14.5, beta=96, lane_scan=2, bu_blocks_per_cu=16,
                    vertices_per_lane=1, packed=0, lds_kb=64, lds_density=0.03, batch_alpha=8,
                    batch_blocks_per_cu=4)]
    p = tmp_path / "t.inc"
    write_table(entries, p)
    rows = [l for l in p.read_text().splitlines() if not l.startswith("//")]
    parsed = [ROW.match(r).groups() for r in rows]
    assert [int(x[0]) for x in parsed] == [20, 26]
    assert parsed[0] == ("20", "14.5", "96.0", "2", "16", "1", "0", "64", "0.03", "8.0", "4",
                         "0.00")
    assert parsed[1][-1] == "1.40"


def test_shipped_table_parses():
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(here, "paper_2012_13548_amd", "csrc", "tuned_table.inc")).read()
    rows = [l for l in text.splitlines() if l and not l.startswith("//")]
    assert rows and all(ROW.match(r) for r in rows)
