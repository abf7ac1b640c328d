"""Host side of the Sec. 4 evaluation report (no GPU): the paper's Table 1
ratios (tests/golden/table1_time_ratios.json, Sec. 4) are read and printed
beside the measured ratios of the same grid and scheme."""
import json
import os

from paper_1712_05145_amd import evaluation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_time_ratios.json")


def test_table1_fixture_read_as_printed():
    t = evaluation.paper_table1(GOLDEN)
    raw = json.load(open(GOLDEN))
    assert raw["n"] == [8, 16, 32, 64, 128, 256, 512, 1024]
    # two printed entries of Table 1, Sec. 4
    assert t[(64, "basic")] == 23.7463 and t[(1024, "cg")] == 4.8484
    # the CG version of the paper is the BiCGSTAB routine: same column
    assert all(t[(n, "bicgstab")] == t[(n, "cg")] for n in raw["n"])


def test_report_prints_paper_ratio_beside_measured(tmp_path):
    row = {"n": 64, "scheme": "cg", "first": {"iters": 12, "seconds": 0.01},
           "second": {"iters": 15, "seconds": 0.045}, "ratio": 4.5}
    out = tmp_path / "eval.md"
    evaluation.write_markdown(str(out), [row], [], "cmd")
    txt = out.read_text()
    line = [l for l in txt.splitlines() if l.startswith("| 64 | CG |")][0]
    assert line.rstrip().endswith("| 4.500 | 4.7257 |")
