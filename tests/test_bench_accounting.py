"""Host-side checks of the benchmark's accounting: the algorithmic bytes and
flops per cell that the roofline figure divides by, counted term by term for
the 256x256 beach case (r = 2, 16 x 16 samples, three stored fields, SSP3
stages 2-3 combining 1.5 stored residuals on average), and the refusal of a
multi-GPU run."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_stage_work_per_cell_counted_by_term():
    S, r, nf, m = 16, 2, 3, 1.5
    NP = (r + 1) ** 2
    # words: samples, zeta^n and q^n, H(zeta^n) and the all-wet B vector,
    # m residuals read, the volume residual and the stage state written
    words = S * S + 3 * NP + 2 * NP + nf * NP * m + nf * NP + nf * NP
    # per sample: 5 interpolations and 8 accumulations of r+1 terms each, and
    # 40 pointwise flops; per cell: two dense NP x NP products per field
    flops = S * S * (5 * 2 * (r + 1) + 8 * 2 * (r + 1) + 40) + nf * 2 * NP * NP
    b, f = bench.element_stage_work(S, r, nf, m)
    assert b == 8 * words == 3164.0
    assert f == flops == 30694.0
    # one launch over the 65,536 cells
    assert b * 65536 == 207355904.0 and f * 65536 == 2011561984.0


def test_multi_gpu_request_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "--gpus 1" in p.stderr
    assert p.stdout.strip() == ""


def test_tracer_work_per_cell_counted_by_term():
    S, r, m = 8, 3, 1.5
    NP, NX, NT = 16, 10, 136
    words = S * S + 3 * NP + 2 * NP + NP * m + 2 * NP
    flops = S * S * (2 * 4 + 2 * NX + 2 * 4 * 3 + 2 * 4 * 2) + 2 * S * NT + NP ** 3 / 3 + 2 * NP * NP
    b, f = bench.tracer_stage_work(S, r, m)
    assert b == 8 * words and f == flops


def test_roofline_bound_from_counters():
    # a launch of 100 us moving 220 MB by the counters (0.275 of 8 TB/s) and
    # issuing 33.3 M VALU instructions (0.54 of 1,024 SIMDs x 2.4 GHz / 4)
    c = {"bytes_per_launch": 220e6, "valu_insts_per_launch": 33.3e6}
    roof = bench.roofline(207e6, 2.0e9, 100e-6, c, "k")
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s" and roof["bound_from"] == "counters"
    assert abs(roof["valu_issue_frac"] - 33.3e6 * 4 / (1024 * 2.4e9 * 100e-6)) < 1e-4
    assert abs(roof["frac"] - 20.0 / 78.6) < 1e-4
    # HBM-busy counters give an HBM bound at the algorithmic rate
    roof = bench.roofline(207e6, 2.0e9, 100e-6, {"bytes_per_launch": 700e6, "valu_insts_per_launch": 1e6}, "k")
    assert roof["bound"] == "hbm" and abs(roof["frac"] - 2070.0 / 8000.0) < 1e-4
    # without counters the larger algorithmic fraction decides, and says so
    roof = bench.roofline(207e6, 2.0e9, 100e-6, None, "k")
    assert roof["bound"] == "hbm" and roof["traffic"] is None and "no counter" in roof["bound_from"]


def test_lanes_per_cell():
    assert [bench.lanes_for(S) for S in (3, 5, 8, 9, 16, 17, 32)] == [4, 8, 8, 16, 16, 32, 32]
