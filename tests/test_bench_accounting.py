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
