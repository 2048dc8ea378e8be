"""Host logic of bench.py (no GPU): the one-GPU refusal and the operation
counts its roofline uses.

The algorithmic count of the orbit gather + push is the sum, per orbit piece,
of the tensor-product quadrature sums of grad phi-bar (3 s^3 per point), of
D A with A^n and A^{n+1} (3 (2 s^3 + 3 s^2 + 3 s) per point) and of the
weights (s^3 per point), plus the closing 3 s^3, all FMAs; per particle the
end-point interpolant (3 s^3 FMAs) and ~100 flops of breakpoints and push.
The figures below are that count worked out by hand for each degree.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stdout and p.stderr.strip() == ""


@pytest.mark.parametrize("r,per_push,per_piece", [
    # n_q = the smallest Gauss rule exact for degree 3 r (2 n_q - 1 >= 3 r)
    # r = 1: s = 2, n_q = 2: 2 (24 + 3 (16 + 12 + 6) + 8) + 24 = 292 FMAs
    (1, 2 * 24 + 100, 2 * 292),
    # r = 2: s = 3, n_q = 4: 4 (81 + 3 (54 + 27 + 9) + 27) + 81 = 1593 FMAs
    (2, 2 * 81 + 100, 2 * 1593),
    # r = 3: s = 4, n_q = 5: 5 (192 + 3 (128 + 48 + 12) + 64) + 192 = 4292 FMAs
    (3, 2 * 192 + 100, 2 * 4292),
])
def test_algorithmic_flop_count_by_hand(r, per_push, per_piece):
    assert bench.algorithmic_flops_per_push(r, 0.0) == per_push
    assert bench.algorithmic_flops_per_push(r, 1.0) == per_push + per_piece
    assert bench.algorithmic_flops_per_push(r, 1.306) == pytest.approx(per_push + 1.306 * per_piece)


def test_headline_count_at_the_measured_piece_count():
    """4422 flops per particle-push at the 32^3 workload's 1.3056 pieces per
    orbit (r = 2), the figure the measurement notes quote; the kernel's own
    count there is 566 + 1920 per piece."""
    assert round(bench.algorithmic_flops_per_push(2, 1.3056103515625)) == 4422
    assert bench.kernel_flops_per_push(2, 1.0) == pytest.approx(566 + 1920)
    assert bench.kernel_flops_per_push(2, 0.0) == pytest.approx(566)
