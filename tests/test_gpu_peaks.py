"""The device microbenchmarks behind the roofline's measured peaks
(ecpic_measure_peaks): figures between a loose floor and the published
MI355X peaks (FP64 vector 78.6 TFLOP/s, HBM 8 TB/s; 5% allowed above them
for the clock and the rounding of the published figures), and the argument
checks."""
import pytest

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_2606_15035_amd.ecpic")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    E.lib()
    return torch


def test_measured_peaks_lie_below_the_published_ones():
    p = E.measure_peaks(nbytes=2 << 30, repeats=3)
    print(p, flush=True)
    assert 20.0 <= p["fp64_tflops"] <= 78.6 * 1.05
    assert 1000.0 <= p["hbm_GBs"] <= 8000.0 * 1.05


def test_measure_peaks_rejects_small_buffers_and_no_repeats():
    for nbytes, repeats in ((1 << 20, 1), (64 << 20, 0)):
        with pytest.raises(E.EcpicError) as ei:
            E.measure_peaks(nbytes=nbytes, repeats=repeats)
        assert ei.value.status == E.EINVAL
