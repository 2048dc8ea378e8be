"""The paper's cold two-stream run (Sec. 5.4: 16^3, L = 2 pi, v0 = 0.3,
131,072 particles, linear shape, 16-point rule, tol 1e-11), first 100 of its
1200 steps, split against unsplit orbit integration on the GPU.

What the paper reports, checked as properties: the Lorenz-gauge and Gauss
residuals stay at roundoff for both variants; with split orbits the
chain-rule residual R_A and the energy drift stay at roundoff; without
splitting both are many orders larger (the paper's unsplit drift reaches
O(1e-5) by T = 30; 4.6e-7 by step 100 here).
"""
import numpy as np
import pytest

from paper_2606_15035_amd import workloads as W

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_2606_15035_amd.ecpic")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    E.lib()


def test_split_conserves_energy_unsplit_drifts():
    from paper_2606_15035_amd import replica
    wl = W.paper_two_stream(100)
    s, _ = replica.run(wl, True, 100, log_every=0)
    u, _ = replica.run(wl, False, 100, log_every=0)
    print(f"split {s}\nunsplit {u}", flush=True)
    for r in (s, u):
        assert r["max_gauge"] < 1e-13 and r["max_gauss"] < 1e-13
        assert r["mean_passes"] <= 8
    assert s["max_abs_drift"] < 1e-13 and s["max_RA_rms"] < 1e-15
    assert s["max_abs_step_defect"] < 1e-14
    assert u["max_abs_drift"] > 1e-8 and u["max_RA_rms"] > 1e-10
    assert u["max_abs_drift"] > 1e5 * s["max_abs_drift"]
