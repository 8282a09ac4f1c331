"""Batched multi-source, multi-wavelength sensing (40 m class geometry): six
guide stars through a three-layer atmosphere, sensed at 650 and 850 nm by two
plans whose pwfs_measure calls are captured in one HIP graph.  Replays must
equal the same calls launched one by one, bit for bit, on every replay with
eager work in between; the 850 nm plan (modulation radius 9.18 focal pixels)
is checked against the FP64 oracle on one source."""
import numpy as np
import pytest

from synth.configs import CFG3, CFG3_850, ATMO3, CFG3_LAYERS, CFG3_GS_ARCSEC
from synth.screens import layered_opd_nm
import oracle
from tests.gpu_common import torch_cuda, say, check_frame

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_eager_and_oracle_at_850nm():
    from paper_1607_07624_amd.multisource import MultiSourceSensor
    torch = torch_cuda()
    ms = MultiSourceSensor([CFG3, CFG3_850], n_sources=len(CFG3_GS_ARCSEC), autotune=True, reps=2)
    say(f"[gpu] multi-source schedules: {ms.schedules}")
    ms.capture()
    eager = [torch.empty_like(s) for s in ms.slopes]
    opd = None
    for seed in (1, 2, 3):
        opd = torch.from_numpy(layered_opd_nm(CFG3, ATMO3, CFG3_LAYERS, CFG3_GS_ARCSEC, seed=seed)).cuda()
        ms.opd.copy_(opd)
        ms.measure_eager(eager)                      # eager work between replays
        torch.cuda.synchronize()
        ms.measure()
        torch.cuda.synchronize()
        for w, (g, e) in enumerate(zip(ms.slopes, eager)):
            assert torch.equal(g, e), (seed, w)
        say(f"[gpu] multi-source seed {seed}: graph replay == eager for both wavelengths")
    s850 = ms.slopes[1].cpu().numpy()
    o = opd.cpu().numpy()
    orc = oracle.Oracle(CFG3_850)
    _, s_o = orc.measure(o[2].astype(np.float64))
    check_frame("cfg3 850 nm, source 2", s850[2], s_o)
    # the sources differ (layers shift with direction) but share the ground layer
    s650 = ms.slopes[0].cpu().numpy()
    c = np.corrcoef(s650.reshape(len(CFG3_GS_ARCSEC), -1))
    assert 0.0 < c[0, 3] < 0.999
    ms.close()
