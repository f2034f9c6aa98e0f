"""fdemri_waveform_batch (one persistent launch over many waveforms of uneven
sizes) equals separate fdemri_waveform calls bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def batch_members():
    ws = [W.config1(), W.config3(), W.linear_chirp_workload(f0=1e-4, fdot=1e-9, T=1e5, Nf=3001)]
    for prm in W.batch_params(4, 123):
        prm["T"] = min(prm["T"], 0.6 * W.YRSID_SI)
        w = W.batch_workload(prm, K=60 + 10 * len(ws))
        w.f = w.f[: 150_000 + 17 * len(ws)]          # ragged grid sizes
        ws.append(w)
    return ws


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_single_calls(ctx, prec):
    ws = batch_members()
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    outs = ctx.waveform_batch(dws, prec)
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    total = ctx.last_eval_count()
    counts = 0
    for dw, (bp, bc) in zip(dws, outs):
        sp, sc = ctx.waveform_dev(dw, prec)
        torch.cuda.synchronize()
        counts += ctx.last_eval_count()
        assert torch.equal(bp, sp) and torch.equal(bc, sc)
    assert total == counts > 0


def test_batch_repeat_deterministic(ctx):
    ws = batch_members()
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    a = ctx.waveform_batch(dws, "fp64")
    b = ctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    for (ap, ac), (bp, bc) in zip(a, b):
        assert torch.equal(ap, bp) and torch.equal(ac, bc)
