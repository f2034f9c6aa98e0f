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
    ws = [W.inspiral_20_modes(), W.inspiral_20_modes_log_grid(), W.linear_chirp_workload(f0=1e-4, fdot=1e-9, T=1e5, Nf=3001)]
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


def test_batch_with_maximum_knot_counts(ctx):
    """Members with K = 512 (FDEMRI_MAX_KNOTS) and 257 beside a small one: the
    batched spline, piece and gather kernels at their largest tables equal
    single calls."""
    ws = [W.inspiral_20_modes(K=512), W.inspiral_20_modes(K=257), W.inspiral_20_modes(K=40)]
    for w in ws:
        w.f = w.f[:200_000]
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    for prec in ("fp64", "mixed"):
        outs = ctx.waveform_batch(dws, prec)
        torch.cuda.synchronize()
        assert ctx.sync_flags() == 0
        for dw, (bp, bc) in zip(dws, outs):
            sp, sc = ctx.waveform_dev(dw, prec)
            torch.cuda.synchronize()
            assert torch.equal(bp, sp) and torch.equal(bc, sc)


def test_batch_repeat_deterministic(ctx):
    ws = batch_members()
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    a = ctx.waveform_batch(dws, "fp64")
    b = ctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    for (ap, ac), (bp, bc) in zip(a, b):
        assert torch.equal(ap, bp) and torch.equal(ac, bc)


def test_batch_graph_replays_match_eager(ctx):
    """A captured batch replayed several times, with eager work and
    synchronisations in between, equals the eager batch every time."""
    ws = batch_members()
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    ref = ctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    gctx = fd.Context(0, graphs=True)
    outs = [(torch.empty_like(a), torch.empty_like(b)) for a, b in ref]
    x = torch.randn(512, 512, device=ctx.device)
    for rep in range(4):
        for o in outs:
            o[0].fill_(float("nan"))
            o[1].fill_(float("nan"))
        gctx.waveform_batch(dws, "fp64", outs=outs)
        y = x @ x                      # unrelated eager work on the same stream
        ctx.waveform_dev(dws[0], "fp64")
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        for (gp, gc), (rp, rc) in zip(outs, ref):
            assert torch.equal(gp, rp) and torch.equal(gc, rc), rep
    assert gctx.last_eval_count() > 0
    gctx.close()


def test_batch_graph_follows_changed_angles_and_scale(ctx):
    """The graph of a batch is keyed on its pointers and shapes only: new
    viewing angles and scales (same buffers) are written into the records the
    replay reads, so every replay equals the eager batch at the new values;
    more distinct buffers than the graph cache holds evict the least recently
    used graph, which is captured again when it comes back."""
    ws = batch_members()[:5]
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    gctx = fd.Context(0, graphs=True)
    outs = [(torch.empty(d.Nf, dtype=torch.complex128, device=ctx.device),
             torch.empty(d.Nf, dtype=torch.complex128, device=ctx.device)) for d in dws]
    rng = np.random.default_rng(5)
    for rep in range(10):
        for d in dws:
            d.theta, d.phi, d.scale = float(rng.uniform(0.1, 3.0)), float(rng.uniform(0, 6.2)), float(rng.uniform(0.5, 2.0)) * 1e-20
        gctx.waveform_batch(dws, "fp64", outs=outs)
        ref = ctx.waveform_batch(dws, "fp64")
        torch.cuda.synchronize()
        for (gp, gc), (rp, rc) in zip(outs, ref):
            assert torch.equal(gp, rp) and torch.equal(gc, rc), rep
    # 10 distinct output sets (10 graph keys) against a cache of 8, then the first again
    sets = [[(torch.empty(d.Nf, dtype=torch.complex128, device=ctx.device),
              torch.empty(d.Nf, dtype=torch.complex128, device=ctx.device)) for d in dws[:2]] for _ in range(10)]
    ref = ctx.waveform_batch(dws[:2], "fp64")
    for o in sets + sets[:1]:
        gctx.waveform_batch(dws[:2], "fp64", outs=o)
    torch.cuda.synchronize()
    for o in sets:
        for (gp, gc), (rp, rc) in zip(o, ref):
            assert torch.equal(gp, rp) and torch.equal(gc, rc)
    gctx.close()


def test_autotune_choice_and_invariance(ctx, tmp_path, monkeypatch):
    """The autotuner picks one of the tile sizes, records it in the cache
    file, and results do not depend on the tile size."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FDEMRI_TUNE_CACHE", str(cache))
    ws = batch_members()[:4]
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    before = ctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    tctx = fd.Context(0)
    bpl = tctx.autotune(dws, "fp64")
    assert bpl in (1, 2, 4)
    after = tctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    for (a, b), (c, d) in zip(before, after):
        assert torch.equal(a, c) and torch.equal(b, d)
    lines = cache.read_text().split("\n")
    assert any(line.endswith(f" {bpl}") for line in lines if line)
    tctx.close()
    # a new context reads the cache back
    c2 = fd.Context(0)
    again = c2.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    assert all(torch.equal(a, c) for (a, _), (c, _) in zip(before, again))
    c2.close()
