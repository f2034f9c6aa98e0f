"""Device-side input checks and allocation failure, through the C ABI.

The host does not read device data, so the conditions of the boundary that
depend on it (t finite and strictly increasing, every trajectory and
amplitude value finite, f finite, >= 0 and ascending, the DFT grid for the
Hann kernel) are checked on the device: a waveform that fails them gets zero
outputs and raises FDEMRI_FLAG_BAD_INPUT.  An allocation failure (injected
with FDEMRI_TEST_FAIL_ALLOC) returns FDEMRI_ENOMEM with nothing enqueued."""
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


def small():
    w = W.inspiral_20_modes()
    w.f = w.f[:60_000]
    return w


def corrupt(dw, what):
    """A copy of the device inputs of dw with one defect."""
    d2 = fd.DeviceWaveform.from_workload(small(), device=dw.device)
    if what == "t repeated":
        d2.t[5] = d2.t[4]
    elif what == "t decreasing":
        d2.t[7] = d2.t[6] - 1.0
    elif what == "t nan":
        d2.t[3] = float("nan")
    elif what == "Fphi inf":
        d2.Fphi[7] = float("inf")
    elif what == "Phir nan":
        d2.Phir[2] = float("nan")
    elif what == "A nan":
        d2.A[3, 10, 0] = float("nan")
    elif what == "f descending":
        d2.f[100], d2.f[99] = d2.f[99].item(), d2.f[100].item()
    elif what == "f negative":
        d2.f[0] = -1e-5
    elif what == "f nan":
        d2.f[50_000] = float("nan")
    return d2


DEFECTS = ["t repeated", "t decreasing", "t nan", "Fphi inf", "Phir nan", "A nan", "f descending", "f negative",
           "f nan"]


@pytest.mark.parametrize("what", DEFECTS)
def test_bad_device_inputs_give_zeros_and_the_flag(ctx, what):
    good = fd.DeviceWaveform.from_workload(small(), device=ctx.device)
    bad = corrupt(good, what)
    for prec in ("fp64", "mixed"):
        hp, hc = ctx.waveform_dev(bad, prec)
        # other bits may come with it (garbage knots can also overflow the piece table)
        assert ctx.sync_flags() & fd.FDEMRI_FLAG_BAD_INPUT, (what, prec)
        assert not bool(hp.abs().sum()) and not bool(hc.abs().sum()), (what, prec)
        # the status is per call: the next, valid call is unaffected
        gp, gc = ctx.waveform_dev(good, prec)
        assert ctx.sync_flags() == 0
        assert bool(gp.abs().sum() > 0)
    g = torch.ones(bad.Nf, dtype=torch.complex128, device=ctx.device)
    out = ctx.vjp_dev(bad, g, g)
    assert ctx.sync_flags() & fd.FDEMRI_FLAG_BAD_INPUT
    for key, v in out.items():
        assert not bool(v.abs().sum()), (what, key)


def test_bad_member_of_a_batch(ctx):
    """Only the member with bad inputs is zero; the others equal single calls."""
    ws = [small(), small(), small()]
    ws[2].f = ws[2].f[:30_000]
    dws = [fd.DeviceWaveform.from_workload(w, device=ctx.device) for w in ws]
    dws[1] = corrupt(dws[1], "t repeated")
    outs = ctx.waveform_batch(dws, "fp64")
    assert ctx.sync_flags() & fd.FDEMRI_FLAG_BAD_INPUT
    assert not bool(outs[1][0].abs().sum()) and not bool(outs[1][1].abs().sum())
    for j in (0, 2):
        sp, sc = ctx.waveform_dev(dws[j], "fp64")
        torch.cuda.synchronize()
        assert torch.equal(sp, outs[j][0]) and torch.equal(sc, outs[j][1])
    assert ctx.sync_flags() == 0


def test_hann_kernel_needs_the_dft_grid(ctx):
    """FDEMRI_LL_HANN on a grid that is not f_k = k f_1 (here: offset by ten
    bins) raises the flag and compares the data with a zero model; on the
    first bins of the DFT grid it is accepted."""
    w = small()
    dev = ctx.device
    rng = np.random.default_rng(3)
    for lo, ok in ((0, True), (10, False)):
        f = w.f[lo:lo + 20_000]
        dw = fd.DeviceWaveform.from_workload(w, device=dev, f=f)
        dp = torch.as_tensor(rng.normal(size=f.size) + 1j * rng.normal(size=f.size), device=dev) * 1e-20
        dc = torch.as_tensor(rng.normal(size=f.size) + 1j * rng.normal(size=f.size), device=dev) * 1e-20
        wS = torch.full((f.size,), 1e38, dtype=torch.float64, device=dev)
        out = ctx.loglike_dev(dw, dp, dc, wS, hann=True).cpu().numpy()
        flags = ctx.sync_flags()
        if ok:
            assert flags == 0 and out[1] > 0
        else:
            assert flags == fd.FDEMRI_FLAG_BAD_INPUT
            ref = -0.5 * float(torch.sum(wS * (dp.abs() ** 2 + dc.abs() ** 2)))
            assert out[1] == 0.0 and out[2] == 0.0
            assert abs(out[0] - ref) <= 1e-12 * abs(ref)
        # without the Hann kernel any ascending grid is accepted
        ctx.loglike_dev(dw, dp, dc, wS, hann=False)
        assert ctx.sync_flags() == 0


def test_allocation_failure_leaves_outputs_and_context_usable(monkeypatch):
    monkeypatch.setenv("FDEMRI_TEST_FAIL_ALLOC", "1")
    c = fd.Context(0)
    monkeypatch.delenv("FDEMRI_TEST_FAIL_ALLOC")
    dw = fd.DeviceWaveform.from_workload(small(), device=c.device)
    hp = torch.full((dw.Nf,), 5.0 + 5.0j, dtype=torch.complex128, device=c.device)
    hc = torch.full((dw.Nf,), 5.0 + 5.0j, dtype=torch.complex128, device=c.device)
    with pytest.raises(fd.FdemriError) as ei:
        c.waveform_dev(dw, "fp64", out=(hp, hc))
    assert ei.value.status == fd.FDEMRI_ENOMEM
    torch.cuda.synchronize()
    assert bool((hp == 5.0 + 5.0j).all()) and bool((hc == 5.0 + 5.0j).all())
    # the hook fires once: the next call allocates and equals a normal context's result
    c.waveform_dev(dw, "fp64", out=(hp, hc))
    ref = fd.Context(0)
    rp, rc = ref.waveform_dev(dw, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(hp, rp) and torch.equal(hc, rc)
    ref.close()
    c.close()
