"""fdemri_waveform_noalloc (the entry point that allocates nothing: its
scratch is a fixed device array) against fdemri_waveform, through the C ABI.

Both run the same kernels on the same inputs, so the outputs must be equal
bit for bit (stronger than the rel L2 <= 1e-10 bar of the FP64 path).  Two
calls in a row share the fixed scratch: the second, smaller input must not
see anything of the first.  A request beyond the fixed size is rejected
with FDEMRI_ENOTSUP and leaves the outputs untouched."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_2307_12585_amd")
from gpu_helpers import rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def _both(ctx, dw, prec):
    ref = ctx.waveform_dev(dw, prec)
    ctype = ref[0].dtype
    out = (torch.full((dw.Nf,), 7.0 + 7.0j, dtype=ctype, device=dw.device),
           torch.full((dw.Nf,), 7.0 + 7.0j, dtype=ctype, device=dw.device))
    ctx.waveform_noalloc_dev(dw, out, prec)
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    return [r.cpu().numpy() for r in ref], [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_waveform_on_two_calls(ctx, prec):
    big = W.inspiral_3842_modes()
    small = W.inspiral_20_modes_log_grid()
    for w, what in ((big, "3842 modes"), (small, "20 modes, log grid")):
        dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
        ref, got = _both(ctx, dw, prec)
        for name, g, r in zip(("h+", "hx"), got, ref):
            err = rel_l2(g, r)
            print(f"{what} {prec} {name}: rel L2 against fdemri_waveform {err:.3e}")
            assert np.array_equal(g, r), (what, prec, name, err)


def test_noalloc_rejects_requests_beyond_the_fixed_scratch(ctx):
    K, Nm, Nf = 512, 3843, 64
    dev = ctx.device
    z = lambda n: torch.linspace(0.0, 1.0, n, dtype=torch.float64, device=dev)
    ones = torch.ones(Nm, dtype=torch.int32, device=dev)
    dw = fd.DeviceWaveform(z(K) * 1e6, z(K) * 1e-3, z(K) * 1e-4, z(K), z(K), ones * 2, ones * 2, ones,
                           torch.zeros(Nm, K, 2, dtype=torch.float64, device=dev), 1.0, 0.5, 1e-20,
                           z(Nf) * 1e-2, device=dev)
    hp = torch.full((Nf,), 3.0 + 1.0j, dtype=torch.complex128, device=dev)
    hc = torch.full((Nf,), 3.0 + 1.0j, dtype=torch.complex128, device=dev)
    with pytest.raises(fd.FdemriError) as ei:
        ctx.waveform_noalloc_dev(dw, (hp, hc), "fp64")
    assert ei.value.status == fd.FDEMRI_ENOTSUP
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((hp == 3.0 + 1.0j).all()) and bool((hc == 3.0 + 1.0j).all())
    # the context still works afterwards
    w = W.inspiral_20_modes_log_grid()
    ref, got = _both(ctx, fd.DeviceWaveform.from_workload(w, device=dev), "fp64")
    assert all(np.array_equal(g, r) for g, r in zip(got, ref))
