"""Helpers shared by the GPU tests: run the HIP path through the C ABI on
inputs from the seeded generators, and compare with the oracle."""
import numpy as np
import torch

import paper_2307_12585_amd as fd


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def gpu_waveform(ctx, w, prec="fp64", partners=True, f=None, check_flags=True):
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device, partners=partners, f=f)
    hp, hc = ctx.waveform_dev(dw, prec)
    torch.cuda.synchronize()
    if check_flags:
        assert ctx.sync_flags() == 0, "device flag word set"
    return hp.cpu().numpy(), hc.cpu().numpy()


def support_mismatch(a, b):
    """Bins that are exactly zero on one side and not on the other (a piece
    edge assigned differently)."""
    return int(np.count_nonzero((a == 0) != (b == 0)))
