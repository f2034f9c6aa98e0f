"""fdemri_select_modes (through the C ABI) against the oracle's selection:
identical kept rows, except rows whose power share is within rounding of the
threshold (there the summation order decides)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle.selection import margin, select_modes

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def compare(ctx, A, eps):
    got = ctx.select_modes(torch.as_tensor(A, device=ctx.device), eps).cpu().numpy()
    torch.cuda.synchronize()
    ref = select_modes(A, eps)
    assert np.all(np.diff(got) > 0)  # table order
    diff = np.setxor1d(got, ref)
    if diff.size:
        r = margin(A, eps)[diff]
        assert np.all(np.abs(r - 1) < 1e-12), (diff, r)
    return got, ref


def test_select_3843_mode_table(ctx):
    full = W.inspiral_3842_modes(eps=0.0)
    got, ref = compare(ctx, full.A, 1e-5)
    assert got.size == ref.size == 3842
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("Nm,K", [(1, 1), (1, 4), (257, 4), (5000, 200), (300, 513)])
def test_select_random_tables(ctx, Nm, K):
    rng = np.random.default_rng(Nm + K)
    t = np.linspace(0, 1, K)
    a = rng.lognormal(0, 2.5, Nm) * np.exp(1j * rng.uniform(0, 2 * np.pi, Nm))
    # per-row time variation, so that rows pass at different knots
    g = 1.0 + 0.8 * np.sin(2 * np.pi * (t[None, :] * rng.uniform(0.5, 3, Nm)[:, None] + rng.uniform(0, 1, Nm)[:, None]))
    A = a[:, None] * g
    for eps in (0.0, 1e-6, 1e-3, 0.2):
        compare(ctx, A, eps)


def test_select_deterministic_and_invalid(ctx):
    full = W.inspiral_3842_modes(eps=0.0)
    A = torch.as_tensor(full.A, device=ctx.device)
    a = ctx.select_modes(A, 3e-4)
    b = ctx.select_modes(A, 3e-4)
    assert torch.equal(a, b)
    lib = fd.lib()
    idx = torch.full((4,), -7, dtype=torch.int32, device=ctx.device)
    cnt = torch.full((1,), -7, dtype=torch.int32, device=ctx.device)
    A4 = torch.ones(4, 4, dtype=torch.complex128, device=ctx.device)
    assert lib.fdemri_select_modes(ctx._h, 0, 4, A4.data_ptr(), 1e-3, idx.data_ptr(), cnt.data_ptr(), None) == 1
    assert lib.fdemri_select_modes(ctx._h, 4, 4, A4.data_ptr(), -1.0, idx.data_ptr(), cnt.data_ptr(), None) == 1
    assert lib.fdemri_select_modes(ctx._h, 4, 4, None, 1e-3, idx.data_ptr(), cnt.data_ptr(), None) == 1
    torch.cuda.synchronize()
    assert int(cnt.item()) == -7 and torch.all(idx == -7)
    # no rows: zero kept
    assert lib.fdemri_select_modes(ctx._h, 4, 0, None, 1e-3, None, cnt.data_ptr(), None) == 0
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
