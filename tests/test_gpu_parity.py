"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 bar: relative L2 <= 1e-10 per polarization (the target of the mode sum
in FP64).  Mixed bar: relative L2 <= 1e-6 against the GPU FP64 result.
Bins in or out of a voice's frequency range must agree exactly."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.waveform import Voice, splines, waveform_voices, count_evals
from oracle.harmonics import swsh

pytestmark = pytest.mark.gpu

fd = pytest.importorskip("paper_2307_12585_amd")
from gpu_helpers import gpu_waveform, rel_l2, support_mismatch  # noqa: E402

TOL64 = 1e-10
TOLMIX = 1e-6


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def _check64(hg, ho, what):
    for name, g, o in zip(("h+", "hx"), hg, ho):
        err = rel_l2(g, o)
        print(f"{what} {name}: rel L2 {err:.3e}, support mismatch {support_mismatch(g, o)}")
        assert support_mismatch(g, o) == 0, what
        assert err <= TOL64, (what, name, err)


def test_20_modes_full_grid(ctx):
    w = W.inspiral_20_modes()
    hg = gpu_waveform(ctx, w)
    ho = oracle.waveform(w)
    _check64(hg, ho, "inspiral_20_modes")
    assert ctx.last_eval_count() == count_evals(w) == 8724


def test_20_modes_log_grid(ctx):
    w = W.inspiral_20_modes_log_grid()
    _check64(gpu_waveform(ctx, w), oracle.waveform(w), "inspiral_20_modes_log_grid")


def test_20_modes_ragged_and_offset_grids(ctx):
    w = W.inspiral_20_modes()
    for lo, hi in [(0, 1), (0, 255), (3, 1000), (12345, 12345 + 777), (100001, 100001 + 65 * 64 + 3)]:
        f = w.f[lo:hi]
        hg = gpu_waveform(ctx, w, f=f)
        ho = oracle.waveform(w, f=f)
        for g, o in zip(hg, ho):
            assert support_mismatch(g, o) == 0
            if np.any(o != 0):
                assert rel_l2(g, o) <= TOL64


def test_3842_modes_sampled_bins(ctx):
    """The full-size 3842-mode waveform on the GPU; the oracle evaluates a sample of bins
    (each bin is independent) drawn across the active band and the tail."""
    w = W.inspiral_3842_modes()
    hp, hc = gpu_waveform(ctx, w)
    rng = np.random.default_rng(11)
    act = np.nonzero(w.f < 9e-3)[0]
    idx = np.unique(np.concatenate([rng.choice(act, 1500, replace=False),
                                    rng.choice(w.Nf, 200, replace=False), [0, 1, w.Nf - 1]]))
    op, oc = oracle.waveform(w, f=w.f[idx])
    _check64((hp[idx], hc[idx]), (op, oc), "inspiral_3842_modes-sampled")
    assert np.all(hp[w.f > 1.2e-2] == 0)


@pytest.mark.parametrize("K", [129, 257, 512])
def test_knot_counts_up_to_the_maximum(ctx, K):
    """Knot counts past each block-size step of the spline and set-up kernels,
    up to FDEMRI_MAX_KNOTS (the largest trajectory tables the gather stages in
    LDS): FP64 against the oracle, mixed against FP64."""
    w = W.inspiral_20_modes(K=K)
    h64 = gpu_waveform(ctx, w)
    _check64(h64, oracle.waveform(w), f"inspiral_20_modes K={K}")
    hm = gpu_waveform(ctx, w, prec="mixed")
    for g, o in zip(hm, h64):
        assert rel_l2(g.astype(np.complex128), o) <= TOLMIX


def _replicas(w, sel, reps, seed, real=False):
    """The rows `sel` of w repeated reps times, copy r of row j with amplitude
    A_j c_rj (seeded factors, complex unless real); returns the new workload
    and c."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.5, 1.5, (reps, sel.size))
    if not real:
        c = c * np.exp(1j * rng.uniform(0, 2 * np.pi, (reps, sel.size)))
    r = W.inspiral_20_modes()
    r.l, r.m, r.n = (np.tile(x[sel], reps) for x in (w.l, w.m, w.n))
    r.A = (w.A[sel][None, :, :] * c[:, :, None]).reshape(-1, w.K)
    return r, c


def test_active_list_in_windows(ctx):
    """520 rows of one voice, active in the same bins: one voice group of 520
    members (more than the 512-entry active list of a workgroup would hold as
    single rows)."""
    w = W.inspiral_20_modes()
    r, _ = _replicas(w, np.array([8]), 520, 5)
    ho = oracle.waveform(r)
    act = np.nonzero(ho[0])[0]
    assert act.size > 256
    f_idx = np.arange(max(act.min() - 70, 0), act.max() + 70)
    hg = gpu_waveform(ctx, r, f=r.f[f_idx])
    _check64(hg, tuple(x[f_idx] for x in ho), "520 replicas of one voice")


def test_mode_table_scanned_in_rounds(ctx):
    """4200 table rows (more than one scan round of 4096 rows per workgroup):
    the sum equals the combination of the 20 single-row GPU waveforms with the
    rows' factors.  The factors are real: a row's partner voice carries the
    conjugate amplitude, so the waveform is linear in A over the reals only."""
    w = W.inspiral_20_modes()
    w.f = w.f[:70_000]
    sel = np.arange(20)
    r, c = _replicas(w, sel, 210, 6, real=True)
    r.f = w.f
    hg = gpu_waveform(ctx, r)
    ref = [np.zeros(w.Nf, complex), np.zeros(w.Nf, complex)]
    for j in sel:
        one = W.inspiral_20_modes()
        one.l, one.m, one.n, one.A, one.f = w.l[j:j + 1], w.m[j:j + 1], w.n[j:j + 1], w.A[j:j + 1], w.f
        hj = gpu_waveform(ctx, one)
        for q in range(2):
            ref[q] += np.sum(c[:, j]) * hj[q]
    for q in range(2):
        assert support_mismatch(hg[q], ref[q]) == 0
        assert rel_l2(hg[q], ref[q]) <= 1e-12


def test_more_rows_than_groups_hold(ctx):
    """4200 rows (more than the 4096 that are sorted into voice groups, so
    each row is solved on its own) active in the same bins: the workgroups'
    active lists take more than 512 entries and are walked window by window.
    The sum equals the single row's GPU waveform times the sum of the (real)
    factors."""
    w = W.inspiral_20_modes()
    w.f = w.f[:70_000]
    r, c = _replicas(w, np.array([8]), 4200, 7, real=True)
    r.f = w.f
    hg = gpu_waveform(ctx, r)
    one = W.inspiral_20_modes()
    one.l, one.m, one.n, one.A, one.f = w.l[8:9], w.m[8:9], w.n[8:9], w.A[8:9], w.f
    h1 = gpu_waveform(ctx, one)
    assert np.count_nonzero(h1[0]) > 256
    for q in range(2):
        ref = np.sum(c) * h1[q]
        assert support_mismatch(hg[q], ref) == 0
        assert rel_l2(hg[q], ref) <= 1e-12


def _rows(w, idx, n_shift=0):
    import copy
    r = copy.copy(w)
    r.l, r.m, r.n, r.A = w.l[idx], w.m[idx], w.n[idx] + n_shift, w.A[idx]
    return r


def test_3842_modes_more_knots_sampled_bins(ctx):
    """The 3842-mode table on a 300-knot trajectory: the set-up's workgroups
    have 512 threads (the voice groups' sort among them); FP64 against the
    oracle on sampled bins."""
    w = W.inspiral_3842_modes(K=300)
    hp, hc = gpu_waveform(ctx, w)
    rng = np.random.default_rng(13)
    act = np.nonzero(w.f < 9e-3)[0]
    idx = np.unique(np.concatenate([rng.choice(act, 600, replace=False), [0, 1, w.Nf - 1]]))
    op, oc = oracle.waveform(w, f=w.f[idx])
    _check64((hp[idx], hc[idx]), (op, oc), "inspiral_3842_modes K=300, sampled")


@pytest.mark.parametrize("K", [200, 300])
def test_voice_groups_row_order(ctx, K):
    """Rows with the same (m, n) share one root per bin (voice groups, set up
    by a sort whose workgroup size follows the knot count): a permutation of
    the rows changes only the order of the sum, within rounding, FP64 and
    mixed."""
    w = W.inspiral_3842_modes(K=K)
    assert 256 < w.Nm <= 4096
    perm = np.random.default_rng(21).permutation(w.Nm)
    wp = _rows(w, perm)
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-6)):
        h0 = gpu_waveform(ctx, w, prec=prec)
        h1 = gpu_waveform(ctx, wp, prec=prec)
        for a, b in zip(h0, h1):
            assert support_mismatch(a, b) == 0
            err = rel_l2(b.astype(np.complex128), a.astype(np.complex128))
            print(f"K={K} {prec}: rel L2 {err:.3e}")
            assert err <= tol


def test_group_eval_count(ctx):
    """fdemri_last_group_eval_count counts the (piece, bin) pairs of one row
    per distinct (m, n): the oracle's count over those rows; the row count
    stays the oracle's count over all rows."""
    w = W.inspiral_3842_modes()
    f = w.f[::97]
    gpu_waveform(ctx, w, f=f)
    ev, gev = ctx.last_eval_count(), ctx.last_group_eval_count()
    _, first = np.unique(np.stack([w.m, w.n], 1), axis=0, return_index=True)
    assert ev == count_evals(w, f)
    assert gev == count_evals(_rows(w, np.sort(first)), f)
    assert gev < ev / 4
    small = W.inspiral_20_modes()
    gpu_waveform(ctx, small)
    assert ctx.last_group_eval_count() == ctx.last_eval_count() == 8724


def test_voice_groups_with_rejected_and_lone_rows(ctx):
    """Rejected rows (l above FDEMRI_MAX_L, |m| > l, m < 0 without
    FDEMRI_NO_PARTNERS) that share (m, n) with valid rows join no group: the
    sum is bitwise the one without them.  Rows whose n lies outside the group
    key's field (n +- 4096 of a valid row) are solved on their own: the sum is
    the valid table's plus their single-row waveforms."""
    w = W.inspiral_3842_modes()
    h0 = gpu_waveform(ctx, w)
    j = [5, 400, 2000]
    bad_l = np.array([50, 2, 3], dtype=w.l.dtype)
    bad_m = np.array([w.m[5], 3, -2], dtype=w.m.dtype)
    bad_n = np.array([w.n[5], 0, 0], dtype=w.n.dtype)
    ins = [100, 1500, w.Nm]
    wb = _rows(w, np.arange(w.Nm))
    wb.l = np.insert(w.l, ins, bad_l)
    wb.m = np.insert(w.m, ins, bad_m)
    wb.n = np.insert(w.n, ins, bad_n)
    wb.A = np.insert(w.A, ins, w.A[j], axis=0)
    hb = gpu_waveform(ctx, wb, check_flags=False)
    assert ctx.sync_flags() == fd.FDEMRI_FLAG_BAD_MODE
    assert np.array_equal(hb[0], h0[0]) and np.array_equal(hb[1], h0[1])
    lone = np.array([7, 900, 3000])
    wl = _rows(w, np.concatenate([np.arange(w.Nm), lone, lone]))
    wl.n = np.concatenate([w.n, w.n[lone] + 4096, w.n[lone] - 4096]).astype(w.n.dtype)
    hl = gpu_waveform(ctx, wl)
    ref = [h0[0].copy(), h0[1].copy()]
    for shift in (4096, -4096):
        for i in lone:
            hi = gpu_waveform(ctx, _rows(w, np.array([i]), shift))
            ref[0] += hi[0]
            ref[1] += hi[1]
    for g, o in zip(hl, ref):
        assert support_mismatch(g, o) == 0
        assert rel_l2(g, o) <= 1e-13


def test_dense_batch_draw_sampled_bins(ctx):
    """A dense draw of the batch distribution (M = 1.9e5, 3835 modes, 6.1e6
    bins, about 1600 evaluations per bin): the first Halley step is rejected
    on almost every lane there, the segment walk and the longer asymptotic
    tiers of the special function are common.  FP64 against the oracle on
    sampled bins; mixed against FP64 on the whole grid."""
    w = W.batch_workload(W.batch_params(8, 4)[3])
    assert w.Nm == 3835 and w.Nf == 6082894
    hp, hc = gpu_waveform(ctx, w)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([rng.choice(np.arange(1, w.Nf), 120, replace=False), [0, 1, w.Nf - 1]]))
    op, oc = oracle.waveform(w, f=w.f[idx])
    _check64((hp[idx], hc[idx]), (op, oc), "dense batch draw, sampled")
    mp, mc = gpu_waveform(ctx, w, prec="mixed")
    for g, o in ((mp, hp), (mc, hc)):
        assert rel_l2(g.astype(np.complex128), o) <= TOLMIX


def test_linear_chirp_and_turnover(ctx):
    from test_oracle_waveform import turnover_workload
    for w in [W.linear_chirp_workload(f0=1e-4, fdot=1e-9, T=1e5, Nf=3001),
              W.linear_chirp_workload(f0=2e-4, fdot=-1e-9, T=1e5, Nf=3001),
              turnover_workload(1e-2, 1e-9), turnover_workload(6e-2, -1e-9),
              turnover_workload(1e-2, 1e-9, K=40), turnover_workload(6e-2, -1e-9, K=40)]:
        _check64(gpu_waveform(ctx, w, partners=False), oracle.waveform(w, partners=False), "chirp/turnover")
        _check64(gpu_waveform(ctx, w, partners=True), oracle.waveform(w, partners=True), "chirp/turnover+partner")


@pytest.mark.parametrize("fdot", [1e-9, -1e-9])
@pytest.mark.parametrize("at_knot", [False, True])
def test_zero_crossing_chirp(ctx, fdot, at_knot):
    """A voice whose frequency passes through zero (between knots, or exactly
    on a knot): the F_V < 0 piece feeds h(-f).  Against the oracle (itself
    pinned to the exact Fresnel transforms on both sides), with and without
    the partner voice, FP64 and mixed."""
    from test_oracle_waveform import zero_crossing_workload
    w, _ = zero_crossing_workload(fdot, at_knot)
    for partners in (False, True):
        ho = oracle.waveform(w, partners=partners)
        assert all(np.count_nonzero(x) > 1000 for x in ho)
        hg = gpu_waveform(ctx, w, partners=partners)
        _check64(hg, ho, f"zero crossing fdot={fdot} at_knot={at_knot} partners={partners}")
        hm = gpu_waveform(ctx, w, prec="mixed", partners=partners)
        for g, o in zip(hm, hg):
            assert rel_l2(g.astype(np.complex128), o) <= TOLMIX


def test_3842_modes_zero_crossing_and_turnover_rows(ctx):
    """The rows of the 3842-mode workload whose voice frequency crosses zero
    (3 rows, (l,8,-11)) or turns over (15 rows) on their own, on every bin of
    the full grid where any of them is active: element-wise against the
    oracle."""
    w = W.inspiral_3842_modes()
    FV = w.m[:, None] * w.traj.Fphi[None, :] + w.n[:, None] * w.traj.Fr[None, :]
    zc = np.nonzero((FV.min(1) < 0) & (FV.max(1) > 0))[0]
    dF = np.diff(FV, axis=1)
    to = np.nonzero((dF.min(1) < 0) & (dF.max(1) > 0))[0]
    assert zc.size == 3 and to.size == 15
    sel = np.concatenate([zc, to])
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    w.f = w.f[: int(np.searchsorted(w.f, 1.05 * np.abs(FV[sel]).max()))]
    ho = oracle.waveform(w)
    hg = gpu_waveform(ctx, w)
    _check64(hg, ho, "3842-mode workload: zero-crossing and turnover rows")
    assert ctx.last_eval_count() == count_evals(w)


def test_explicit_voices_no_partners(ctx):
    """FDEMRI_NO_PARTNERS with rows of both signs of m equals the oracle's
    explicit voice list."""
    w = W.inspiral_20_modes()
    w.m = np.where(np.arange(w.Nm) % 2 == 0, w.m, -w.m).astype(np.int32)
    f = w.f[::3]
    hg = gpu_waveform(ctx, w, partners=False, f=f)
    sp = splines(w.traj, w.A)
    vs = [Voice(int(m), int(n), mu, False, w.scale * complex(swsh(-2, int(l), int(m), w.theta, w.phi)))
          for mu, (l, m, n) in enumerate(zip(w.l, w.m, w.n))]
    ho = waveform_voices(w.traj, sp, vs, f)
    _check64(hg, ho, "no-partners")


def test_mixed_precision_against_fp64(ctx):
    for w in [W.inspiral_20_modes(), W.inspiral_3842_modes()]:
        h64 = gpu_waveform(ctx, w, "fp64")
        hmx = gpu_waveform(ctx, w, "mixed")
        for g, o in zip(hmx, h64):
            err = rel_l2(g.astype(np.complex128), o)
            print(f"mixed vs fp64 {w.meta['name']}: {err:.3e}")
            assert err <= TOLMIX


def test_deterministic_bitwise(ctx):
    w = W.inspiral_20_modes()
    a = gpu_waveform(ctx, w)
    b = gpu_waveform(ctx, w)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_workspace_growth_between_queued_calls():
    """A context whose workspace grows while the kernels of earlier calls are
    still queued on the stream (no synchronisation between the calls): the
    old workspace is retired behind an event, not freed under them, and every
    result equals the same call on a fresh context."""
    small = W.inspiral_20_modes()
    large = W.inspiral_3842_modes()
    large.f = large.f[:400_000]
    c = fd.Context(0)
    try:
        ds = fd.DeviceWaveform.from_workload(small, device=c.device)
        dl = fd.DeviceWaveform.from_workload(large, device=c.device)
        a = c.waveform_dev(ds, "fp64")
        b = c.waveform_dev(dl, "fp64")   # grows the workspace behind the queued small call
        a2 = c.waveform_dev(ds, "mixed")
        b2 = c.waveform_dev(dl, "mixed")
        torch.cuda.synchronize()
        got = [x.cpu().numpy() for x in (*a, *b, *a2, *b2)]
    finally:
        c.close()
    ref = []
    for dw_, prec in ((ds, "fp64"), (dl, "fp64"), (ds, "mixed"), (dl, "mixed")):
        f = fd.Context(0)
        try:
            ref += [x.cpu().numpy() for x in f.waveform_dev(dw_, prec)]
            torch.cuda.synchronize()
        finally:
            f.close()
    assert all(np.array_equal(x, y) for x, y in zip(got, ref))


def test_outputs_fully_overwritten(ctx):
    w = W.inspiral_20_modes()
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    hp = torch.full((dw.Nf,), complex(float("nan"), float("nan")), dtype=torch.complex128, device=ctx.device)
    hc = hp.clone()
    ctx.waveform_dev(dw, "fp64", out=(hp, hc))
    torch.cuda.synchronize()
    assert not torch.isnan(torch.view_as_real(hp)).any() and not torch.isnan(torch.view_as_real(hc)).any()
    assert hp[0] == 0


def test_degenerate_inputs(ctx):
    w = W.inspiral_20_modes()
    # all frequencies outside every voice
    f = np.linspace(0.2, 0.3, 1000)
    hp, hc = gpu_waveform(ctx, w, f=f)
    assert np.all(hp == 0) and np.all(hc == 0)
    # only the DC bin
    hp, hc = gpu_waveform(ctx, w, f=np.zeros(1))
    assert hp[0] == 0 and hc[0] == 0
    # minimal trajectory (K = 4) and an (l,0,0) mode with F = 0
    w4 = W.inspiral_20_modes(K=4)
    w4.l = np.array([2, 3], np.int32)
    w4.m = np.array([2, 0], np.int32)
    w4.n = np.array([1, 0], np.int32)
    w4.A = w4.A[:2]
    f = w4.f[::5]
    _check64(gpu_waveform(ctx, w4, f=f), oracle.waveform(w4, f=f), "K=4")


def test_invalid_arguments_leave_outputs(ctx):
    w = W.inspiral_20_modes()
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    hp = torch.full((dw.Nf,), 7 + 7j, dtype=torch.complex128, device=ctx.device)
    hc = hp.clone()
    d = dw.desc()
    d.K = 3
    import ctypes
    st = ctx._lib.fdemri_waveform(ctx._h, ctypes.byref(d), 0, fd._ptr(hp), fd._ptr(hc), fd._stream(ctx.device))
    assert st == fd.FDEMRI_EINVAL
    assert b"K=3" in ctx._lib.fdemri_last_error(ctx._h)
    torch.cuda.synchronize()
    assert torch.all(hp == 7 + 7j)


def _amplitude_coefficients(w):
    """Not-a-knot spline coefficients of every amplitude series, [Nm, K-1, 4, 2]
    in ascending powers of t - t_i (SciPy, on the test side)."""
    from scipy.interpolate import CubicSpline
    t = w.traj.t
    coef = np.empty((w.A.shape[0], t.size - 1, 4, 2))
    for mu in range(w.A.shape[0]):
        for part, comp in ((0, w.A[mu].real), (1, w.A[mu].imag)):
            coef[mu, :, :, part] = CubicSpline(t, comp, bc_type="not-a-knot").c[::-1].T
    return coef


def test_amplitude_coefficients_given(ctx):
    """FDEMRI_COEFFS_GIVEN: the amplitude splines passed as coefficients give
    the oracle's waveform (which splines the same knots), and the coefficient
    gradient of the adjoint does not depend on how the coefficients arrived;
    amplitude knot gradients are refused."""
    w = W.inspiral_20_modes()
    tr = w.traj
    coef = _amplitude_coefficients(w)
    dwc = fd.DeviceWaveform(tr.t, tr.Fphi, tr.Fr, tr.Phiphi, tr.Phir, w.l, w.m, w.n, coef, w.theta, w.phi,
                            w.scale, w.f, device=ctx.device, coeffs_given=True)
    dwk = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    hp, hc = ctx.waveform_dev(dwc, "fp64")
    kp, kc = ctx.waveform_dev(dwk, "fp64")
    torch.cuda.synchronize()
    hg = (hp.cpu().numpy(), hc.cpu().numpy())
    _check64(hg, oracle.waveform(w), "coefficients given")
    for a, b in zip(hg, (kp.cpu().numpy(), kc.cpu().numpy())):
        assert rel_l2(a, b) <= 1e-12
    mp, mc = ctx.waveform_dev(dwc, "mixed")
    torch.cuda.synchronize()
    for a, b in zip((mp.cpu().numpy(), mc.cpu().numpy()), hg):
        assert rel_l2(a.astype(np.complex128), b) <= TOLMIX
    rng = np.random.default_rng(3)
    g = [torch.as_tensor(rng.standard_normal(w.f.size) + 1j * rng.standard_normal(w.f.size), device=ctx.device)
         for _ in range(2)]
    gc = ctx.vjp_dev(dwc, g[0], g[1], "fp64")
    gk = ctx.vjp_dev(dwk, g[0], g[1], "fp64")
    assert "gA_knots" not in gc
    for key in ("gA", "gPhi", "gPhi_knots", "g_scalars"):
        a, b = gc[key].cpu().numpy(), gk[key].cpu().numpy()
        assert rel_l2(a, b) <= 1e-11, key
    d = dwc.desc()
    import ctypes
    buf = torch.empty(w.Nm * tr.t.size * 2, dtype=torch.float64, device=ctx.device)
    st = ctx._lib.fdemri_vjp(ctx._h, ctypes.byref(d), 0, ctypes.c_void_p(g[0].data_ptr()),
                             ctypes.c_void_p(g[1].data_ptr()), None, None, ctypes.c_void_p(buf.data_ptr()), None,
                             ctypes.c_void_p(buf.data_ptr()), None)
    assert st == 1  # FDEMRI_EINVAL: no amplitude knots to differentiate


def test_voice_groups_against_rows_on_every_bin(ctx):
    """The grouped sum (one root per (m, n), combined amplitude splines) of
    the 3842-mode table against the same table evaluated row by row (caller-
    given coefficients, which are never grouped) on all 3 155 816 bins: FP64
    within rounding, with the same support; and the group count below the
    row count only on the grouped call."""
    w = W.inspiral_3842_modes()
    tr = w.traj
    coef = _amplitude_coefficients(w)
    dwc = fd.DeviceWaveform(tr.t, tr.Fphi, tr.Fr, tr.Phiphi, tr.Phir, w.l, w.m, w.n, coef, w.theta, w.phi,
                            w.scale, w.f, device=ctx.device, coeffs_given=True)
    dwk = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    rp, rc = ctx.waveform_dev(dwc, "fp64")
    torch.cuda.synchronize()
    assert ctx.last_group_eval_count() == ctx.last_eval_count()
    gp, gc = ctx.waveform_dev(dwk, "fp64")
    torch.cuda.synchronize()
    assert ctx.last_group_eval_count() < ctx.last_eval_count()
    for g, r in ((gp, rp), (gc, rc)):
        g, r = g.cpu().numpy(), r.cpu().numpy()
        assert support_mismatch(g, r) == 0
        err = rel_l2(g, r)
        print(f"grouped vs rows: rel L2 {err:.3e}")
        assert err <= 1e-12


def test_out_of_range_mode_rows_are_flagged_and_skipped(ctx):
    """Rows with l above FDEMRI_MAX_L or |m| > l contribute nothing, set
    FDEMRI_FLAG_BAD_MODE, and leave the other rows' sum unchanged; the
    adjoint stays finite."""
    w = W.inspiral_20_modes()
    hp0, hc0 = gpu_waveform(ctx, w)
    import copy
    wb = copy.deepcopy(w)
    wb.l = np.concatenate([w.l, [50, 2]]).astype(w.l.dtype)
    wb.m = np.concatenate([w.m, [2, 3]]).astype(w.m.dtype)
    wb.n = np.concatenate([w.n, [0, 0]]).astype(w.n.dtype)
    wb.A = np.concatenate([w.A, w.A[:2]])
    hp, hc = gpu_waveform(ctx, wb, check_flags=False)
    assert ctx.sync_flags() == fd.FDEMRI_FLAG_BAD_MODE
    assert np.array_equal(hp, hp0) and np.array_equal(hc, hc0)
    dw = fd.DeviceWaveform.from_workload(wb, device=ctx.device)
    rng = np.random.default_rng(4)
    g = [torch.as_tensor(rng.standard_normal(w.f.size) + 1j * rng.standard_normal(w.f.size), device=ctx.device)
         for _ in range(2)]
    out = ctx.vjp_dev(dw, g[0], g[1], "fp64")
    assert all(bool(torch.isfinite(torch.view_as_real(v) if v.is_complex() else v).all()) for v in out.values())
    ctx.sync_flags()


def test_profile_classes(ctx):
    """Profiling brackets only the selected kernel classes; an unknown class
    bit is rejected and leaves the selection as it was."""
    w = W.inspiral_20_modes()
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    ctx.profile(True, classes=["gather"])
    ctx.profile_read()
    ctx.waveform_dev(dw, "fp64")
    got = ctx.profile_read()
    assert got["gather"][1] == 1 and got["spline"][1] == 0 and got["pieces"][1] == 0
    assert got["gather"][0] > 0
    assert ctx._lib.fdemri_profile_classes(ctx._h, 1 << 7) == 1
    ctx.waveform_dev(dw, "fp64")
    got = ctx.profile_read()
    assert got["gather"][1] == 1 and got["spline"][1] == 0
    ctx.profile(True)
    ctx.waveform_dev(dw, "fp64")
    got = ctx.profile_read()
    # a 20-mode waveform has its set-up fused into one launch (the pieces class)
    assert got["gather"][1] == 1 and got["spline"][1] == 0 and got["pieces"][1] == 1
    w2 = W.inspiral_20_modes(K=300)  # above the fused set-up's knot limit: splines, then set-up
    dw2 = fd.DeviceWaveform.from_workload(w2, device=ctx.device)
    ctx.waveform_dev(dw2, "fp64")
    got = ctx.profile_read()
    assert got["gather"][1] == 1 and got["spline"][1] == 1 and got["pieces"][1] == 1
    ctx.profile(False)
    ctx.waveform_dev(dw, "fp64")
    assert all(v[1] == 0 for v in ctx.profile_read().values())


@pytest.mark.parametrize("workload", ["inspiral_20_modes_log_grid", "inspiral_20_modes"])
def test_single_waveform_graph_replays_match_eager(ctx, workload):
    """fdemri_waveform captured into a HIP graph (through torch's graph
    capture on the current stream) and replayed several times, with eager
    work and synchronisations in between, equals the eager call every time."""
    w = getattr(W, workload)()
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    ref = ctx.waveform_dev(dw, "fp64")
    torch.cuda.synchronize()
    out = (torch.empty_like(ref[0]), torch.empty_like(ref[1]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up on the capture stream
        ctx.waveform_dev(dw, "fp64", out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.waveform_dev(dw, "fp64", out=out)
    # the graph holds the context's workspace: unrelated library work runs on
    # a context of its own, so that nothing reallocates that workspace
    other = fd.Context(0)
    x = torch.randn(256, 256, device=ctx.device)
    for rep in range(4):
        out[0].fill_(float("nan"))
        out[1].fill_(float("nan"))
        g.replay()
        y = x @ x
        other.waveform_dev(dw, "mixed")
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep
    other.close()
    del g
    assert ctx.sync_flags() == 0
