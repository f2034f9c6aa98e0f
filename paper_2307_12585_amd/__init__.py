"""Frequency-domain EMRI mode summation on AMD MI355X (gfx950).

Thin ctypes binding of the C ABI in include/fdemri.h.  It only marshals
arguments: torch tensors provide device memory and the current HIP stream,
and every step of the computation runs in the HIP kernels of libfdemri.so.
There is no CPU fallback: if the library is missing, importing the binding
functions raises.

    import paper_2307_12585_amd as fd
    ctx = fd.Context()
    hp, hc = ctx.waveform(t, Fphi, Fr, Phiphi, Phir, l, m, n, A, theta, phi, scale, f)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdemri.so")

FDEMRI_OK, FDEMRI_EINVAL, FDEMRI_ENOMEM, FDEMRI_EDEVICE, FDEMRI_ENOTSUP = range(5)
FDEMRI_FP64, FDEMRI_MIXED = 0, 1
FDEMRI_NO_PARTNERS = 0x1
FDEMRI_COEFFS_GIVEN = 0x2
FDEMRI_CTX_BATCH_GRAPHS = 0x1
FDEMRI_FLAG_PIECE_OVERFLOW = 0x1
FDEMRI_FLAG_BAD_MODE = 0x2
FDEMRI_FLAG_TRAJ_STEPS = 0x4
FDEMRI_FLAG_BAD_INPUT = 0x8
FDEMRI_LL_HANN = 0x1
PRECISIONS = {"fp64": FDEMRI_FP64, "mixed": FDEMRI_MIXED}

EXPORTED = [
    "fdemri_create", "fdemri_destroy", "fdemri_last_error", "fdemri_sync_flags",
    "fdemri_waveform", "fdemri_waveform_batch", "fdemri_vjp", "fdemri_last_eval_count",
    "fdemri_profile_enable", "fdemri_profile_read", "fdemri_autotune", "fdemri_loglike",
    "fdemri_loglike_batch", "fdemri_select_modes", "fdemri_td_waveform", "fdemri_trajectory",
    "fdemri_signal_band", "fdemri_profile_classes", "fdemri_waveform_noalloc", "fdemri_spa_factor",
    "fdemri_last_group_eval_count",
]
KERNEL_CLASSES = ["spline", "pieces", "gather", "vjp"]


class TrajParams(ctypes.Structure):
    """fdemri_traj_params: M, mu (solar masses), p0, e0, T (s), Phiphi0, Phir0 (rad)."""
    _fields_ = [(n, ctypes.c_double) for n in ("M", "mu", "p0", "e0", "T", "Phiphi0", "Phir0")]


class FdemriError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fdemri status {status}: {msg}")
        self.status = status


class WaveformDesc(ctypes.Structure):
    """Mirror of fdemri_waveform_desc."""
    _fields_ = [
        ("K", ctypes.c_int32),
        ("t", ctypes.c_void_p), ("Fphi", ctypes.c_void_p), ("Fr", ctypes.c_void_p),
        ("Phiphi", ctypes.c_void_p), ("Phir", ctypes.c_void_p),
        ("Nm", ctypes.c_int32),
        ("l", ctypes.c_void_p), ("m", ctypes.c_void_p), ("n", ctypes.c_void_p),
        ("A", ctypes.c_void_p),
        ("theta", ctypes.c_double), ("phi", ctypes.c_double), ("scale", ctypes.c_double),
        ("Nf", ctypes.c_int32),
        ("f", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


_lib_handle = None


def lib():
    """Load libfdemri.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise FdemriError(-1, f"{LIB_PATH} is missing: build it with `python -m paper_2307_12585_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        L.fdemri_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, u32]
        L.fdemri_create.restype = ctypes.c_int
        L.fdemri_destroy.argtypes = [vp]
        L.fdemri_destroy.restype = None
        L.fdemri_last_error.argtypes = [vp]
        L.fdemri_last_error.restype = ctypes.c_char_p
        L.fdemri_sync_flags.argtypes = [vp, vp, ctypes.POINTER(u32)]
        L.fdemri_sync_flags.restype = ctypes.c_int
        L.fdemri_waveform.argtypes = [vp, ctypes.POINTER(WaveformDesc), ctypes.c_int, vp, vp, vp]
        L.fdemri_waveform.restype = ctypes.c_int
        L.fdemri_waveform_noalloc.argtypes = [vp, ctypes.POINTER(WaveformDesc), ctypes.c_int, vp, vp, vp]
        L.fdemri_waveform_noalloc.restype = ctypes.c_int
        L.fdemri_waveform_batch.argtypes = [vp, i32, ctypes.POINTER(WaveformDesc), ctypes.c_int,
                                            ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.fdemri_waveform_batch.restype = ctypes.c_int
        L.fdemri_vjp.argtypes = [vp, ctypes.POINTER(WaveformDesc), ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fdemri_vjp.restype = ctypes.c_int
        L.fdemri_loglike.argtypes = [vp, ctypes.POINTER(WaveformDesc), ctypes.c_int, vp, vp, vp, u32, vp, vp]
        L.fdemri_loglike.restype = ctypes.c_int
        L.fdemri_select_modes.argtypes = [vp, i32, i32, vp, ctypes.c_double, vp, vp, vp]
        L.fdemri_select_modes.restype = ctypes.c_int
        L.fdemri_signal_band.argtypes = [vp, ctypes.POINTER(WaveformDesc), vp, vp]
        L.fdemri_signal_band.restype = ctypes.c_int
        L.fdemri_trajectory.argtypes = [vp, i32, ctypes.POINTER(TrajParams), i32, vp, vp]
        L.fdemri_trajectory.restype = ctypes.c_int
        L.fdemri_td_waveform.argtypes = [vp, ctypes.POINTER(WaveformDesc), ctypes.c_double, ctypes.c_double, i32,
                                         vp, vp, vp]
        L.fdemri_td_waveform.restype = ctypes.c_int
        L.fdemri_loglike_batch.argtypes = [vp, i32, ctypes.POINTER(WaveformDesc), ctypes.c_int,
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), u32, vp, vp]
        L.fdemri_loglike_batch.restype = ctypes.c_int
        L.fdemri_last_eval_count.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.fdemri_last_eval_count.restype = ctypes.c_int
        L.fdemri_last_group_eval_count.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.fdemri_last_group_eval_count.restype = ctypes.c_int
        L.fdemri_autotune.argtypes = [vp, i32, ctypes.POINTER(WaveformDesc), ctypes.c_int,
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.POINTER(i32)]
        L.fdemri_autotune.restype = ctypes.c_int
        L.fdemri_profile_enable.argtypes = [vp, ctypes.c_int]
        L.fdemri_profile_enable.restype = ctypes.c_int
        L.fdemri_profile_read.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.fdemri_profile_read.restype = ctypes.c_int
        L.fdemri_spa_factor.argtypes = [vp, ctypes.c_int, i32, vp, vp, vp, vp, vp]
        L.fdemri_spa_factor.restype = ctypes.c_int
        L.fdemri_profile_classes.argtypes = [vp, u32]
        L.fdemri_profile_classes.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class DeviceWaveform:
    """Device-resident inputs of one waveform, in the layouts of
    fdemri_waveform_desc (float64 / int32 contiguous tensors; A as [Nm, K, 2]
    knot values, or with coeffs_given=True as [Nm, K-1, 4, 2] spline
    coefficients in ascending powers of t - t_i)."""

    def __init__(self, t, Fphi, Fr, Phiphi, Phir, l, m, n, A, theta, phi, scale, f,
                 partners=True, device="cuda", coeffs_given=False):
        dev = torch.device(device)
        d64 = dict(dtype=torch.float64, device=dev)
        self.t = torch.as_tensor(t, **d64).contiguous()
        self.Fphi = torch.as_tensor(Fphi, **d64).contiguous()
        self.Fr = torch.as_tensor(Fr, **d64).contiguous()
        self.Phiphi = torch.as_tensor(Phiphi, **d64).contiguous()
        self.Phir = torch.as_tensor(Phir, **d64).contiguous()
        self.l = torch.as_tensor(l, dtype=torch.int32, device=dev).contiguous()
        self.m = torch.as_tensor(m, dtype=torch.int32, device=dev).contiguous()
        self.n = torch.as_tensor(n, dtype=torch.int32, device=dev).contiguous()
        A = torch.as_tensor(A, device=dev)
        if A.is_complex():
            A = torch.view_as_real(A.to(torch.complex128))
        self.A = A.to(torch.float64).contiguous()
        self.f = torch.as_tensor(f, **d64).contiguous()
        self.theta, self.phi, self.scale = float(theta), float(phi), float(scale)
        self.partners = bool(partners)
        self.coeffs_given = bool(coeffs_given)
        self.device = dev

    @property
    def K(self):
        return int(self.t.numel())

    @property
    def Nm(self):
        return int(self.l.numel())

    @property
    def Nf(self):
        return int(self.f.numel())

    def desc(self) -> WaveformDesc:
        return WaveformDesc(
            K=self.K, t=_ptr(self.t).value, Fphi=_ptr(self.Fphi).value, Fr=_ptr(self.Fr).value,
            Phiphi=_ptr(self.Phiphi).value, Phir=_ptr(self.Phir).value, Nm=self.Nm,
            l=_ptr(self.l).value, m=_ptr(self.m).value, n=_ptr(self.n).value, A=_ptr(self.A).value,
            theta=self.theta, phi=self.phi, scale=self.scale, Nf=self.Nf, f=_ptr(self.f).value,
            flags=(0 if self.partners else FDEMRI_NO_PARTNERS)
            | (FDEMRI_COEFFS_GIVEN if self.coeffs_given else 0))

    @classmethod
    def from_workload(cls, w, device="cuda", partners=True, f=None):
        """From any object with the attributes of workloads.Workload."""
        tr = w.traj
        return cls(tr.t, tr.Fphi, tr.Fr, tr.Phiphi, tr.Phir, w.l, w.m, w.n, w.A, w.theta, w.phi,
                   w.scale, w.f if f is None else f, partners=partners, device=device)


class Context:
    """An fdemri context on one HIP device."""

    def __init__(self, device=None, graphs=False):
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        self._lib = lib()
        h = ctypes.c_void_p()
        st = self._lib.fdemri_create(ctypes.byref(h), idx, FDEMRI_CTX_BATCH_GRAPHS if graphs else 0)
        if st != FDEMRI_OK:
            raise FdemriError(st, "fdemri_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.fdemri_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != FDEMRI_OK:
            raise FdemriError(st, self._lib.fdemri_last_error(self._h).decode())

    def sync_flags(self) -> int:
        v = ctypes.c_uint32()
        self._check(self._lib.fdemri_sync_flags(self._h, _stream(self.device), ctypes.byref(v)))
        return int(v.value)

    def last_eval_count(self) -> int:
        v = ctypes.c_int64()
        self._check(self._lib.fdemri_last_eval_count(self._h, _stream(self.device), ctypes.byref(v)))
        return int(v.value)

    def last_group_eval_count(self) -> int:
        """Evaluations of the last call whose root was solved (one per voice
        group of rows with the same (m, n), piece and bin)."""
        v = ctypes.c_int64()
        self._check(self._lib.fdemri_last_group_eval_count(self._h, _stream(self.device), ctypes.byref(v)))
        return int(v.value)

    def profile(self, enable: bool, classes=None):
        """Bracket kernel launches with HIP events on their stream: every
        class, or only the kernel classes named in `classes` (KERNEL_CLASSES)."""
        names = KERNEL_CLASSES if classes is None else classes
        mask = 0
        for k in names:
            mask |= 1 << KERNEL_CLASSES.index(k)
        self._check(self._lib.fdemri_profile_classes(self._h, mask))
        self._check(self._lib.fdemri_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read (synchronises)."""
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(self._lib.fdemri_profile_read(self._h, _stream(self.device), ms, cnt))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def waveform_dev(self, dw: DeviceWaveform, prec="fp64", out=None):
        """h_+(f), h_x(f) for device inputs; complex128 (fp64) or complex64 (mixed)."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        if out is None:
            hp = torch.empty(dw.Nf, dtype=ctype, device=dw.device)
            hc = torch.empty(dw.Nf, dtype=ctype, device=dw.device)
        else:
            hp, hc = out
            assert hp.dtype == ctype and hc.dtype == ctype and hp.numel() == dw.Nf and hc.numel() == dw.Nf
            assert hp.is_contiguous() and hc.is_contiguous()
        d = dw.desc()
        self._check(self._lib.fdemri_waveform(self._h, ctypes.byref(d), p, _ptr(hp), _ptr(hc),
                                              _stream(self.device)))
        return hp, hc

    def waveform_noalloc_dev(self, dw: DeviceWaveform, out, prec="fp64"):
        """fdemri_waveform_noalloc into the caller's (h_+, h_x) tensors: the
        library allocates nothing (its scratch is a fixed device array)."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        hp, hc = out
        assert hp.dtype == ctype and hc.dtype == ctype and hp.numel() == dw.Nf and hc.numel() == dw.Nf
        assert hp.is_contiguous() and hc.is_contiguous()
        d = dw.desc()
        self._check(self._lib.fdemri_waveform_noalloc(self._h, ctypes.byref(d), p, _ptr(hp), _ptr(hc),
                                                      _stream(self.device)))
        return hp, hc

    def spa_factor(self, gd, gdd, direction, prec="fp64"):
        """fdemri_spa_factor: G of Eq. extendedspa1 for float64 device tensors
        gd, gdd and int32 piece directions; complex128 (fp64) or complex64."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        gd = gd.to(torch.float64).contiguous()
        gdd = gdd.to(torch.float64).contiguous()
        direction = direction.to(torch.int32).contiguous()
        assert gd.numel() == gdd.numel() == direction.numel()
        out = torch.empty(gd.numel(), dtype=ctype, device=gd.device)
        self._check(self._lib.fdemri_spa_factor(self._h, p, gd.numel(), _ptr(gd), _ptr(gdd), _ptr(direction),
                                                _ptr(out), _stream(self.device)))
        return out

    def waveform(self, t, Fphi, Fr, Phiphi, Phir, l, m, n, A, theta, phi, scale, f,
                 prec="fp64", partners=True):
        dw = DeviceWaveform(t, Fphi, Fr, Phiphi, Phir, l, m, n, A, theta, phi, scale, f,
                            partners=partners, device=self.device)
        return self.waveform_dev(dw, prec)

    def loglike_dev(self, dw: DeviceWaveform, d_p, d_c, wS, prec="fp64", hann=False, out=None):
        """Whittle log-likelihood with the mode sum fused (fdemri_loglike):
        returns a float64 device tensor (log L, <h|h>, <d|h>) for data d_p, d_c
        ([Nf] complex of the precision's type) and per-bin weights
        wS = 4 w_k / S_n(f_k) ([Nf] float64)."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        assert d_p.dtype == ctype and d_c.dtype == ctype and wS.dtype == torch.float64
        assert d_p.numel() == dw.Nf and d_c.numel() == dw.Nf and wS.numel() == dw.Nf
        assert d_p.is_contiguous() and d_c.is_contiguous() and wS.is_contiguous()
        if out is None:
            out = torch.empty(3, dtype=torch.float64, device=dw.device)
        d = dw.desc()
        self._check(self._lib.fdemri_loglike(self._h, ctypes.byref(d), p, _ptr(d_p), _ptr(d_c), _ptr(wS),
                                             FDEMRI_LL_HANN if hann else 0, _ptr(out), _stream(self.device)))
        return out

    def td_waveform_dev(self, dw: DeviceWaveform, t0, dt, Nt, out=None):
        """h_+(t_k), h_x(t_k) (float64 device tensors) of the time-domain voice
        sum on t_k = t0 + k dt, k < Nt (fdemri_td_waveform)."""
        if out is None:
            out = (torch.empty(Nt, dtype=torch.float64, device=dw.device),
                   torch.empty(Nt, dtype=torch.float64, device=dw.device))
        hp, hc = out
        assert hp.dtype == torch.float64 and hc.dtype == torch.float64 and hp.numel() == Nt and hc.numel() == Nt
        d = dw.desc()
        self._check(self._lib.fdemri_td_waveform(self._h, ctypes.byref(d), float(t0), float(dt), int(Nt),
                                                 _ptr(hp), _ptr(hc), _stream(self.device)))
        return hp, hc

    def trajectory(self, params, K):
        """fdemri_trajectory for a list of dicts with keys M, mu, p0, e0, T and
        optionally Phiphi0, Phir0: a float64 device tensor [B, 7, K] with rows
        t, Fphi, Fr, Phiphi, Phir, p, e."""
        B = len(params)
        arr = (TrajParams * B)(*[TrajParams(P["M"], P["mu"], P["p0"], P["e0"], P["T"], P.get("Phiphi0", 0.0),
                                            P.get("Phir0", 0.0)) for P in params])
        out = torch.empty(B, 7, K, dtype=torch.float64, device=self.device)
        self._check(self._lib.fdemri_trajectory(self._h, B, arr, K, _ptr(out), _stream(self.device)))
        return out

    def signal_band(self, dw: DeviceWaveform):
        """(f_min, f_max) of the voices of dw (fdemri_signal_band; synchronises)."""
        band = torch.empty(2, dtype=torch.float64, device=dw.device)
        d = dw.desc()
        self._check(self._lib.fdemri_signal_band(self._h, ctypes.byref(d), _ptr(band), _stream(self.device)))
        b = band.cpu()
        return float(b[0]), float(b[1])

    def select_modes(self, A, eps):
        """fdemri_select_modes: indices (int32 device tensor, table order) of the
        rows of A ([Nm, K] complex128 device tensor of amplitude knot values)
        kept by the power criterion at threshold eps (synchronises to read the
        count)."""
        A = A.to(torch.complex128).contiguous()
        Nm, K = A.shape
        idx = torch.empty(max(Nm, 1), dtype=torch.int32, device=A.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=A.device)
        self._check(self._lib.fdemri_select_modes(self._h, K, Nm, _ptr(A), float(eps), _ptr(idx), _ptr(cnt),
                                                  _stream(self.device)))
        return idx[: int(cnt.item())]

    def loglike_batch(self, dws, ds_p, ds_c, wSs, prec="fp64", hann=False, out=None):
        """fdemri_loglike_batch: a [B, 3] float64 device tensor of (log L,
        <h|h>, <d|h>) per waveform, for lists of data and weight tensors."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        B = len(dws)
        for dw, a, b, w in zip(dws, ds_p, ds_c, wSs):
            assert a.dtype == ctype and b.dtype == ctype and w.dtype == torch.float64
            assert a.numel() == dw.Nf and b.numel() == dw.Nf and w.numel() == dw.Nf
            assert a.is_contiguous() and b.is_contiguous() and w.is_contiguous()
        if out is None:
            out = torch.empty(B, 3, dtype=torch.float64, device=dws[0].device)
        descs = (WaveformDesc * B)(*[d.desc() for d in dws])
        arr = lambda ts: (ctypes.c_void_p * B)(*[t.data_ptr() for t in ts])
        self._check(self._lib.fdemri_loglike_batch(self._h, B, descs, p, arr(ds_p), arr(ds_c), arr(wSs),
                                                   FDEMRI_LL_HANN if hann else 0, _ptr(out),
                                                   _stream(self.device)))
        return out

    def vjp_dev(self, dw: DeviceWaveform, g_hp, g_hc, prec="fp64", coef=True, knots=True):
        """Gradients of a real loss from the cotangents g = dL/dRe h + i dL/dIm h.
        Returns a dict with (as requested) gA [Nm, K-1, 4] complex128 (spline
        coefficients), gPhi [2, K-1, 4], gA_knots [Nm, K] complex128,
        gPhi_knots [2, K] and g_scalars [5] (theta, phi, scale, Phi_phi0, Phi_r0)."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        g_hp = g_hp.to(ctype).contiguous()
        g_hc = g_hc.to(ctype).contiguous()
        assert g_hp.numel() == dw.Nf and g_hc.numel() == dw.Nf
        K, Nm, dev = dw.K, dw.Nm, dw.device
        out = {"g_scalars": torch.empty(5, dtype=torch.float64, device=dev)}
        if coef:
            out["gA"] = torch.empty(Nm, K - 1, 4, 2, dtype=torch.float64, device=dev)
            out["gPhi"] = torch.empty(2, K - 1, 4, dtype=torch.float64, device=dev)
        if knots:
            if not dw.coeffs_given:  # given coefficients have no amplitude knots
                out["gA_knots"] = torch.empty(Nm, K, 2, dtype=torch.float64, device=dev)
            out["gPhi_knots"] = torch.empty(2, K, dtype=torch.float64, device=dev)
        d = dw.desc()
        self._check(self._lib.fdemri_vjp(
            self._h, ctypes.byref(d), p, _ptr(g_hp), _ptr(g_hc), _ptr(out.get("gA")), _ptr(out.get("gPhi")),
            _ptr(out.get("gA_knots")), _ptr(out.get("gPhi_knots")), _ptr(out["g_scalars"]), _stream(self.device)))
        if coef:
            out["gA"] = torch.view_as_complex(out["gA"])
        if "gA_knots" in out:
            out["gA_knots"] = torch.view_as_complex(out["gA_knots"])
        return out

    def autotune(self, dws, prec="fp64", outs=None) -> int:
        """Pick the gather's bins-per-lane for this workload class (see
        fdemri_autotune); returns the choice."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        B = len(dws)
        if outs is None:
            outs = [(torch.empty(d.Nf, dtype=ctype, device=d.device),
                     torch.empty(d.Nf, dtype=ctype, device=d.device)) for d in dws]
        descs = (WaveformDesc * B)(*[d.desc() for d in dws])
        hp = (ctypes.c_void_p * B)(*[o[0].data_ptr() for o in outs])
        hc = (ctypes.c_void_p * B)(*[o[1].data_ptr() for o in outs])
        bpl = ctypes.c_int32()
        self._check(self._lib.fdemri_autotune(self._h, B, descs, p, hp, hc, _stream(self.device),
                                              ctypes.byref(bpl)))
        return int(bpl.value)

    def waveform_batch(self, dws, prec="fp64", outs=None):
        """Several waveforms in one call; returns a list of (h_+, h_x)."""
        p = PRECISIONS[prec]
        ctype = torch.complex128 if p == FDEMRI_FP64 else torch.complex64
        B = len(dws)
        if outs is None:
            outs = [(torch.empty(d.Nf, dtype=ctype, device=d.device),
                     torch.empty(d.Nf, dtype=ctype, device=d.device)) for d in dws]
        descs = (WaveformDesc * B)(*[d.desc() for d in dws])
        hp = (ctypes.c_void_p * B)(*[o[0].data_ptr() for o in outs])
        hc = (ctypes.c_void_p * B)(*[o[1].data_ptr() for o in outs])
        self._check(self._lib.fdemri_waveform_batch(self._h, B, descs, p, hp, hc, _stream(self.device)))
        return outs
