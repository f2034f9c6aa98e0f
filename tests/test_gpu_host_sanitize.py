"""Every C-ABI entry point on device 0, from a host program whose runtime
host code (api.hip) and driver are built with AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged): a small synthetic
waveform in both precisions, the no-allocation entry, a graph-replayed
batch, the adjoint, the likelihood, trajectories, mode selection, band, time
domain, the special function, autotune with a malformed tuning cache,
profiling, argument errors and the allocation-failure hook."""
import pytest

from test_host_sanitize import assert_clean, run_driver

pytestmark = pytest.mark.gpu


def test_abi_entry_points_on_device_under_sanitizers():
    print("case: abi_driver_san device", flush=True)
    rc, out = run_driver("device", 300)
    assert_clean(rc, out)
