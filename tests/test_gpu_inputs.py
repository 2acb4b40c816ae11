"""The device brick generator reproduces the host generator (same Philox
definition; Box-Muller through the device log/cos may differ in the last ulp)."""
import numpy as np
import pytest

from gwinputs import configs, philox

pytestmark = pytest.mark.gpu


def test_device_normals_match_host():
    import torch
    from gwinputs import device
    idx = np.concatenate([np.arange(5000), np.array([2**32 - 1, 2**32, 2**40 + 17, 2**63 - 5])]).astype(np.uint64)
    host = philox.normal(7, 3, idx)
    dev = device.normal_on_device(7, 3, idx).cpu().numpy()
    assert np.max(np.abs(dev - host)) <= 4e-15 * np.max(np.abs(host))


def test_device_bricks_match_host():
    import torch
    from gwinputs import device
    w = configs.strip(14, n_ao=13, n_ri=40, filter_eps=1e-9)
    s = w.system
    trip = s.triples()[::97]
    host = s.bricks(trip)
    dev = device.bricks_on_device(s, trip).cpu().numpy()
    assert np.max(np.abs(dev - host) / (np.abs(host) + 1e-300)) < 1e-14
