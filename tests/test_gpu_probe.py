"""The bandwidth probe of the collide-stream's access pattern (measurement
only): it times, it leaves the handle without a state, and a state set
afterwards steps exactly like a fresh handle's."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_pull_copy_probe_times_and_resets_the_state():
    from paper_2607_25444_amd import capi
    w = W.sessile((40, 36, 24), 8.0, 60.0)
    s = capi.Sim(w.shape, w.params)
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0)
    s.step(3)
    ms = s.pull_copy_probe(5)
    assert ms > 0.0
    with pytest.raises(capi.CacError) as e:
        s.step(1)
    assert e.value.status == capi.CAC_ERR_STATE
    s.set_state(w.phi0)
    s.step(4)
    a = [t.cpu().numpy() for t in s.fields()]
    t = capi.Sim(w.shape, w.params)
    t.set_geometry(w.solid, w.theta)
    t.set_state(w.phi0)
    t.step(4)
    b = [x.cpu().numpy() for x in t.fields()]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(capi.CacError):
        s.pull_copy_probe(0)
    s.close()
    t.close()
