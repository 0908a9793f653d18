"""The allocation-free volume entry point (cac_volume_noalloc) against
cac_volume, called through the C ABI: two calls in a row on one device, the
second on a smaller lattice, so that partials left by the first call cannot
leak into the second."""
import numpy as np
import pytest

from paper_2607_25444_amd import capi
from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stepped(w, steps):
    sim = capi.Sim(w.shape, w.params)
    sim.set_geometry(w.solid, w.theta)
    sim.set_state(w.phi0)
    sim.step(steps)
    return sim


def _check_one(torch, w, steps):
    sim = _stepped(w, steps)
    ref = sim.volume()  # cac_volume: same kernels, handle memory for the partials
    phi, _, _ = sim.fields()
    solid = torch.from_numpy(np.ascontiguousarray(w.solid.reshape(-1), dtype=np.uint8)).to(sim.device)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=sim.device)
    capi.volume_noalloc(w.shape, solid, phi, out, stream=sim.stream)
    torch.cuda.synchronize()
    got = float(out.item())
    # same kernels and summation order as cac_volume: bitwise equal
    assert got == ref, (got, ref)
    # and the fluid sum itself, in FP64 on the host in another order
    host = np.asarray(phi.cpu().numpy(), dtype=np.float64)[w.solid.reshape(-1) == 0].sum()
    assert abs(got - host) <= 1e-12 * abs(host), (got, host)
    sim.close()
    return got


def test_noalloc_volume_matches_cac_volume_twice():
    torch = pytest.importorskip("torch")
    big = W.sessile_32(60.0)                                  # 32^3 = 32768 nodes
    small = W.sessile((24, 20, 16), 6.0, 120.0)               # 7680 nodes
    v1 = _check_one(torch, big, 20)
    v2 = _check_one(torch, small, 7)
    assert v2 < v1


def test_noalloc_volume_refuses_oversized_lattice():
    torch = pytest.importorskip("torch")
    d = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.CacError) as ei:
        capi.volume_noalloc((1024, 1024, 129), d, d, d)
    assert ei.value.status == capi.CAC_ERR_ARG
    assert "limit" in str(ei.value)
