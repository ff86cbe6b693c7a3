"""Contexts whose device memory comes from the caller's allocator (here
torch's caching allocator, through the C-ABI's mrsdc_allocator): torch then
accounts the library's buffers, returns them at destroy, and the results are
the same bit for bit as with the library's own allocations."""
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def problem():
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0)
    return mi.machine(stand_nodes=(9, 11, 31), stock_nodes=(7, 8, 11), stand_L=(0.2, 0.3, 0.9),
                      stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5,
                      scheme=sc, nsteps=3)


def test_torch_allocator_owns_the_buffers():
    import torch
    import paper_1707_03581_amd as m
    pb = problem()
    ref = m.simulation(pb)
    ref.advance(pb.nsteps * pb.scheme.dt)
    T_ref = m.get_state(ref, pb)
    ref.destroy()

    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    alloc = m.torch_allocator(0)
    ctx = m.simulation(pb, alloc=alloc)
    ctx.advance(pb.nsteps * pb.scheme.dt)
    held = torch.cuda.memory_allocated() - base
    fp = ctx.footprint_bytes()
    print(f"  torch holds {held} bytes, footprint {fp}", flush=True)
    assert held >= fp > 0
    assert np.array_equal(m.get_state(ctx, pb), T_ref)
    ctx.set_stationary(rtol=1e-10)  # its temporary buffers come and go through torch too
    ctx.destroy()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_torch_allocator_batch():
    import torch
    import paper_1707_03581_amd as m
    pb = problem()
    members = []
    for s in range(3):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    d = m.batch_simulation(pb, members)
    d.advance_steps(2)
    ref = [d.get_scenario_temperature(s, pb.N) for s in range(3)]
    d.destroy()
    base = torch.cuda.memory_allocated()
    g = m.batch_simulation(pb, members, alloc=m.torch_allocator(0))
    g.advance_steps(2)
    assert torch.cuda.memory_allocated() - base >= g.footprint_bytes()
    for s in range(3):
        assert np.array_equal(g.get_scenario_temperature(s, pb.N), ref[s])
    g.destroy()
    assert torch.cuda.memory_allocated() == base
