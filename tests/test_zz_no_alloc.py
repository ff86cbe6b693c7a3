"""The allocation-free stationary solve (mrsdc_set_stationary_noalloc, fixed
library scratch) against the allocating one (mrsdc_set_stationary), through
the C-ABI: the same kernels on the same data, so the field and the iteration
count must agree bit for bit.  Two calls in a row on one device, the second
on a smaller problem, so the second runs on the scratch the first left
behind."""
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


def problems():
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0)
    big = mi.machine(stand_nodes=(11, 11, 41), stock_nodes=(8, 8, 11), stand_L=(0.4, 0.4, 1.6),
                     stock_L=(0.28, 0.28, 0.4), y_offset=0.06, period=3.0, stroke=0.8,
                     scheme=sc, nsteps=1, seed=3)
    big.T_amb = [15.0, 35.0]
    small = mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                       stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5,
                       scheme=sc, nsteps=1, seed=4, jitter=0.2)
    small.T_amb = [25.0, 18.0]
    assert small.N < big.N
    return [big, small]


def test_noalloc_stationary_matches_allocating_entry():
    import paper_1707_03581_amd as m
    for pb in problems():
        ref_ctx = m.simulation(pb)
        it_ref = ref_ctx.set_stationary(rtol=1e-13)
        T_ref = m.get_state(ref_ctx, pb)
        ref_ctx.destroy()

        ctx = m.simulation(pb)
        with pytest.raises(m.MrsdcError) as ei:  # no device state yet: nothing to use
            ctx.set_stationary_noalloc(rtol=1e-13)
        assert ei.value.status == m.ESTATE
        ctx.advance(0.0)  # creates the context's device state
        it = ctx.set_stationary_noalloc(rtol=1e-13)
        T = m.get_state(ctx, pb)
        print(f"  N={pb.N} iterations {it} (allocating entry {it_ref}) "
              f"max |diff| {np.abs(T - T_ref).max():.3e}", flush=True)
        assert it == it_ref and it > 0
        assert np.array_equal(T, T_ref)
        # the field then steps like any other
        ctx.advance(pb.scheme.dt)
        assert np.all(np.isfinite(m.get_state(ctx, pb)))
        ctx.destroy()
