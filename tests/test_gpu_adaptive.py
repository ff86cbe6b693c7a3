"""Residual-controlled sweeps on the GPU (single and batched) against the
oracle with the same rule: same number of sweeps, temperatures within the
FP64 bar.  The tolerance is placed between two residual levels and every
residual the oracle meets is checked to stay clear of it, so both sides take
the same decisions."""
import dataclasses
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def machine(nsteps=4, **kw):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0)
    return mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                      stock_L=(0.15, 0.2, 0.3), period=3.0, stroke=0.5, scheme=sc,
                      nsteps=nsteps, **kw)


def controlled(pb, T0=None, **over):
    """Tolerance between the first step's residuals of iterates 1 and 2, and
    the oracle's controlled run (T, sweeps) with its residuals checked."""
    _, _, res = oracle.run(pb, nsteps=1, T0=T0, residuals=True, **over)
    tol = float(np.sqrt(res[0][1] * res[0][2]))
    sc = dataclasses.replace(pb.scheme, sweep_tol=tol)
    T, st, r = oracle.run(pb, T0=T0, scheme=sc, residuals=True, **over)
    seen = r[r > 0]
    assert np.all(np.abs(np.log(seen / tol)) > np.log(1.02)), (seen, tol)
    return tol, sc, T, st["sweeps"]


def test_single_context_controlled_sweeps():
    import paper_1707_03581_amd as m
    pb = machine()
    tol, sc, ref, sweeps = controlled(pb)
    assert 0 < sweeps < pb.nsteps * pb.scheme.K
    pb2 = dataclasses.replace(pb, scheme=sc)
    ctx = m.simulation(pb2)
    st = ctx.advance(pb.nsteps * pb.scheme.dt)
    T = m.get_state(ctx, pb)
    ctx.destroy()
    print(f"  tol {tol:.3e}: sweeps gpu {st['sweeps']} oracle {sweeps}, rel_l2 {rel(T, ref):.3e}",
          flush=True)
    assert st["sweeps"] == sweeps
    assert rel(T, ref) <= TOL


@pytest.mark.parametrize("precision,tol_T", [(mi.FP64, TOL), (mi.FP32_REFINE, 1e-7)])
def test_batched_controlled_sweeps(precision, tol_T):
    import paper_1707_03581_amd as m
    pb = machine()
    pb.scheme = dataclasses.replace(pb.scheme, precision=precision)
    members, refs, total = [], [], 0
    for s in range(3):
        h, alpha, pf, period, rng = mi.scenario_params(1600 + s)
        mb = dict(h=h, alpha=alpha, friction_W=pf, period=period,
                  T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N))
        members.append(mb)
    over = dict(h=members[0]["h"], alpha=members[0]["alpha"],
                friction_W=members[0]["friction_W"], period=members[0]["period"])
    tol, _, _, _ = controlled(pb, T0=members[0]["T0"], **over)
    sc = dataclasses.replace(pb.scheme, sweep_tol=tol)
    for mb in members:
        T, st, r = oracle.run(pb, T0=mb["T0"], scheme=sc, residuals=True, h=mb["h"],
                              alpha=mb["alpha"], friction_W=mb["friction_W"],
                              period=mb["period"])
        seen = r[r > 0]
        assert np.all(np.abs(np.log(seen / tol)) > np.log(1.02)), (seen, tol)
        refs.append(T)
        total += st["sweeps"]
    ctx = m.batch_simulation(dataclasses.replace(pb, scheme=sc), members)
    st = ctx.advance_steps(pb.nsteps)
    outs = [ctx.get_scenario_temperature(s, pb.N) for s in range(3)]
    ctx.destroy()
    print(f"  sweeps gpu {st['sweeps']} oracle {total}", flush=True)
    assert st["sweeps"] == total
    for s in range(3):
        assert rel(outs[s], refs[s]) <= tol_T
    # a member alone takes the same decisions, bitwise the same result
    alone = m.batch_simulation(dataclasses.replace(pb, scheme=sc), [members[1]])
    alone.advance_steps(pb.nsteps)
    assert np.array_equal(alone.get_scenario_temperature(0, pb.N), outs[1])
    alone.destroy()
