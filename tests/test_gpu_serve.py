"""Serving: requests arriving over time, admitted into free slots of per-level
batched contexts (continuous batching).  Each request's result must be
bitwise the same as running it alone, and match the oracle."""
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def levels(precision=mi.FP64):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0, precision=precision)
    a = mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                   stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5, scheme=sc)
    b = mi.machine(stand_nodes=(6, 9, 23), stock_nodes=(5, 6, 9), stand_L=(0.2, 0.3, 0.9),
                   stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5, scheme=sc)
    return {"coarse": a, "fine": b}


def trace(lv, n=10, seed=7, gap=0.05):
    from paper_1707_03581_amd.serve import Request
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    names = list(lv)
    for i in range(n):
        t += rng.exponential(gap)
        name = names[int(rng.integers(0, len(names)))]
        h, alpha, pf, period, r2 = mi.scenario_params(500 + i)
        out.append(Request(id=i, arrival=t, level=name, nsteps=int(rng.integers(2, 6)), h=h,
                           alpha=alpha, friction_W=pf, period=period,
                           T0=20.0 + r2.uniform(-0.5, 0.5, size=lv[name].N)))
    return out


@pytest.mark.parametrize("precision,tol", [(mi.FP64, 1e-10), (mi.FP32_REFINE, 1e-7)])
def test_served_results_equal_alone_and_oracle(precision, tol):
    import paper_1707_03581_amd as m
    from paper_1707_03581_amd.serve import Server, summarize
    lv = levels(precision)
    reqs = Server(lv, slots_per_level=4).run(trace(lv))
    summ = summarize(reqs, 5.0, {k: v.N for k, v in lv.items()})
    print("  ", {k: round(v, 4) for k, v in summ.items()}, flush=True)
    overlapped = any(a.admitted < b.finished and b.admitted < a.finished and a.level == b.level
                     for a in reqs for b in reqs if a.id < b.id)
    assert overlapped, "no two requests shared a batch"
    for r in reqs:
        pb = lv[r.level]
        ctx = m.batch_simulation(pb, [dict(h=r.h, alpha=r.alpha, friction_W=r.friction_W,
                                           period=r.period, T0=r.T0)])
        ctx.advance_steps(r.nsteps)
        alone = ctx.get_scenario_temperature(0, pb.N)
        ctx.destroy()
        assert np.array_equal(alone, r.result), r.id
    for r in reqs[:3]:
        pb = lv[r.level]
        ref, _ = oracle.run(pb, nsteps=r.nsteps, T0=r.T0, h=r.h, alpha=r.alpha,
                            friction_W=r.friction_W, period=r.period)
        e = float(np.linalg.norm(r.result - ref) / np.linalg.norm(ref))
        print(f"  request {r.id} ({r.level}, {r.nsteps} steps): rel_l2={e:.3e}", flush=True)
        assert e <= tol


def test_small_budget_queues_and_rejects():
    """An HBM budget that holds two slots of the coarse level, one of the fine
    one and no pool of a large level: requests queue for the slots, the
    large level's requests are rejected, and every served result is still the
    same as its run alone."""
    import paper_1707_03581_amd as m
    from paper_1707_03581_amd.serve import Server, level_bytes, summarize
    lv = levels()
    sc = lv["coarse"].scheme
    lv["large"] = mi.machine(stand_nodes=(9, 11, 31), stock_nodes=(7, 8, 11),
                             stand_L=(0.2, 0.3, 0.9), stock_L=(0.15, 0.2, 0.3), y_offset=0.05,
                             period=3.0, stroke=0.5, scheme=sc)
    lb = {n: level_bytes(pb) for n, pb in lv.items()}
    print("  level bytes (shared, per slot):", lb, flush=True)
    budget = lb["coarse"][0] + 2 * lb["coarse"][1] + lb["fine"][0] + lb["fine"][1]
    assert budget < sum(lb["large"])  # the large level cannot fit even alone
    srv = Server(lv, slots_per_level=2, hbm_budget_bytes=budget)
    plan = srv.size_pools()
    assert plan == {"coarse": 2, "fine": 1, "large": 0}
    reqs = srv.run(trace(lv, n=12, seed=11, gap=0.002))  # a burst
    assert srv.held_bytes <= budget
    summ = summarize(reqs, 5.0, {k: v.N for k, v in lv.items()})
    print("  ", summ, flush=True)
    rejected = [r for r in reqs if r.rejected]
    served = [r for r in reqs if not r.rejected]
    assert rejected and all(r.level == "large" and r.result is None for r in rejected)
    assert all(r.level != "large" for r in served)
    # a request that arrived while its level's slots were taken waited for one
    assert any(r.admitted - r.arrival > 0.02 for r in served)
    for r in served:
        pb = lv[r.level]
        ctx = m.batch_simulation(pb, [dict(h=r.h, alpha=r.alpha, friction_W=r.friction_W,
                                           period=r.period, T0=r.T0)])
        ctx.advance_steps(r.nsteps)
        alone = ctx.get_scenario_temperature(0, pb.N)
        ctx.destroy()
        assert np.array_equal(alone, r.result), r.id


def test_slot_bytes_add_up_to_the_footprint():
    import paper_1707_03581_amd as m
    pb = levels()["fine"]
    for S in (1, 3):
        ctx = m.batch_simulation(pb, [dict(h=10.0, alpha=900.0, friction_W=100.0, period=3.0,
                                           T0=pb.T0)] * S)
        ctx.advance_steps(0)
        per, shared = ctx.slot_bytes()
        fp = ctx.footprint_bytes()
        ctx.destroy()
        print(f"  S={S}: per slot {per}, shared {shared}, footprint {fp}", flush=True)
        assert per > 8 * pb.N and shared > 0
        assert 0 <= shared + S * per - fp < S
