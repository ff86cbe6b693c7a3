"""The autotuner of batched contexts, through the C-ABI: every launch variant
it chooses among (stages in flight of the column-sweep product, row groups in
flight of the two CG updates) gives bit for bit the results of the default
launch, in both forms, and a tuned context reports its choice."""
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


def small_machine():
    return mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                      stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5, nsteps=2,
                      scheme=mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0))


def members_for(pb, n, seed0=2100):
    out = []
    for s in range(n):
        h, alpha, pf, period, rng = mi.scenario_params(seed0 + s)
        out.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                        T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    return out


def run(pb, mem, precision=mi.FP32_REFINE, **over):
    import paper_1707_03581_amd as m
    ctx = m.batch_simulation(pb, mem, precision=precision, **over)
    st = ctx.advance_steps(pb.nsteps)
    out = np.stack([ctx.get_scenario_temperature(s, pb.N) for s in range(len(mem))])
    ctx.destroy()
    return out, st


# FP32: S = 8 rows of 16-byte units, S = 6 4-byte copies and stores; FP64:
# S = 6 16-byte units, S = 5 4-byte copies and 8-byte stores
@pytest.mark.parametrize("precision,S", [(mi.FP32_REFINE, 8), (mi.FP32_REFINE, 6),
                                         (mi.FP64, 6), (mi.FP64, 5)])
def test_every_variant_matches_the_default_launch(precision, S):
    pb = small_machine()
    mem = members_for(pb, S)
    ref, st0 = run(pb, mem, precision)
    assert st0["col_depth"] == 2 and st0["groups_b"] == 4 and st0["groups_c"] == 4
    assert st0["autotuned"] == 0
    for v in range(8):
        out, st = run(pb, mem, precision, autotune=2 + v)
        assert st["col_depth"] == (1 if v & 1 else 2), v
        assert st["groups_b"] == (2 if v & 2 else 4), v
        assert st["groups_c"] == (8 if v & 4 else 4), v
        assert np.array_equal(out, ref), f"variant {v}"
        assert st["pcg_iters"] == st0["pcg_iters"]


@pytest.mark.parametrize("precision", [mi.FP32_REFINE, mi.FP64])
def test_tuned_context_matches_and_reports_its_choice(precision):
    pb = small_machine()
    mem = members_for(pb, 8, seed0=2300)
    ref, _ = run(pb, mem, precision)
    out, st = run(pb, mem, precision, autotune=1)
    assert st["autotuned"] == 1
    assert st["col_depth"] in (1, 2) and st["groups_b"] in (2, 4) and st["groups_c"] in (4, 8)
    if precision == mi.FP64:  # the operator only
        assert st["groups_b"] == 4 and st["groups_c"] == 4
    assert np.array_equal(out, ref)
    # a second context on the same mesh and scenario count takes the kept choice
    out2, st2 = run(pb, mem, precision, autotune=1)
    assert (st2["col_depth"], st2["groups_b"], st2["groups_c"]) == \
        (st["col_depth"], st["groups_b"], st["groups_c"])
    assert np.array_equal(out2, ref)
