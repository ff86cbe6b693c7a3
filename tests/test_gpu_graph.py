"""The time step captured into a HIP graph and replayed (use_graph) against
the same step launched directly, through the C-ABI.

A context with use_graph runs its first WARM steps directly (they learn the
CG launch budgets) and captures the step after them.  Each test advances a
captured and a direct context side by side one step at a time, with the program's own host work and synchronisations between the
replays, and compares every step: FP64 bit for bit (a converged solve's
spare launches change nothing), FP32 + refinement within the refinement's
tolerance; both against the oracle as well.
"""
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle

pytestmark = pytest.mark.gpu
WARM = 3  # steps a use_graph context runs directly before its first capture


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def pkg():
    import paper_1707_03581_amd as m
    return m


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def small(precision=mi.FP64, nsteps=6):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0, precision=precision)
    return mi.machine(stand_nodes=(9, 11, 31), stock_nodes=(7, 8, 11), stand_L=(0.2, 0.3, 0.9),
                      stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5,
                      scheme=sc, nsteps=nsteps)


@pytest.mark.parametrize("precision", [mi.FP64, mi.FP32_REFINE], ids=["fp64", "fp32refine"])
def test_single_captured_step_matches_direct(precision):
    m = pkg()
    pb = small(precision)
    g = m.simulation(pb, use_graph=1)
    d = m.simulation(pb)
    captures = launches = 0
    for n in range(pb.nsteps):
        sg = g.advance(pb.scheme.dt)
        d.advance(pb.scheme.dt)
        captures += sg["graph_captures"]
        launches += sg["graph_launches"]
        Tg, Td = m.get_state(g, pb), m.get_state(d, pb)
        if precision == mi.FP64:
            assert np.array_equal(Tg, Td), f"step {n}"
        else:
            assert rel(Tg, Td) <= 1e-9, f"step {n}"
    g.destroy()
    d.destroy()
    print(f"  captures {captures}, graph launches {launches}", flush=True)
    assert launches == pb.nsteps - WARM and 1 <= captures <= launches
    ref, _ = oracle.run(pb, nsteps=pb.nsteps)
    assert rel(Tg, ref) <= (1e-10 if precision == mi.FP64 else 1e-7)


def test_single_machine_310k_captured():
    """The 310,042-DOF machine, 3 steps captured after the direct ones, bit for
    bit the direct run."""
    m = pkg()
    pb = mi.machine_310k(nsteps=WARM + 3)
    g = m.simulation(pb, use_graph=1)
    d = m.simulation(pb)
    for n in range(WARM + 3):
        st = g.advance(pb.scheme.dt)
        d.advance(pb.scheme.dt)
        assert st["graph_launches"] == (1 if n >= WARM else 0)
        assert np.array_equal(m.get_state(g, pb), m.get_state(d, pb)), f"step {n}"
    g.destroy()
    d.destroy()


@pytest.mark.parametrize("precision", [mi.FP64, mi.FP32_REFINE], ids=["fp64", "fp32refine"])
def test_batch_captured_step_matches_direct(precision):
    m = pkg()
    pb = small(precision)
    members = []
    for s in range(3):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    g = m.batch_simulation(pb, members, use_graph=1)
    d = m.batch_simulation(pb, members)
    launches = 0
    for n in range(pb.nsteps):
        launches += g.advance_steps(1)["graph_launches"]
        d.advance_steps(1)
        for s in range(3):
            Tg, Td = g.get_scenario_temperature(s, pb.N), d.get_scenario_temperature(s, pb.N)
            if precision == mi.FP64:
                assert np.array_equal(Tg, Td), f"step {n} member {s}"
            else:
                assert rel(Tg, Td) <= 1e-9, f"step {n} member {s}"
    # a member leaves and joins mid-run: the captured step follows the flags
    g.set_active(1, False)
    d.set_active(1, False)
    g.advance_steps(2)
    d.advance_steps(2)
    for s in range(3):
        Tg, Td = g.get_scenario_temperature(s, pb.N), d.get_scenario_temperature(s, pb.N)
        assert rel(Tg, Td) <= (0.0 if precision == mi.FP64 else 1e-9)
    g.destroy()
    d.destroy()
    assert launches == pb.nsteps - WARM
