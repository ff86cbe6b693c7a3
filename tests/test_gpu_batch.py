"""Batched ensembles on the GPU: every member against the FP64 oracle run with
that member's parameters (<= 1e-10 relative L2), and each member's result
bitwise the same alone and inside the batch."""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def members_for(pb, n, seed0=1000):
    out = []
    for s in range(n):
        h, alpha, pf, period, rng = mi.scenario_params(seed0 + s)
        out.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                        T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    return out


def small_machine(**kw):
    base = dict(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                stock_L=(0.15, 0.2, 0.3), y_offset=0.05, period=3.0, stroke=0.5, nsteps=3,
                scheme=mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0))
    base.update(kw)
    return mi.machine(**base)


def run_batch(pb, members, nsteps, **over):
    import paper_1707_03581_amd as m
    ctx = m.batch_simulation(pb, members, **over)
    st = ctx.advance_steps(nsteps)
    out = [ctx.get_scenario_temperature(s, pb.N) for s in range(len(members))]
    times = [ctx.get_scenario_time(s) for s in range(len(members))]
    ctx.destroy()
    return out, st, times


@pytest.mark.parametrize("S", [3, 64])
def test_batch_members_match_oracle(S):
    pb = small_machine()
    mem = members_for(pb, S)
    outs, st, times = run_batch(pb, mem, pb.nsteps)
    assert all(t == pytest.approx(pb.nsteps * pb.scheme.dt) for t in times)
    check = range(S) if S <= 4 else [0, 17, 40, 63]
    for s in check:
        mb = mem[s]
        ref, _ = oracle.run(pb, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                            friction_W=mb["friction_W"], period=mb["period"])
        e = rel(outs[s], ref)
        print(f"  S={S} member {s}: rel_l2={e:.3e}", flush=True)
        assert e <= 1e-10


@pytest.mark.parametrize("S", [5, 8])
def test_member_alone_equals_member_in_batch(S):
    pb = small_machine()
    mem = members_for(pb, S)
    outs, _, _ = run_batch(pb, mem, 2)
    for s in (0, 3):
        alone, _, _ = run_batch(pb, [mem[s]], 2)
        assert np.array_equal(alone[0], outs[s])


def test_inactive_member_keeps_state_and_clock():
    import paper_1707_03581_amd as m
    pb = small_machine()
    mem = members_for(pb, 3)
    ctx = m.batch_simulation(pb, mem)
    ctx.advance_steps(1)
    frozen = ctx.get_scenario_temperature(1, pb.N)
    ctx.set_active(1, False)
    ctx.advance_steps(2)
    assert np.array_equal(ctx.get_scenario_temperature(1, pb.N), frozen)
    assert ctx.get_scenario_time(1) == pytest.approx(pb.scheme.dt)
    assert ctx.get_scenario_time(0) == pytest.approx(3 * pb.scheme.dt)
    # re-activated, it continues from where it stopped: same as 3 uninterrupted steps
    ctx.set_active(1, True)
    ctx.advance_steps(2)
    a = ctx.get_scenario_temperature(1, pb.N)
    ctx.destroy()
    ref, _, _ = run_batch(pb, [mem[1]], 3)
    assert np.array_equal(a, ref[0])


def test_ensemble_7p5mm_sampled():
    """The 64-member ensemble on the 7.5 mm machine (714,798 DOF per member),
    2 steps; 3 members checked against the oracle."""
    pb = mi.ensemble_member(0, nsteps=2, precision=mi.FP64)
    mem = []
    for s in range(64):
        q = mi.scenario_params(s)
        rng = q[4]
        mem.append(dict(h=q[0], alpha=q[1], friction_W=q[2], period=q[3],
                        T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    outs, st, _ = run_batch(pb, mem, 2)
    print(f"  cg iterations {st['pcg_iters']} max {st['max_iters']}", flush=True)
    for s in (0, 31, 63):
        mb = mem[s]
        ref, _ = oracle.run(pb, nsteps=2, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                            friction_W=mb["friction_W"], period=mb["period"])
        e = rel(outs[s], ref)
        print(f"  member {s}: rel_l2={e:.3e}", flush=True)
        assert e <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_blown_up_member_does_not_leak_into_others(precision):
    """A member whose state overflows makes the step fail (ENOCONV, nothing
    committed); once it is switched off, its non-finite CG vectors must not
    reach the other members (rows shorter than the gather chunk read a
    placeholder slot), which then match their runs alone bitwise."""
    import paper_1707_03581_amd as m
    pb = small_machine()
    mem = members_for(pb, 3, seed0=1200)
    sign = np.where(np.arange(pb.N) % 2 == 0, 1.0, -1.0)
    mem[0] = dict(mem[0], T0=1e308 * sign)
    over = dict(precision=precision, pcg_maxit=60, refine_maxit=4)
    ctx = m.batch_simulation(pb, mem, **over)
    with pytest.raises(m.MrsdcError) as e:
        ctx.advance_steps(1)
    assert e.value.status == m.ENOCONV
    for s in (1, 2):
        assert ctx.get_scenario_time(s) == 0.0
        assert np.array_equal(ctx.get_scenario_temperature(s, pb.N), mem[s]["T0"])
    ctx.set_active(0, False)
    ctx.advance_steps(2)
    outs = [ctx.get_scenario_temperature(s, pb.N) for s in (1, 2)]
    ctx.destroy()
    for s, got in zip((1, 2), outs):
        alone, _, _ = run_batch(pb, [mem[s]], 2, **over)
        assert np.all(np.isfinite(got))
        assert np.array_equal(alone[0], got), s


# ---------------------------------------------------------------------------
# FP32 inner solves + FP64 refinement, batched: <= 1e-7 relative L2 against
# the FP64 oracle run with each member's parameters.
# ---------------------------------------------------------------------------
TOL32 = 1e-7


@pytest.mark.parametrize("S", [3, 64])
def test_batch_fp32_refine_members_match_oracle(S):
    pb = small_machine()
    mem = members_for(pb, S, seed0=1400)
    outs, st, _ = run_batch(pb, mem, pb.nsteps, precision=1)
    print(f"  S={S} inner iterations {st['pcg_iters']} refinements {st['refine_steps']}",
          flush=True)
    assert st["refine_steps"] > 0
    check = range(S) if S <= 4 else [0, 21, 63]
    for s in check:
        mb = mem[s]
        ref, _ = oracle.run(pb, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                            friction_W=mb["friction_W"], period=mb["period"])
        e = rel(outs[s], ref)
        print(f"  S={S} member {s}: rel_l2={e:.3e}", flush=True)
        assert e <= TOL32


@pytest.mark.parametrize("S", [6, 8])
def test_batch_fp32_member_alone_equals_member_in_batch(S):
    pb = small_machine()
    mem = members_for(pb, S, seed0=1500)
    outs, _, _ = run_batch(pb, mem, 2, precision=1)
    for s in (0, 4):
        alone, _, _ = run_batch(pb, [mem[s]], 2, precision=1)
        assert np.array_equal(alone[0], outs[s])


def test_ensemble_7p5mm_fp32_refine_sampled():
    """The 64-member 7.5 mm ensemble in the FP32 + refinement form, 2 steps;
    2 members checked against the FP64 oracle."""
    pb = mi.ensemble_member(0, nsteps=2, precision=mi.FP32_REFINE)
    mem = []
    for s in range(64):
        q = mi.scenario_params(s)
        rng = q[4]
        mem.append(dict(h=q[0], alpha=q[1], friction_W=q[2], period=q[3],
                        T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    outs, st, _ = run_batch(pb, mem, 2)
    print(f"  inner iterations {st['pcg_iters']} refinements {st['refine_steps']}", flush=True)
    assert st["refine_steps"] > 0
    for s in (5, 63):
        mb = mem[s]
        ref, _ = oracle.run(pb, nsteps=2, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                            friction_W=mb["friction_W"], period=mb["period"])
        e = rel(outs[s], ref)
        print(f"  member {s}: rel_l2={e:.3e}", flush=True)
        assert e <= TOL32


def test_node_block_tiles_equal_row_run_tiles():
    """With stored values (OP_VALUES), box bodies are tiled by 3 x 3 x 3 node
    blocks, other operators by runs of consecutive rows.  A stored zero
    outside the 27-point pattern (it adds no arithmetic) turns the stand into
    a general operator, so the same problem runs through both tilings: every
    row keeps its entry order, so the results must agree bitwise."""
    import paper_1707_03581_amd as m
    from dataclasses import replace
    pb = small_machine()
    mem = members_for(pb, 5, seed0=1700)
    blocks, st, _ = run_batch(pb, mem, 2, op_form=m.OP_VALUES)
    assert st["col_depth"] == 0
    b = pb.bodies[0]
    n = b.n
    rp = b.rowptr.copy()
    rp[1:] += 1
    col = np.insert(b.col, int(b.rowptr[1]), n - 1).astype(np.int32)
    K = np.insert(b.K, int(b.rowptr[1]), 0.0)
    R = np.insert(b.R, int(b.rowptr[1]), 0.0)
    pb2 = replace(pb, bodies=[replace(b, rowptr=rp, col=col, K=K, R=R), pb.bodies[1]])
    runs, st, _ = run_batch(pb2, mem, 2)
    assert st["col_depth"] == 0
    for s in range(len(mem)):
        assert np.array_equal(blocks[s], runs[s]), s


# (FP64, FP32 + refinement) x (S = 6: 16-byte rows in FP64 only; 5: 4-byte
# copies; 40: both FP64 halves, the second one partly idle)
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("S", [6, 5, 40])
def test_column_sweep_agrees_with_tiles(precision, S):
    """On box bodies the CG product runs as the column sweep; OP_VALUES runs
    the LDS tiles of the stored entries instead.  Each row's sums are formed
    in the same order, p.q is reduced in another order, so the two agree to
    rounding, and each matches the oracle."""
    import paper_1707_03581_amd as m
    pb = small_machine()
    mem = members_for(pb, S, seed0=1900)
    cols, sc, _ = run_batch(pb, mem, 2, precision=precision)
    tiles, stl, _ = run_batch(pb, mem, 2, precision=precision, op_form=m.OP_VALUES)
    assert sc["col_depth"] > 0 and stl["col_depth"] == 0
    for s in (0, S - 1):
        e = rel(cols[s], tiles[s])
        print(f"  precision {precision} S={S} member {s}: columns vs tiles {e:.3e}", flush=True)
        # (both solves stop at the same relative residual, 1e-13)
        assert e <= (1e-11 if precision == 0 else 1e-9)
    mb = mem[S - 1]
    ref, _ = oracle.run(pb, nsteps=2, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                        friction_W=mb["friction_W"], period=mb["period"])
    assert rel(cols[S - 1], ref) <= (1e-10 if precision == 0 else TOL32)


def test_per_scenario_horizons():
    """Each member advanced by its own horizon: every result equals the member
    run alone for its own number of steps, bit for bit, and its clock shows
    its own horizon; all members are active again afterwards."""
    import paper_1707_03581_amd as m
    pb = small_machine()
    mem = members_for(pb, 4, seed0=1900)
    dt = pb.scheme.dt
    horizons = [2 * dt, 4 * dt, 0.0, 3 * dt]
    ctx = m.batch_simulation(pb, mem)
    st = ctx.advance_horizons(horizons)
    assert st["steps"] == 4
    for s, hz in enumerate(horizons):
        assert ctx.get_scenario_time(s) == pytest.approx(hz)
        got = ctx.get_scenario_temperature(s, pb.N)
        alone, _, _ = run_batch(pb, [mem[s]], int(round(hz / dt)))
        assert np.array_equal(got, alone[0] if hz > 0 else mem[s]["T0"]), s
    # all of them step again afterwards
    ctx.advance_steps(1)
    assert all(ctx.get_scenario_time(s) == pytest.approx(hz + dt)
               for s, hz in enumerate(horizons))
    with pytest.raises(m.MrsdcError):
        ctx.advance_horizons([dt, 0.5 * dt, dt, dt])  # not a multiple of dt
    ctx.destroy()


def test_device_copy_out():
    import torch
    import paper_1707_03581_amd as m
    pb = small_machine()
    mem = members_for(pb, 3, seed0=1950)
    ctx = m.batch_simulation(pb, mem)
    ctx.advance_steps(2)
    for s in range(3):
        t = torch.empty(pb.N, dtype=torch.float64, device="cuda")
        ctx.get_scenario_temperature_device(s, t)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), ctx.get_scenario_temperature(s, pb.N))
    ctx.destroy()


def test_boundary_load_without_r_entries():
    """A row with a boundary load g but no R entries (its R row and column
    cleared: R stays symmetric positive semidefinite) keeps g in the column
    sweeps' zero R stencil: the sweeps agree with the tiles and the oracle."""
    import paper_1707_03581_amd as m
    from dataclasses import replace
    pb = small_machine()
    b = pb.bodies[0]
    rows = np.repeat(np.arange(b.n), np.diff(b.rowptr))
    hasR = np.zeros(b.n, bool)
    np.logical_or.at(hasR, rows, b.R != 0)
    cand = np.flatnonzero(hasR & (b.rload != 0))
    i = int(cand[len(cand) // 2])
    R = b.R.copy()
    R[(rows == i) | (b.col == i)] = 0.0
    pb2 = replace(pb, bodies=[replace(b, R=R), pb.bodies[1]])
    assert b.rload[i] != 0.0
    mem = members_for(pb2, 6, seed0=2500)
    for precision in (0, 1):
        cols, sc, _ = run_batch(pb2, mem, 2, precision=precision)
        tiles, stl, _ = run_batch(pb2, mem, 2, precision=precision, op_form=m.OP_VALUES)
        assert sc["col_depth"] > 0 and stl["col_depth"] == 0
        for s in (0, 5):
            e = rel(cols[s], tiles[s])
            print(f"  precision {precision} member {s}: columns vs tiles {e:.3e}", flush=True)
            assert e <= (1e-11 if precision == 0 else 1e-9)
    mb = mem[5]
    ref, _ = oracle.run(pb2, nsteps=2, T0=mb["T0"], h=mb["h"], alpha=mb["alpha"],
                        friction_W=mb["friction_W"], period=mb["period"])
    cols, _, _ = run_batch(pb2, mem, 2)
    assert rel(cols[5], ref) <= 1e-10
