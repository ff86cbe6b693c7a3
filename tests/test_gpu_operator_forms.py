"""GPU parity of every storage form of the operator L = K + hR (§2, eq.
femDiscr) that the CG product, the F_j evaluation, the predictor init and the
refinement update read, against the CPU FP64 oracle.

Forms: value array, 1-byte value dictionary, 2-byte packed offset + index,
1-byte row patterns; 16-bit column offsets or int32 columns.  The library
picks the most compact form that applies; `op_form` forces one, and the
advance reports the one it read.  All forms hold the same entries in the same
order, so within one precision every form gives the same field bit for bit.

Meshes: a uniform machine (every form applies), the same machine on
irregular tensor meshes (more than 256 distinct values: the value array), and
that machine with each body's nodes in a seeded random order (column offsets
beyond 16 bits at full size: int32 columns).
"""
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-7


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


def run(pb, nsteps, **over):
    m = pkg()
    ctx = m.simulation(pb, **over)
    st = ctx.advance(nsteps * pb.scheme.dt)
    T = m.get_state(ctx, pb)
    ctx.destroy()
    return T, st


def small(precision, **kw):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0, precision=precision)
    # 4,961 + 704 rows: 89 SELL slices, the last one ragged; 4 cm cells in both
    # bodies, so the uniform operator holds 13 distinct values (every form applies)
    return mi.machine(**SMALL, scheme=sc, nsteps=3, **kw)


SMALL = dict(stand_nodes=(11, 11, 41), stock_nodes=(8, 8, 11), stand_L=(0.4, 0.4, 1.6),
             stock_L=(0.28, 0.28, 0.4), y_offset=0.06, period=3.0, stroke=0.8)


FORMS = [("values", "OP_VALUES", 0), ("values_col32", "OP_VALUES", 1), ("dict", "OP_DICT", 0),
         ("dict_col32", "OP_DICT", 1), ("packed", "OP_PACKED", 0), ("patterns", "OP_PATTERNS", 0)]

_ref_cache = {}


def oracle_ref(precision):
    if precision not in _ref_cache:
        pb = small(precision)
        _ref_cache[precision] = oracle.run(pb, nsteps=pb.nsteps)[0]
    return _ref_cache[precision]


_field_cache = {}


@pytest.mark.parametrize("precision", [mi.FP64, mi.FP32_REFINE], ids=["fp64", "fp32refine"])
@pytest.mark.parametrize("name,form,col32", FORMS, ids=[f[0] for f in FORMS])
def test_every_form_matches_oracle(name, form, col32, precision):
    m = pkg()
    pb = small(precision)
    code = getattr(m, form) | (m.OP_COL32 if col32 else 0)
    T, st = run(pb, pb.nsteps, op_form=code)
    e = rel(T, oracle_ref(precision))
    print(f"  {name}: op_form={st['op_form']} col_bytes={st['col_bytes']} rel_l2={e:.3e} "
          f"iters={st['pcg_iters']}", flush=True)
    assert st["op_form"] == getattr(m, form)
    assert st["col_bytes"] == (4 if col32 else 2)
    assert e <= (TOL64 if precision == mi.FP64 else TOL32)
    # same entries, same order: the same field as every other form, bit for bit
    first = _field_cache.setdefault(precision, (name, T))
    assert np.array_equal(T, first[1]), f"{name} differs from {first[0]}"


def test_auto_picks_row_patterns_on_uniform_mesh():
    m = pkg()
    pb = small(mi.FP64)
    T, st = run(pb, 1)
    assert st["op_form"] == m.OP_PATTERNS and st["col_bytes"] == 2


def test_forms_that_do_not_apply_are_rejected():
    m = pkg()
    pb = small(mi.FP64, jitter=0.2)
    for form in (m.OP_DICT, m.OP_PACKED, m.OP_PATTERNS):
        ctx = m.simulation(pb, op_form=form)
        with pytest.raises(m.MrsdcError) as ei:
            ctx.advance(pb.scheme.dt)
        assert ei.value.status == m.EINVAL
        ctx.destroy()
    # patterns need 16-bit offsets
    ctx = m.simulation(small(mi.FP64), op_form=m.OP_PATTERNS | m.OP_COL32)
    with pytest.raises(m.MrsdcError):
        ctx.advance(pb.scheme.dt)
    ctx.destroy()
    # batched contexts take OP_AUTO or OP_VALUES only
    for form in (m.OP_DICT, m.OP_PACKED, m.OP_PATTERNS, m.OP_VALUES | m.OP_COL32):
        ctx = m.batch_simulation(small(mi.FP64), [dict(h=10.0, alpha=1000.0, friction_W=100.0,
                                                       period=3.0, T0=small(mi.FP64).T0)],
                                 op_form=form)
        with pytest.raises(m.MrsdcError) as ei:
            ctx.advance_steps(1)
        assert ei.value.status == m.EINVAL
        ctx.destroy()


@pytest.mark.parametrize("precision", [mi.FP64, mi.FP32_REFINE], ids=["fp64", "fp32refine"])
@pytest.mark.parametrize("renumber", [False, True], ids=["ordered", "renumbered"])
def test_irregular_small_mesh(renumber, precision):
    m = pkg()
    pb = small(precision, jitter=0.2, renumber=renumber)
    ref, _ = oracle.run(pb, nsteps=pb.nsteps)
    T, st = run(pb, pb.nsteps)
    e = rel(T, ref)
    print(f"  op_form={st['op_form']} col_bytes={st['col_bytes']} rel_l2={e:.3e}", flush=True)
    assert st["op_form"] == m.OP_VALUES and st["col_bytes"] == 2
    assert e <= (TOL64 if precision == mi.FP64 else TOL32)


@pytest.mark.parametrize("precision", [mi.FP64, mi.FP32_REFINE], ids=["fp64", "fp32refine"])
@pytest.mark.parametrize("renumber", [False, True], ids=["ordered", "renumbered"])
def test_irregular_machine_310k(renumber, precision):
    """The 310,042-node machine on irregular meshes, 2 steps: the value array
    with 16-bit offsets (ordered) or int32 columns (renumbered: offsets up to
    the body size)."""
    m = pkg()
    pb = mi.machine_310k_irregular(nsteps=2, renumber=renumber)
    pb.scheme.precision = precision
    ref, _ = oracle.run(pb, nsteps=2)
    T, st = run(pb, 2)
    e = rel(T, ref)
    print(f"  op_form={st['op_form']} col_bytes={st['col_bytes']} rel_l2={e:.3e} "
          f"iters={st['pcg_iters']}", flush=True)
    assert st["op_form"] == m.OP_VALUES
    assert st["col_bytes"] == (4 if renumber else 2)
    assert e <= (TOL64 if precision == mi.FP64 else TOL32)


@pytest.mark.parametrize("renumber", [False, True], ids=["ordered", "renumbered"])
def test_irregular_batch(renumber):
    """Batched ensemble (S = 3) on the irregular small machine, each member
    against the oracle run with its own parameters (FP32 + refinement)."""
    m = pkg()
    pb = small(mi.FP32_REFINE, jitter=0.2, renumber=renumber)
    members = []
    for s in range(3):
        h, alpha, pf, period, rng = mi.scenario_params(s)
        members.append(dict(h=h, alpha=alpha, friction_W=pf, period=period,
                            T0=20.0 + rng.uniform(-0.5, 0.5, size=pb.N)))
    ctx = m.batch_simulation(pb, members)
    ctx.advance_steps(2)
    for s, mb in enumerate(members):
        T = ctx.get_scenario_temperature(s, pb.N)
        q = mi.machine(**dict(SMALL, period=mb["period"]), h=mb["h"], alpha=mb["alpha"],
                       friction_W=mb["friction_W"], scheme=pb.scheme, nsteps=2, jitter=0.2,
                       renumber=renumber)
        q.T0 = mb["T0"]
        ref, _ = oracle.run(q, nsteps=2)
        e = rel(T, ref)
        print(f"  member {s}: rel_l2={e:.3e}", flush=True)
        assert e <= TOL32
    ctx.destroy()
