"""GPU parity of the thermo-elastic deformation (§5: K_u factorised once,
forward and backward block solves per output) through the C-ABI.

Bar: relative L2 <= 1e-10 against the oracle's sparse direct solve on meshes
it solves in milliseconds (several blocks, a ragged last block, padding, a
single pivot tile, and 7 or 8 tiles of 64 per block, so that the symmetric
block product has full and ragged strips of tiles), both bodies of a machine, outputs after time steps on one
factorisation; the closed-form free expansion under uniform heating; and on
the 270,641-node stand (811,923 DOFs) the relative residual
||K_u u - f|| / ||f||, which a backward-stable solve keeps near
(cond K_u) eps ~ 1e-10 (measured there: see the printed value), <= 1e-8."""
import sys

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle.deform as od
from mrsdc_inputs.elastic import elastic_box

pytestmark = pytest.mark.gpu
TOL = 1e-10
ROLLERS = (("x0", (0,)), ("y0", (1,)), ("z0", (2,)))


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def single(nodes, L=(0.2, 0.25, 0.5), seed=0):
    pb = mi.patch_box(L=L, nodes=nodes, nsteps=2,
                      scheme=mi.Scheme(M=3, family=mi.LOBATTO, P=2, K=1, dt=1.0))
    pb.T0 = 20.0 + np.random.default_rng(seed).uniform(-4.0, 6.0, size=pb.N)
    return pb


@pytest.mark.parametrize("nodes", [(5, 6, 9), (2, 2, 3), (7, 5, 12), (4, 4, 2), (12, 10, 8),
                                   (14, 11, 9)])
def test_deformation_matches_oracle(nodes):
    import paper_1707_03581_amd as m
    pb = single(nodes)
    el = elastic_box(pb.bodies[0])
    ctx = m.simulation(pb)
    info = ctx.deform_setup(el)
    u = ctx.deform()
    ref = od.deform(el, pb.T0)
    e = rel(u, ref)
    print(f"  n={el.n} block={info['block']} padded={info['padded_block']} "
          f"blocks={info['nblocks']} rel_l2={e:.3e}", flush=True)
    assert e <= TOL
    ctx.destroy()


def test_uniform_heating_closed_form():
    import paper_1707_03581_amd as m
    pb = single((6, 7, 15))
    b = pb.bodies[0]
    el = elastic_box(b, fixed=ROLLERS)
    pb.T0 = np.full(pb.N, 20.0 + 9.0)
    ctx = m.simulation(pb)
    ctx.deform_setup(el)
    u = ctx.deform()
    ctx.destroy()
    exact = (el.alpha * 9.0 * b.coords).ravel()[el.free]
    assert np.abs(u - exact).max() <= 1e-10 * np.abs(exact).max()


@pytest.mark.parametrize("body", [0, 1])
def test_machine_body_after_steps(body):
    """Either body of a machine, from the device-resident temperature after
    time steps; two outputs on one factorisation."""
    import paper_1707_03581_amd as m
    import oracle
    pb = mi.machine(stand_nodes=(5, 7, 13), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                    stock_L=(0.15, 0.2, 0.3), nsteps=2,
                    scheme=mi.Scheme(M=3, family=mi.LOBATTO, P=2, K=1, dt=2.0))
    el = elastic_box(pb.bodies[body])
    ctx = m.simulation(pb)
    ctx.deform_setup(el, body=body)
    off = pb.offsets
    outs = []
    for steps in (1, 2):
        ctx.advance(pb.scheme.dt)
        T = m.get_state(ctx, pb)
        outs.append((ctx.deform(), T[off[body]:off[body + 1]]))
    ctx.destroy()
    Tref, _ = oracle.run(pb, nsteps=2)
    assert rel(outs[1][1], Tref[off[body]:off[body + 1]]) <= TOL
    solve = od.Deformation(el)
    for u, T in outs:
        e = rel(u, solve(T))
        print(f"  body {body}: rel_l2={e:.3e}", flush=True)
        assert e <= TOL


def test_error_paths():
    import paper_1707_03581_amd as m
    pb = single((4, 4, 5))
    el = elastic_box(pb.bodies[0])
    ctx = m.simulation(pb)
    with pytest.raises(m.MrsdcError) as e:
        ctx._df_n = el.n
        ctx.deform()
    assert e.value.status == m.ESTATE
    neg = type(el)(**{**el.__dict__, "K": -el.K})
    with pytest.raises(m.MrsdcError) as e:
        ctx.deform_setup(neg)
    assert e.value.status == m.EINVAL and "positive definite" in str(e.value)
    bad = type(el)(**{**el.__dict__, "g_col": el.g_col + pb.N})
    with pytest.raises(m.MrsdcError) as e:
        ctx.deform_setup(bad)
    assert e.value.status == m.EINVAL
    ctx.deform_setup(el)  # a valid registration after the failures
    assert rel(ctx.deform(), od.deform(el, pb.T0)) <= TOL
    ctx.destroy()


def test_stand_1cm_residual():
    """The 1 cm stand (41 x 41 x 161 nodes, clamped floor), temperature of the
    310,042-node machine after 2 steps."""
    import paper_1707_03581_amd as m
    pb = mi.machine_310k(nsteps=2)
    el = elastic_box(pb.bodies[0])
    ctx = m.simulation(pb)
    info = ctx.deform_setup(el)
    ctx.advance(2 * pb.scheme.dt)
    T = ctx.get_temperature(0, pb.bodies[0].n)
    u = ctx.deform()
    ctx.destroy()
    f = el.gcsr() @ (T - el.T_ref)
    r = np.linalg.norm(el.csr() @ u - f) / np.linalg.norm(f)
    print(f"  n={el.n} block={info['block']} blocks={info['nblocks']} "
          f"factor {info['factor_ms']:.0f} ms, {info['factor_bytes'] / 2**30:.1f} GiB; "
          f"relative residual {r:.3e}", flush=True)
    assert r <= 1e-8
