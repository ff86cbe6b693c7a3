"""GPU parity of the single-rate SDC path (the coupling in the implicit
operator, §3 single-rate variant as compared in §5) and of implicit Euler,
through the C-ABI, against the FP64 oracle: relative L2 <= 1e-10, residuals
of every iterate to the same relative bar, on both node families, both
coupling kinds, K = 0, a degenerate first interval, residual control and the
310,042-node machine."""
import sys
from dataclasses import replace

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-10
SR = mi.SINGLE_RATE


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gpu(pb, nsteps, **over):
    import paper_1707_03581_amd as m
    ctx = m.simulation(pb, **over)
    st = ctx.advance(nsteps * pb.scheme.dt)
    T = m.get_state(ctx, pb)
    ctx.destroy()
    return T, st


def small_machine(sc, **kw):
    base = dict(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                stock_L=(0.15, 0.2, 0.3), y_offset=0.05, alpha=1000.0, friction_W=150.0,
                period=3.0, stroke=0.5, nsteps=4, h=10.0, scheme=sc)
    base.update(kw)
    return mi.machine(**base)


CASES = {
    "machine_lobatto3_K2": lambda: small_machine(mi.Scheme(M=3, family=mi.LOBATTO, P=2, K=2, dt=2.0, method=SR)),
    "machine_lobatto5_K4": lambda: small_machine(mi.Scheme(M=5, family=mi.LOBATTO, P=1, K=4, dt=5.0, method=SR)),
    "machine_equi3_K0": lambda: small_machine(mi.Scheme(M=3, family=mi.EQUI_NOLEFT, P=3, K=0, dt=2.0, method=SR)),
    "machine_implicit_euler": lambda: small_machine(mi.Scheme(M=1, family=mi.EQUI_NOLEFT, P=1, K=0, dt=1.0, method=SR), nsteps=6),
    "patch_equi2_K1": lambda: mi.patch_box(L=(0.2, 0.2, 0.5), nodes=(5, 6, 17), alpha=300.0, T_fixed=45.0, nsteps=5,
                                           scheme=mi.Scheme(M=2, family=mi.EQUI_NOLEFT, P=2, K=1, dt=2.0, method=SR)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_single_rate_matches_oracle(name):
    pb = CASES[name]()
    ref, ost, ores = oracle.run(pb, nsteps=pb.nsteps, residuals=True)
    T, st = run_gpu(pb, pb.nsteps, final_residual=1)
    e = rel(T, ref)
    K = pb.scheme.K
    gres = np.array(st["residual"][:K + 1])
    # residuals of the last step, iterate by iterate; below the solves'
    # stopping level (pcg_rtol ||M T||_2) a residual is round-off on both sides
    mass = np.concatenate([b.mass for b in pb.bodies])
    floor = 10 * pb.scheme.pcg_rtol * np.linalg.norm(mass * ref)
    dr = np.abs(gres - ores[-1]).max()
    print(f"  N={pb.N} rel_l2={e:.3e} resid gpu {gres} oracle {ores[-1]} iters gpu "
          f"{st['pcg_iters']} oracle {ost['pcg_iters']}", flush=True)
    assert st["steps"] == pb.nsteps
    assert e <= TOL
    assert dr <= 1e-8 * np.abs(ores[-1]).max() + floor


def test_single_rate_residual_control():
    """Same rule on both sides; the tolerance sits between two residual levels
    and clear of every residual the oracle meets, so both take the same
    decisions."""
    from test_gpu_adaptive import controlled
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=2, K=6, dt=2.0, method=SR, pcg_rtol=1e-14)
    pb = small_machine(sc)
    tol, sc2, ref, sweeps = controlled(pb)
    assert 0 < sweeps < pb.nsteps * sc.K
    T, st = run_gpu(replace(pb, scheme=sc2), pb.nsteps)
    print(f"  tol {tol:.3e}: sweeps gpu {st['sweeps']} oracle {sweeps} rel_l2={rel(T, ref):.3e}",
          flush=True)
    assert st["sweeps"] == sweeps
    assert rel(T, ref) <= TOL


def test_single_rate_differs_from_multirate():
    """Same machine and nodes: the two methods are different schemes (the
    coupling is implicit at the nodes in one, explicit on substeps in the
    other), each matching its own oracle."""
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=4, K=2, dt=2.0)
    pb = small_machine(sc)
    a, _ = run_gpu(pb, 3)
    b, _ = run_gpu(pb, 3, method=SR)
    ra, _ = oracle.run(pb, nsteps=3)
    rb, _ = oracle.run(pb, nsteps=3, scheme=replace(sc, method=SR))
    assert rel(a, ra) <= TOL and rel(b, rb) <= TOL
    assert rel(a, b) > 1e3 * TOL


def test_single_rate_machine_310k_sampled_steps():
    """The 310,042-node machine with single-rate SDC (Lobatto M=3, K=2, dt=5 s),
    2 steps, every node against the oracle."""
    pb = mi.machine_310k(nsteps=2)
    pb.scheme = mi.Scheme(M=3, family=mi.LOBATTO, P=1, K=2, dt=5.0, method=SR)
    ref, _ = oracle.run(pb, nsteps=2)
    T, st = run_gpu(pb, 2)
    e = rel(T, ref)
    print(f"  rel_l2={e:.3e} iters={st['pcg_iters']} max_it={st['max_iters']}", flush=True)
    assert e <= TOL
