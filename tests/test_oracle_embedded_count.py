"""Pin of the reading of the machine workloads' "20 fast substeps" (embedded
nodes per standard interval, §3 "Multi-rate SDC").

The equidistant no-left embedded rule of §3 extrapolates to the left end of
each interval, so its weights grow quickly with P (max |hat s| / dtau about
2.3e3 at P = 20).  With the contact coefficient of the machine workloads
(alpha = 1000 W/m^2K) and dt = 5 s, the correction sweep then amplifies the
residual (eq. residual) instead of reducing it, which contradicts the
contraction per sweep that §3 states for the method.  Reading 20 substeps per
5 s step over the 4 non-degenerate Lobatto intervals gives P = 5 per interval,
for which the sweeps contract as §3 describes.  This test fixes both halves
of that argument on a coarse copy of the machine (5 cm nodes).
"""
import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle


def coarse_machine(P):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=P, K=4, dt=5.0)
    return mi.machine(stand_nodes=(9, 9, 33), stock_nodes=(7, 7, 9), scheme=sc, nsteps=2)


@pytest.mark.parametrize("P", [5, 8])
def test_sweeps_contract_at_the_read_P(P):
    p = coarse_machine(P)
    T, _, res = oracle.run(p, nsteps=2, residuals=True)
    for r in res:  # every step: each sweep lowers the residual, by 1e3 overall
        assert np.all(np.diff(r) < 0), r
        assert r[-1] < 1e-3 * r[0], r
    assert np.abs(T - 20.0).max() < 2.0  # the field stays physical


def test_sweeps_diverge_at_twenty_per_interval():
    p = coarse_machine(20)
    T, _, res = oracle.run(p, nsteps=2, residuals=True)
    for r in res:
        assert np.all(np.diff(r) > 0), r  # every sweep amplifies the residual
    assert res[-1, -1] > 1e6 * res[0, 0]
    assert np.abs(T).max() > 1e3  # and the temperature blows up


def test_machine_workloads_use_five_per_interval():
    assert mi.machine_310k(nsteps=1).scheme.P == 5
    assert mi.ensemble_member(0, stand_nodes=(5, 5, 9), stock_nodes=(4, 4, 5)).scheme.P == 5
    # the single box states "per node interval": P = 10
    assert mi.box_patch_2673().scheme.P == 10
