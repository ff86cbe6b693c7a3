"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point declared in include/mrsdc.h, and its host-only quadrature
agrees with the oracle's independent derivation (paper §3 weight definitions)."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mrsdc.h")).read()
    return sorted(set(re.findall(r"\b(mrsdc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1707_03581_amd as m
    L = m.lib()
    syms = declared_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("M,fam,P,dt", [(3, 0, 10, 1.0), (5, 0, 5, 5.0), (5, 0, 20, 5.0),
                                         (4, 1, 6, 2.0), (8, 0, 3, 1.0), (2, 1, 1, 1.0)])
def test_library_quadrature_matches_oracle(M, fam, P, dt):
    import paper_1707_03581_amd as m
    if fam == 0 and M > 5:
        # oracle has closed-form Lobatto nodes only up to M = 5: check identities
        tau, s, shat, stil, spq = m.quadrature(M, fam, P, dt)
        for k in range(1, M + 1):
            assert s[k].sum() == pytest.approx(tau[k] - tau[k - 1], abs=1e-14)
        return
    got = m.quadrature(M, fam, P, dt)
    ref = oracle.weights(M, fam, P, dt)
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 4e-16 * max(np.abs(r).max(), 1e-300)


def test_quadrature_rejects_bad_arguments():
    import paper_1707_03581_amd as m
    with pytest.raises(m.MrsdcError):
        m.quadrature(1, 0, 2)
    with pytest.raises(m.MrsdcError):
        m.quadrature(3, 0, 0)
    with pytest.raises(m.MrsdcError):
        m.quadrature(3, 7, 2)


def test_config_defaults_and_create_validation():
    import paper_1707_03581_amd as m
    cfg = m.default_config()
    assert (cfg.M, cfg.P, cfg.K, cfg.precision) == (3, 2, 2, m.FP64)
    assert cfg.pcg_rtol == 1e-13
    bad = m.default_config(M=1)
    with pytest.raises(m.MrsdcError) as e:
        m.Context(bad)
    assert e.value.status == m.EINVAL
    assert cfg.method == m.MULTIRATE


@pytest.mark.parametrize("over", [dict(method=m_) for m_ in (2, -1)] +
                         [dict(method=1, precision=1), dict(method=1, M=1, node_family=0)])
def test_create_rejects_bad_method(over):
    """Unknown methods, the single-rate method outside FP64, and one Lobatto
    node are rejected before any device is touched."""
    import paper_1707_03581_amd as m
    with pytest.raises(m.MrsdcError) as e:
        m.Context(m.default_config(**over))
    assert e.value.status == m.EINVAL


def test_batch_rejects_single_rate():
    import paper_1707_03581_amd as m
    with pytest.raises(m.MrsdcError) as e:
        m.BatchContext(m.default_config(method=m.SINGLE_RATE), 4)
    assert e.value.status == m.EINVAL
