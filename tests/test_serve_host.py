"""Host-side pieces of the serving loop that need no GPU."""
import mrsdc_inputs as mi


def test_trace_is_seeded_and_poisson_like():
    a = mi.serving_trace(64)
    b = mi.serving_trace(64)
    assert [r["arrival"] for r in a] == [r["arrival"] for r in b]
    gaps = [a[i + 1]["arrival"] - a[i]["arrival"] for i in range(63)]
    assert 0.02 < sum(gaps) / len(gaps) < 0.08  # mean 1/20 s
    assert {r["level"] for r in a} <= set(mi.MESH_LEVELS)
    assert all(12 <= r["nsteps"] <= 360 for r in a)


def test_pool_plan_fits_the_budget_smallest_levels_first():
    from paper_1707_03581_amd.serve import plan_pools
    lb = {"5mm": (900, 300), "2cm": (20, 5), "1cm": (150, 40)}
    # room for everything: every level gets its full pool
    assert plan_pools(lb, 10**6, 4) == {"2cm": 4, "1cm": 4, "5mm": 4}
    # 2cm: 20 + 4*5 = 40; 1cm: 150 + 4*40 = 310; 5mm needs 1200 for one slot
    plan = plan_pools(lb, 40 + 310 + 1199, 4)
    assert plan == {"2cm": 4, "1cm": 4, "5mm": 0}
    # a budget that cuts a pool short
    plan = plan_pools(lb, 40 + 150 + 2 * 40 + 39, 4)
    assert plan == {"2cm": 4, "1cm": 2, "5mm": 0}
    for budget in (0, 10, 500, 1234, 5000, 10**6):
        plan = plan_pools(lb, budget, 8)
        held = sum(lb[n][0] + k * lb[n][1] for n, k in plan.items() if k)
        assert held <= budget
    # the plan depends on the configured levels only
    assert plan_pools(dict(reversed(list(lb.items()))), 1549, 4) == plan_pools(lb, 1549, 4)
