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


def test_slot_bytes_grows_with_mesh():
    from paper_1707_03581_amd.serve import slot_bytes
    small = mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                       stock_L=(0.15, 0.2, 0.3), y_offset=0.05)
    big = mi.machine(stand_nodes=(6, 9, 23), stock_nodes=(5, 6, 9), stand_L=(0.2, 0.3, 0.9),
                     stock_L=(0.15, 0.2, 0.3), y_offset=0.05)
    assert 0 < slot_bytes(small) < slot_bytes(big)
