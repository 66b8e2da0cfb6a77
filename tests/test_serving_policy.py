"""The serving admission rule (dpk_admit_plan), exercised on the CPU as a pure function."""
import pytest

from paper_2304_09409_amd import dpk

MB = 1 << 20


@pytest.fixture(scope="module")
def plan():
    return dpk.admit_plan


def test_unbounded_budget_takes_any_idle_slot(plan):
    rc, slot, rel = plan([1, 0, 1, 0], [10 * MB] * 4, [-1] * 4, need=5 * MB)
    assert rc == 1 and slot in (1, 3) and not rel


def test_all_busy_waits(plan):
    rc, slot, rel = plan([1, 1], [MB, MB], [-1, -1], need=MB)
    assert rc == 0 and slot == -1


def test_affinity_prefers_the_simulation_slot(plan):
    rc, slot, _ = plan([0, 0, 0], [50 * MB, 5 * MB, 8 * MB], [3, 7, 9], need=6 * MB, simulation=7)
    assert rc == 1 and slot == 1


def test_smallest_sufficient_then_largest(plan):
    rc, slot, _ = plan([0, 0, 0], [20 * MB, 8 * MB, 9 * MB], [-1] * 3, need=7 * MB)
    assert rc == 1 and slot == 1
    rc, slot, _ = plan([0, 0, 0], [2 * MB, 4 * MB, 3 * MB], [-1] * 3, need=7 * MB)
    assert rc == 1 and slot == 1


def test_budget_counts_model_busy_and_idle_workspaces(plan):
    # the idle slot holding 20 grows to 30 (least growth): model 10 + busy 30 + 30 = 70 <= 100
    rc, slot, rel = plan([1, 0, 0], [30 * MB, 20 * MB, 0], [-1] * 3, need=30 * MB, budget=100 * MB,
                         model_bytes=10 * MB)
    assert rc == 1 and slot == 1 and not rel
    # an idle slot that is kept still counts: 10 + 30 (busy) + 40 (idle) + 25 = 105 > 100, and
    # freeing the idle one gives 65: admit with release
    rc, slot, rel = plan([1, 0, 0], [30 * MB, 40 * MB, 25 * MB], [-1] * 3, need=25 * MB, budget=100 * MB,
                         model_bytes=10 * MB)
    assert rc == 1 and slot == 2 and rel
    # slot 1 grows to 50: 10 + 30 + 15 (idle slot 2) + 50 = 105 > 100; freeing slot 2 gives 90
    rc, slot, rel = plan([1, 0, 0], [30 * MB, 20 * MB, 15 * MB], [-1] * 3, need=50 * MB, budget=100 * MB,
                         model_bytes=10 * MB)
    assert rc == 1 and slot == 1 and rel
    # 10 + 30 (busy) + 70 > 100 even after freeing: wait for the busy slot
    rc, slot, rel = plan([1, 0, 0], [30 * MB, 20 * MB, 0], [-1] * 3, need=70 * MB, budget=100 * MB,
                         model_bytes=10 * MB)
    assert rc == 0 and slot == -1


def test_frame_larger_than_budget_is_rejected(plan):
    rc, _, _ = plan([0, 0], [0, 0], [-1, -1], need=95 * MB, budget=100 * MB, model_bytes=10 * MB)
    assert rc == dpk.DPK_E_BUDGET
