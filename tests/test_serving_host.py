"""Host-side policy of the serving loop: admission by device-memory footprint,
first-come-first-served leading request, merging by key, size caps; and the
seeded request stream."""
import numpy as np

from paper_1507_04769_amd import serving as SV


def solve(rid, n, N=64, m=3):
    return SV.SolveRequest(rid, 0.0, np.zeros((n, 6)), N, m, 20.0)


def query(rid, n, level=4, fp32=False):
    return SV.QueryRequest(rid, 0.0, np.zeros((n, 6)), level, fp32)


def unit_footprint(key, n):
    return 100 * n


def test_merges_same_key_behind_oldest():
    a = SV.Admission(hbm_budget=10**9, footprint=unit_footprint)
    pend = [query(0, 5), solve(1, 3), query(2, 7), query(3, 1, fp32=True), query(4, 2)]
    key, chosen, n, nbytes = a.select(pend, used=0)
    assert key == ("query", 4, False)
    assert [r.rid for r in chosen] == [0, 2, 4] and n == 14 and nbytes == 1400


def test_size_cap_and_budget_stop_merging():
    a = SV.Admission(hbm_budget=10**9, max_bvps=10, footprint=unit_footprint)
    pend = [solve(0, 4), solve(1, 5), solve(2, 3), solve(3, 1)]
    _, chosen, n, _ = a.select(pend, used=0)
    assert [r.rid for r in chosen] == [0, 1] and n == 9  # the next one would pass the cap of 10
    b = SV.Admission(hbm_budget=1000, footprint=unit_footprint)
    _, chosen, n, _ = b.select(pend, used=100)
    assert [r.rid for r in chosen] == [0, 1]  # 100 + 900 <= 1000, adding 3 more would not fit


def test_waits_for_memory_and_oversized_runs_alone():
    a = SV.Admission(hbm_budget=1000, footprint=unit_footprint)
    assert a.select([solve(0, 8)], used=300) is None  # 300 + 800 > 1000: wait
    key, chosen, n, nbytes = a.select([solve(0, 20), solve(1, 1)], used=0)
    assert [r.rid for r in chosen] == [0] and nbytes == 2000  # larger than the budget: alone on an idle device
    assert a.select([], used=0) is None


def test_unmerged_policy_takes_one():
    a = SV.Admission(hbm_budget=10**9, merge=False, footprint=unit_footprint)
    _, chosen, _, _ = a.select([query(0, 5), query(1, 5)], used=0)
    assert [r.rid for r in chosen] == [0]


def test_footprint_grows_with_size_and_precision():
    assert SV.footprint(("query", 4, True), 1000) == 1000 * 4 * 9
    assert SV.footprint(("query", 4, False), 1000) == 1000 * 8 * 9
    f1 = SV.footprint(("solve", 3, 64, 20.0), 10)
    assert SV.footprint(("solve", 3, 64, 20.0), 20) > f1 > 0
    assert SV.footprint(("solve", 3, 512, 20.0), 10) > f1


def test_request_stream_is_seeded_and_in_range():
    a = SV.request_stream(200, rate=100.0, seed=1, levels=(3, 4, 5))
    b = SV.request_stream(200, rate=100.0, seed=1, levels=(3, 4, 5))
    assert [r.key() for r in a] == [r.key() for r in b]
    assert all(np.array_equal(getattr(x, "x0", getattr(x, "xq", None)), getattr(y, "x0", getattr(y, "xq", None)))
               for x, y in zip(a, b))
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0) and abs(len(t) / t[-1] - 100.0) < 30.0
    for r in a:
        if isinstance(r, SV.SolveRequest):
            assert 1 <= len(r.x0) <= 512 and r.N in (64, 128, 256, 512) and r.m in (2, 3)
            assert r.T == 20.0
        else:
            assert 1 <= len(r.xq) <= 100_000 and r.level in (3, 4, 5)
    kinds = {type(r).__name__ for r in a}
    assert kinds == {"SolveRequest", "QueryRequest"}


def test_stream_caps_let_other_classes_lead():
    a = SV.Admission(hbm_budget=10**9, footprint=unit_footprint, stream_caps={"solve-2wheel": 1})
    pend = [solve(0, 4, m=2), solve(1, 3, m=2), query(2, 5), solve(3, 2)]
    key, chosen, _, _ = a.select(pend, used=0, busy={})
    assert SV.work_class(key) == "solve-2wheel" and [r.rid for r in chosen] == [0, 1]
    # with the two-wheel class at its cap the oldest request of another class leads
    key, chosen, _, _ = a.select(pend, used=0, busy={"solve-2wheel": 1})
    assert key == ("query", 4, False) and [r.rid for r in chosen] == [2]
    assert a.select(pend[:2], used=0, busy={"solve-2wheel": 1}) is None
    assert SV.work_class(("solve", 3, 64, 20.0)) == "solve"


def test_available_classes():
    a = SV.Admission(hbm_budget=10**9, footprint=unit_footprint)
    pend = [solve(0, 4, m=2), query(1, 5), solve(2, 3)]
    # the two-wheel class has no free stream: the oldest request of a class that has one leads
    key, chosen, _, _ = a.select(pend, used=0, busy={}, avail={"query", "solve"})
    assert key == ("query", 4, False) and [r.rid for r in chosen] == [1]
    assert a.select(pend[:1], used=0, busy={}, avail={"query", "solve"}) is None
    b = SV.Admission(hbm_budget=10**9, footprint=unit_footprint, size_caps={"solve-2wheel": 5})
    _, chosen, n, _ = b.select([solve(0, 4, m=2), solve(1, 3, m=2)], used=0)
    assert [r.rid for r in chosen] == [0] and n == 4  # 4 + 3 would pass the class's size cap
