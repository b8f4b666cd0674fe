"""Host logic of the serving loop (no GPU): which admitted requests run in
the next group launch under each policy, and the device memory a request
is charged against the budget."""
import pytest

from paper_1505_03271_amd import cell_bytes
from paper_1505_03271_amd.serve import POLICIES, Server, request_bytes


def _server(policy, min_cells=8e6, max_sims=128, age_s=1e9):
    """A Server with its scheduling state only (no group, no device)."""
    s = object.__new__(Server)
    s.policy, s.min_cells, s.max_sims, s.age_s = policy, float(min_cells), max_sims, float(age_s)
    return s


def _resident(spec):
    """spec: (id, n, steps left, admission time)"""
    return {k: dict(req=dict(id=k, n=n), left=left, admitted=t) for k, n, left, t in spec}


def test_all_runs_every_resident_request_in_admission_order():
    res = _resident([(5, 512, 100, 0.3), (2, 128, 9000, 0.1), (7, 1024, 50, 0.2)])
    assert _server("all")._choose(res, 1.0) == [2, 7, 5]
    assert _server("all", max_sims=2)._choose(res, 1.0) == [2, 7]


def test_srpt_takes_the_least_remaining_work_until_min_cells():
    # remaining work n^2 * left: id 1: 4.2e6, id 2: 1.6e8, id 3: 5.2e6, id 4: 1.3e7
    res = _resident([(1, 256, 64, 0.0), (2, 1024, 150, 0.1), (3, 512, 20, 0.2), (4, 128, 800, 0.3)])
    s = _server("srpt", min_cells=300_000)
    # 256^2 + 512^2 = 327 680 cells >= 300 000 after the two shortest
    assert s._choose(res, 1.0) == [1, 3]
    assert _server("srpt", min_cells=1)._choose(res, 1.0) == [1]
    assert _server("srpt", min_cells=1e12)._choose(res, 1.0) == [1, 3, 4, 2]
    assert _server("srpt", min_cells=1e12, max_sims=3)._choose(res, 1.0) == [1, 3, 4]


def test_srpt_breaks_ties_by_admission():
    res = _resident([(8, 256, 10, 0.5), (9, 256, 10, 0.2)])
    assert _server("srpt", min_cells=1)._choose(res, 1.0) == [9]


def test_policy_names_and_request_bytes():
    assert POLICIES == ("all", "srpt")
    with pytest.raises(ValueError):
        Server(policy="fifo")
    with pytest.raises(ValueError):
        Server(age_s=0.0)
    # two population states plus the per-row metric and a small fixed part
    assert request_bytes(1000, "bf16s") == 2 * 1000 * 1000 * 44 + 64 * 1000 + 4096
    assert cell_bytes("f32") == 72 and cell_bytes("bf16") == 36 and cell_bytes("bf16s", thermal=False) == 24


def test_srpt_ages_waiting_requests_into_the_running_set():
    """Remaining work is divided by 1 + wait / age_s: a larger request that
    has waited ranks ahead of a smaller one that just arrived."""
    # work 256^2 * 1000 = 6.6e7 (admitted at 0 s) and 128^2 * 1000 = 1.6e7 (at 9.9 s)
    res = _resident([(1, 256, 1000, 0.0), (2, 128, 1000, 9.9)])
    assert _server("srpt", min_cells=1, age_s=1e9)._choose(res, 10.0) == [2]
    # at 10 s with age_s = 1: 6.6e7 / 11 = 6.0e6 against 1.6e7 / 1.1 = 1.5e7
    assert _server("srpt", min_cells=1, age_s=1.0)._choose(res, 10.0) == [1]
