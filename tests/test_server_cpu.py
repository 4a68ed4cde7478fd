"""The server's scheduler on its fake backend (no GPU, no device call): a
request of dimension n is held by a worker for n microseconds and charges
100 n bytes against its reservation.  Admission is FIFO, bounded by the slots
and by the device-memory budget; a request whose reservation is too small
grows it in place while the budget has room, else runs again with four times
as much; a full queue refuses submissions."""

import time

import pytest


@pytest.fixture(scope="module")
def B():
    from paper_2208_05683_amd import binding

    return binding


def _view(B, n):
    v = B.fps_csr_view()
    v.n, v.nnz = n, 0
    v.row_ptr = 0x1000  # never read by the fake backend
    v.col = v.val = None
    return v


C = [1.0, 1.0, 0.5]


def _run(B, sv, ns, hints):
    tickets = [B.fps_server_submit(sv, _view(B, n), C, 2, 1, 0.0, h) for n, h in zip(ns, hints)]
    for t in tickets:
        assert B.fps_server_wait(sv, t, 20000) in (B.FPS_REQ_DONE, B.FPS_REQ_FAILED)
    return tickets, [B.fps_server_request_info(sv, t) for t in tickets]


def test_fifo_within_slots_and_budget(B):
    sv = B.fps_server_create(slots=4, hbm_budget=10_000_000, fake_backend=True)
    try:
        ns = [2000 + 137 * (k % 7) for k in range(40)]
        tickets, info = _run(B, sv, ns, [100 * n for n in ns])
        st = B.fps_server_get_stats(sv)
        assert st["completed"] == 40 and st["failed"] == 0 and st["retries"] == 0
        assert st["peak_running"] <= 4 and st["peak_reserved"] <= st["budget"]
        starts = [x["t_start_ns"] for x in info]
        assert starts == sorted(starts)  # admitted in submission order
        for x in info:
            assert x["state"] == B.FPS_REQ_DONE and x["attempts"] == 1
            assert x["t_submit_ns"] <= x["t_start_ns"] <= x["t_done_ns"]
            assert x["t_done_ns"] - x["t_start_ns"] >= 1000 * x["n"]
        for t in tickets:
            B.fps_server_release(sv, t)
        assert B.fps_server_get_stats(sv)["reserved"] == 0
    finally:
        B.fps_server_destroy(sv)


def test_memory_budget_limits_concurrency(B):
    # 4 slots, but the budget holds only two reservations of 100 n at a time
    n = 3000
    sv = B.fps_server_create(slots=4, hbm_budget=250 * n, fake_backend=True)
    try:
        tickets, info = _run(B, sv, [n] * 12, [100 * n] * 12)
        st = B.fps_server_get_stats(sv)
        assert st["completed"] == 12
        assert st["peak_running"] == 2 and st["peak_reserved"] <= 250 * n
    finally:
        B.fps_server_destroy(sv)


def test_too_small_reservation_is_retried_larger(B):
    sv = B.fps_server_create(slots=2, hbm_budget=1 << 40, fake_backend=True, no_grow=True)
    try:
        n = 1000
        tickets, info = _run(B, sv, [n, n], [10 * n, 100 * n])
        assert info[0]["state"] == B.FPS_REQ_DONE and info[0]["attempts"] == 3  # 10 n -> 40 n -> 160 n
        assert info[0]["reserve"] == 160 * n
        assert info[1]["attempts"] == 1
        assert B.fps_server_get_stats(sv)["retries"] == 2
    finally:
        B.fps_server_destroy(sv)


def test_too_small_reservation_grows_in_place(B):
    sv = B.fps_server_create(slots=2, hbm_budget=1 << 40, fake_backend=True)
    try:
        n = 1000
        tickets, info = _run(B, sv, [n, n], [10 * n, 100 * n])
        assert info[0]["state"] == B.FPS_REQ_DONE and info[0]["attempts"] == 1
        assert info[0]["reserve"] == 125 * n  # a quarter more than the 100 n it needed
        assert info[1]["attempts"] == 1 and info[1]["reserve"] == 100 * n
        st = B.fps_server_get_stats(sv)
        assert st["retries"] == 0 and st["grows"] == 1 and st["completed"] == 2
        for t in tickets:
            B.fps_server_release(sv, t)
        assert B.fps_server_get_stats(sv)["reserved"] == 0
    finally:
        B.fps_server_destroy(sv)


def test_growth_refused_by_a_full_budget_runs_again(B):
    # A (100 n, enough) runs for n microseconds; B starts beside it with 10 n
    # and needs 100 n: 100 n + 100 n is past the budget of 130 n, so B goes
    # back to the queue with 40 n, which fits only once A is done; then it
    # grows in place (to 125 n)
    n = 20000
    sv = B.fps_server_create(slots=2, hbm_budget=130 * n, fake_backend=True)
    try:
        tickets, info = _run(B, sv, [n, n], [100 * n, 10 * n])
        assert [x["state"] for x in info] == [B.FPS_REQ_DONE, B.FPS_REQ_DONE]
        assert info[0]["attempts"] == 1
        assert info[1]["attempts"] == 2 and info[1]["reserve"] == 125 * n
        assert info[1]["t_start_ns"] >= info[0]["t_done_ns"]
        st = B.fps_server_get_stats(sv)
        assert st["retries"] == 1 and st["grows"] == 1 and st["peak_reserved"] <= 130 * n
    finally:
        B.fps_server_destroy(sv)


def test_request_beyond_budget_fails(B):
    n = 1000
    sv = B.fps_server_create(slots=1, hbm_budget=50 * n, fake_backend=True)
    try:
        tickets, info = _run(B, sv, [n, 100], [10 * n, 0])
        assert info[0]["state"] == B.FPS_REQ_FAILED and info[0]["status"] == B.FPS_ERR_CAPACITY
        assert info[0]["reserve"] == 50 * n  # grew up to the whole budget, then gave up
        assert info[1]["state"] == B.FPS_REQ_DONE  # the queue moved on
    finally:
        B.fps_server_destroy(sv)


def test_full_queue_refuses_and_recovers(B):
    sv = B.fps_server_create(slots=1, hbm_budget=1 << 40, max_queue=3, fake_backend=True)
    try:
        first = B.fps_server_submit(sv, _view(B, 200_000), C, 2, 1, 0.0, 0)  # 0.2 s
        time.sleep(0.05)  # running now, queue empty
        waiting = [B.fps_server_submit(sv, _view(B, 1000), C, 2, 1, 0.0, 0) for _ in range(3)]
        with pytest.raises(B.FpsError) as e:
            B.fps_server_submit(sv, _view(B, 1000), C, 2, 1, 0.0, 0)
        assert e.value.status == B.FPS_ERR_CAPACITY
        assert B.fps_server_get_stats(sv)["refused"] == 1
        for t in [first] + waiting:
            assert B.fps_server_wait(sv, t, 20000) == B.FPS_REQ_DONE
        later = B.fps_server_submit(sv, _view(B, 1000), C, 2, 1, 0.0, 0)
        assert B.fps_server_wait(sv, later, 20000) == B.FPS_REQ_DONE
    finally:
        B.fps_server_destroy(sv)


def test_release_rules_and_destroy_with_waiting_requests(B):
    sv = B.fps_server_create(slots=1, hbm_budget=1 << 40, fake_backend=True)
    t1 = B.fps_server_submit(sv, _view(B, 300_000), C, 2, 1, 0.0, 0)
    t2 = B.fps_server_submit(sv, _view(B, 1000), C, 2, 1, 0.0, 0)
    with pytest.raises(B.FpsError) as e:
        B.fps_server_release(sv, t2)  # still queued
    assert e.value.status == B.FPS_ERR_NOT_READY
    with pytest.raises(B.FpsError):
        B.fps_server_result_nnz(sv, t2)
    with pytest.raises(B.FpsError):
        B.fps_server_wait(sv, 12345, 0)  # unknown ticket
    B.fps_server_destroy(sv)  # the running request finishes, the waiting one fails; no hang
    assert t1 != t2


def test_bad_arguments(B):
    with pytest.raises(B.FpsError):
        B.fps_server_create(slots=0, hbm_budget=1, fake_backend=True)
    with pytest.raises(B.FpsError):
        B.fps_server_create(slots=1, hbm_budget=0, fake_backend=True)
    sv = B.fps_server_create(slots=1, hbm_budget=1 << 30, fake_backend=True)
    try:
        with pytest.raises(B.FpsError):
            B.fps_server_submit(sv, _view(B, 10), [1.0, float("inf")], 1, 1, 0.0, 0)
        with pytest.raises(B.FpsError):
            B.fps_server_submit(sv, _view(B, 10), C, 2, 1, -1.0, 0)
    finally:
        B.fps_server_destroy(sv)
