"""The request server's scheduling logic without a GPU (fake-device mode: no
HIP calls, groups complete after a simulated time): validation codes,
admission by memory budget in FIFO order, grouping, in-flight limits,
per-request failure isolation, timing records, draining on destroy."""
import threading
import time

import pytest

from paper_2109_13406_amd import binding as b

FAKE_PTR = 0x1000          # never dereferenced in fake mode


def _gemm(m, n, k, inject=0, alpha=(1.0, 0.0), beta=(0.5, 0.0), transa="N", transb="N",
          lda=None):
    nra = m if transa == "N" else k
    nrb = k if transb == "N" else n
    P = (FAKE_PTR, FAKE_PTR)
    return b.make_request(b.MPDD_OP_GEMM, transa, transb, m, n, k, alpha, P,
                          max(1, nra) if lda is None else lda, P, max(1, nrb), beta, P,
                          max(1, m), inject=inject)


def _syrk(n, k, uplo="U", trans="N"):
    P = (FAKE_PTR, FAKE_PTR)
    nra = n if trans == "N" else k
    return b.make_request(b.MPDD_OP_SYRK, uplo, trans, 0, n, k, (1.0, 0.0), P, max(1, nra),
                          (None, None), 1, (0.0, 0.0), P, max(1, n))


def _bytes(m, n, k):
    return 16 * (m * k + k * n + m * n)


@pytest.fixture
def server_factory():
    made = []

    def make(budget=1 << 40, inflight=1 << 20, rate=1e12, latency=20e-6):
        s = b.mpdd_server_create(None, budget, inflight, b.MPDD_SERVER_FAKE_DEVICE)
        assert b.mpdd_server_set_fake_rate(s, rate, latency) == 0
        made.append(s)
        return s
    yield make
    for s in made:
        b.mpdd_server_destroy(s)


def test_requests_complete_with_ordered_timings(server_factory):
    s = server_factory()
    tickets = [b.mpdd_server_submit(s, _gemm(64 + i, 32, 100)) for i in range(20)]
    tickets += [b.mpdd_server_submit(s, _syrk(70, 30)) for _ in range(5)]
    for t in tickets:
        info, tm = b.mpdd_server_wait(s, t)
        assert info == 0
        assert tm["arrival"] <= tm["submit"] <= tm["admit"] <= tm["start"] <= tm["end"]
        assert tm["group"] > 0
    st = b.mpdd_server_get_stats(s)
    assert st["completed"] == 25 and st["failed"] == 0 and st["inflight_bytes"] == 0


def test_invalid_request_reports_blas_position(server_factory):
    s = server_factory()
    bad = b.mpdd_server_submit(s, _gemm(10, 10, 10, lda=5))
    bad_flag = b.mpdd_server_submit(s, _gemm(10, 10, 10, transa="X"))
    ok = b.mpdd_server_submit(s, _gemm(10, 10, 10))
    assert b.mpdd_server_wait(s, bad)[0] == 8
    assert b.mpdd_server_wait(s, bad_flag)[0] == 1
    assert b.mpdd_server_wait(s, ok)[0] == 0


def test_quick_return_completes_immediately(server_factory):
    s = server_factory()
    t = b.mpdd_server_submit(s, _gemm(0, 10, 10))
    info, tm = b.mpdd_server_wait(s, t)
    assert info == 0 and tm["group"] == 0
    t = b.mpdd_server_submit(s, _gemm(10, 10, 10, alpha=(0.0, 0.0), beta=(1.0, 0.0)))
    assert b.mpdd_server_wait(s, t)[0] == 0


def test_request_larger_than_budget_fails_alone(server_factory):
    s = server_factory(budget=_bytes(100, 100, 100) + 10)
    big = b.mpdd_server_submit(s, _gemm(200, 200, 200))
    small = b.mpdd_server_submit(s, _gemm(100, 100, 100))
    assert b.mpdd_server_wait(s, big)[0] == b.MPDD_ERR_BUDGET
    assert b.mpdd_server_wait(s, small)[0] == 0


def test_admission_respects_budget_and_fifo(server_factory):
    one = _bytes(64, 64, 64)
    s = server_factory(budget=2 * one + 1, rate=1e8, latency=2e-3)
    tickets = [b.mpdd_server_submit(s, _gemm(64, 64, 64)) for _ in range(10)]
    peak = 0
    while True:
        st = b.mpdd_server_get_stats(s)
        peak = max(peak, st["inflight_bytes"])
        assert st["inflight_bytes"] <= 2 * one + 1
        if st["completed"] == 10:
            break
        time.sleep(1e-4)
    timings = [b.mpdd_server_wait(s, t)[1] for t in tickets]
    admits = [tm["admit"] for tm in timings]
    assert admits == sorted(admits), "admission is not FIFO"
    assert peak > 0


def test_inflight_limit(server_factory):
    s = server_factory(inflight=3, rate=1e8, latency=1e-3)
    tickets = [b.mpdd_server_submit(s, _gemm(32, 32, 32)) for _ in range(12)]
    while b.mpdd_server_get_stats(s)["completed"] < 12:
        assert b.mpdd_server_get_stats(s)["inflight_requests"] <= 3
        time.sleep(1e-4)
    for t in tickets:
        assert b.mpdd_server_wait(s, t)[0] == 0


def test_requests_share_groups_under_load(server_factory):
    # a slow simulated device: requests submitted together run as one group
    s = server_factory(rate=1e7, latency=5e-3)
    tickets = [b.mpdd_server_submit(s, _gemm(40, 40, 40)) for _ in range(40)]
    groups = [b.mpdd_server_wait(s, t)[1]["group"] for t in tickets]
    assert len(set(groups)) < len(groups)
    st = b.mpdd_server_get_stats(s)
    assert st["groups"] < 40


def test_injected_device_error_isolated(server_factory):
    s = server_factory(rate=1e8, latency=1e-3)
    tickets = [b.mpdd_server_submit(s, _gemm(30, 30, 30, inject=(1 if i == 3 else 0)))
               for i in range(8)]
    infos = [b.mpdd_server_wait(s, t)[0] for t in tickets]
    assert infos[3] == b.MPDD_ERR_HIP
    assert all(x == 0 for i, x in enumerate(infos) if i != 3)
    # the server keeps serving afterwards
    t = b.mpdd_server_submit(s, _gemm(30, 30, 30))
    assert b.mpdd_server_wait(s, t)[0] == 0


def test_injected_alloc_failure_isolated(server_factory):
    s = server_factory()
    a = b.mpdd_server_submit(s, _gemm(30, 30, 30, inject=2))
    c = b.mpdd_server_submit(s, _gemm(30, 30, 30))
    assert b.mpdd_server_wait(s, a)[0] == b.MPDD_ERR_ALLOC
    assert b.mpdd_server_wait(s, c)[0] == 0


def test_submit_from_many_threads(server_factory):
    s = server_factory(rate=1e9)
    results = []
    lock = threading.Lock()

    def worker(seed):
        ts = [b.mpdd_server_submit(s, _gemm(20 + seed, 30, 40)) for _ in range(25)]
        out = [b.mpdd_server_wait(s, t)[0] for t in ts]
        with lock:
            results.extend(out)
    th = [threading.Thread(target=worker, args=(i,)) for i in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(results) == 150 and all(x == 0 for x in results)


def test_unknown_ticket_and_poll(server_factory):
    s = server_factory(rate=1e8, latency=5e-3)
    t = b.mpdd_server_submit(s, _gemm(30, 30, 30))
    assert b.mpdd_server_poll(s, t) in (False, True)
    b.mpdd_server_wait(s, t)
    with pytest.raises(ValueError):
        b.mpdd_server_wait(s, t)
    with pytest.raises(ValueError):
        b.mpdd_server_poll(s, 999999)


def test_destroy_drains_pending_work():
    s = b.mpdd_server_create(None, 1 << 40, 1 << 20, b.MPDD_SERVER_FAKE_DEVICE)
    b.mpdd_server_set_fake_rate(s, 1e8, 1e-3)
    for _ in range(10):
        b.mpdd_server_submit(s, _gemm(50, 50, 50))
    assert b.mpdd_server_destroy(s) == 0


def test_real_server_needs_a_handle():
    with pytest.raises(RuntimeError):
        b.mpdd_server_create(None, 1 << 30, 16, 0)


def test_struct_layouts_match_binding():
    import ctypes
    for name in ("mpdd_dd", "mpdd_opts", "mpdd_request", "mpdd_timing", "mpdd_server_stats"):
        assert b.mpdd_struct_size(name) == ctypes.sizeof(getattr(b, name)), name


def test_idle_server_launches_from_submit(server_factory):
    """With nothing queued or admitted and a slot free, submit launches the
    request itself: when it returns, the request is already in flight as a
    group (no hand-off to the scheduler thread)."""
    s = server_factory(rate=1e6, latency=0.2)
    t = b.mpdd_server_submit(s, _gemm(40, 40, 40))
    st = b.mpdd_server_get_stats(s)
    assert st["inflight_requests"] == 1 and st["queued_requests"] == 0 and st["groups"] == 1
    info, tm = b.mpdd_server_wait(s, t)
    assert info == 0 and tm["group"] == 1
    assert tm["submit"] <= tm["admit"] <= tm["start"] <= tm["end"]
    # an injected failure still takes the scheduler's path and stays isolated
    bad = b.mpdd_server_submit(s, _gemm(30, 30, 30, inject=1))
    assert b.mpdd_server_wait(s, bad)[0] == b.MPDD_ERR_HIP
