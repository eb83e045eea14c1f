"""The serving scheduler through the C ABI in its device-free test mode: each
launch is modelled as taking sum(2MNK)/rate seconds and nothing is written,
so admission, ordering, continuous batching, overlap, failure reporting and
the latency statistics can be checked on a CPU host."""
import math
import time

import pytest

from paper_2408_15384_amd import api

BASE = 1 << 40  # fake, non-overlapping device addresses (never dereferenced in dry-run)


def prob(i, M, N, K, elem=8):
    a = BASE + i * (1 << 32)
    return api.Problem(M, N, K, a, K, a + (1 << 30), N, a + (2 << 30), N)


def nbytes(M, N, K, elem=8):
    return elem * (M * K + K * N + M * N)


@pytest.fixture(scope="module", autouse=True)
def lib():
    return api.load_library()


def submit(srv, i, M=256, N=256, K=256, method=api.MM_F64, arrival=-1.0):
    return srv.submit_raw(prob(i, M, N, K), method, arrival)


def test_fifo_completion_under_tight_budget():
    n = 256
    # budget fits one request at a time: strictly sequential, in arrival order
    srv = api.Server(budget_bytes=nbytes(n, n, n) + 10, slots=4, max_batch=8, dry_run_tflops=0.01)
    try:
        ids = [submit(srv, i) for i in range(6)]
        lats = [srv.wait(r)[1] for r in ids]
        st = srv.stats()
        assert st["completed"] == 6 and st["failed"] == 0
        assert st["launches"] == 6 and st["mean_batch"] == 1.0
        assert st["peak_bytes"] == nbytes(n, n, n)
        assert all(b > a for a, b in zip(lats, lats[1:]))      # each waits for the previous
        service_ms = 2 * n ** 3 / 0.01e12 * 1e3                 # 3.36 ms
        assert lats[-1] >= 6 * service_ms * 0.9
    finally:
        srv.close()


def test_oversize_request_and_full_queue():
    srv = api.Server(budget_bytes=nbytes(64, 64, 64) * 2, slots=1, max_batch=1, queue_capacity=2,
                     dry_run_tflops=1e-4)
    try:
        with pytest.raises(api.MMError) as e:
            submit(srv, 0, 512, 512, 512)
        assert e.value.status == api.MM_E_NOMEM
        results = []
        for i in range(5):
            try:
                results.append(submit(srv, i + 1, 64, 64, 64))
            except api.MMError as err:
                assert err.status == api.MM_E_BUSY
                results.append(None)
        # at most one request in the only slot plus queue_capacity waiting; the
        # scheduler may or may not have taken the first one yet
        accepted = [r for r in results if r is not None]
        assert 2 <= len(accepted) <= 3
        for r in results:
            if r is not None:
                assert srv.wait(r)[0] == api.MM_OK
    finally:
        srv.close()


def test_continuous_batching_admits_arrivals_while_busy():
    srv = api.Server(budget_bytes=1 << 40, slots=1, max_batch=16, dry_run_tflops=0.01)
    try:
        first = submit(srv, 0, 512, 512, 512)      # ~27 ms on the model
        time.sleep(0.005)
        later = [submit(srv, i + 1, 64, 64, 64) for i in range(5)]
        for r in [first] + later:
            assert srv.wait(r)[0] == api.MM_OK
        st = srv.stats()
        assert st["launches"] == 2                  # the 5 arrivals went out together
        assert st["mean_batch"] == 3.0
    finally:
        srv.close()


def test_slots_overlap():
    n = 512
    service = 2 * n ** 3 / 0.01e12
    srv = api.Server(budget_bytes=1 << 40, slots=4, max_batch=1, dry_run_tflops=0.01)
    try:
        t0 = srv.clock()
        ids = [submit(srv, i, n, n, n) for i in range(4)]
        for r in ids:
            srv.wait(r)
        elapsed = srv.clock() - t0
        assert elapsed < 2.5 * service              # four launches ran side by side
        assert srv.stats()["launches"] == 4
    finally:
        srv.close()


def test_budget_limits_bytes_in_flight():
    n = 256
    srv = api.Server(budget_bytes=2 * nbytes(n, n, n), slots=4, max_batch=1, dry_run_tflops=0.01)
    try:
        ids = [submit(srv, i) for i in range(6)]
        for r in ids:
            srv.wait(r)
        assert srv.stats()["peak_bytes"] == 2 * nbytes(n, n, n)
    finally:
        srv.close()


def test_failed_request_reported_alone():
    srv = api.Server(budget_bytes=1 << 40, slots=2, max_batch=4, dry_run_tflops=1.0, dry_run_fail_id=3)
    try:
        ids = [submit(srv, i, 64, 64, 64) for i in range(5)]
        statuses = [srv.wait(r)[0] for r in ids]
        assert statuses == [api.MM_OK, api.MM_OK, api.MM_E_DEVICE, api.MM_OK, api.MM_OK]
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 5
        assert st["useful_flop"] == 4 * 2 * 64 ** 3
    finally:
        srv.close()


def test_latency_from_scheduled_arrival_and_percentiles():
    srv = api.Server(budget_bytes=1 << 40, slots=2, max_batch=4, dry_run_tflops=0.05)
    try:
        time.sleep(0.03)                            # server clock starts at 0; arrivals must be >= 0
        now = srv.clock()
        ids = [submit(srv, i, 128, 128, 128 * (1 + i % 5), arrival=now - 0.010) for i in range(40)]
        lats = sorted(srv.wait(r)[1] for r in ids)
        assert lats[0] >= 10.0                      # measured from the scheduled arrival
        st = srv.stats()
        nr = lambda q: lats[max(1, math.ceil(q * len(lats))) - 1]
        assert st["p50_ms"] == pytest.approx(nr(0.5))
        assert st["p99_ms"] == pytest.approx(nr(0.99))
        assert st["max_ms"] == pytest.approx(lats[-1])
        assert st["tflops"] > 0
    finally:
        srv.close()


def test_wait_timeout_and_unknown_id():
    srv = api.Server(budget_bytes=1 << 40, slots=1, max_batch=1, dry_run_tflops=1e-4)
    try:
        r = submit(srv, 0, 256, 256, 256)           # ~0.3 s on the model
        with pytest.raises(api.MMError) as e:
            srv.wait(r, timeout_us=1000)
        assert e.value.status == api.MM_E_TIMEOUT
        assert srv.wait(r)[0] == api.MM_OK
        with pytest.raises(api.MMError):
            srv.wait(r)                             # already collected
    finally:
        srv.close()


def test_two_waiters_on_one_request():
    # both threads block in the library (ctypes releases the GIL): the first
    # to wake collects the request, the other reports it unknown and returns
    import threading
    srv = api.Server(budget_bytes=1 << 40, slots=1, max_batch=1, dry_run_tflops=1e-4)
    try:
        r = submit(srv, 0, 256, 256, 256)           # ~0.3 s on the model
        out = []

        def waiter():
            try:
                out.append(srv.wait(r, timeout_us=20_000_000)[0])
            except api.MMError as e:
                out.append(e.status)

        ts = [threading.Thread(target=waiter) for _ in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join(30)
        assert not any(t.is_alive() for t in ts)
        assert sorted(out) == sorted([api.MM_OK, api.MM_E_INVAL])
        assert srv.stats()["completed"] == 1
    finally:
        srv.close()


def test_invalid_requests_rejected():
    srv = api.Server(budget_bytes=1 << 40, slots=1, max_batch=1, dry_run_tflops=1.0)
    try:
        bad = api.Problem(4, 4, 4, BASE, 2, BASE + (1 << 30), 4, BASE + (2 << 30), 4)   # lda < K
        with pytest.raises(api.MMError) as e:
            srv.submit_raw(bad, api.MM_F64)
        assert e.value.status == api.MM_E_INVAL
        with pytest.raises(api.MMError):
            srv.submit_raw(prob(1, 4, 4, 4), 7)
    finally:
        srv.close()
    with pytest.raises(api.MMError):
        api.Server(budget_bytes=1 << 30, slots=0)
    with pytest.raises(api.MMError):
        api.Server(budget_bytes=1 << 30, slots=17)


def test_split_request_with_k_beyond_limit_is_refused():
    # split requests address 16 plane rows with 32-bit offsets: K above
    # 2^26 - 32 is refused at submission; binary64 has no such limit
    K = (1 << 26) - 31
    srv = api.Server(budget_bytes=1 << 62, slots=1, dry_run_tflops=1e6)
    try:
        with pytest.raises(api.MMError) as e:
            submit(srv, 0, 2, 2, K, method=api.MM_SPLIT_BF16_6)
        assert e.value.status == api.MM_E_UNSUPPORTED
        rid = submit(srv, 1, 2, 2, K, method=api.MM_F64)
        assert srv.wait(rid)[0] == api.MM_OK
    finally:
        srv.close()
