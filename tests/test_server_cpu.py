"""The request loop on the CPU, with the echo executor (no device work):
admission by a memory budget, continuous batching across requests, per-read
scatter back to the right request, error isolation, cancellation."""
import time

import numpy as np
import pytest

import paper_1303_3692_amd as S


def make_request(rng, nreads, lo=1, hi=60):
    lens = rng.integers(lo, hi + 1, size=nreads)
    offs = np.zeros(nreads + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    data = np.frombuffer(b"ACGT", dtype=np.uint8)[rng.integers(0, 4, size=int(offs[-1]))]
    return data, offs


def echo_expect(offs, ticket, ref, data):
    n = len(offs) - 1
    lo = np.arange(n)
    csum = np.add.reduceat(np.append(data.astype(np.int64), 0), offs[:-1]) if n else np.zeros(0, np.int64)
    csum = np.where(np.diff(offs) > 0, csum, 0) & 0xFFFF
    return np.stack([lo, lo + ticket, np.diff(offs), ref + 256 * csum], axis=1).astype(np.int32)


def wait_all(srv, tickets, timeout_s=20.0):
    end = time.time() + timeout_s
    res = {}
    for t in tickets:
        while True:
            rc, st = srv.poll(t, timeout_us=100_000)
            if rc != S.SA_PENDING:
                res[t] = (rc, st)
                break
            assert time.time() < end, "request did not finish"
    return res


def test_echo_many_requests_are_batched_and_scattered():
    rng = np.random.default_rng(0)
    srv = S.Server([None, None], test_echo=1, max_batch_reads=37, nstreams=3)
    reqs = []
    for i in range(60):
        data, offs = make_request(rng, int(rng.integers(0, 200)))
        ref = i % 2
        t, out = srv.submit(ref, data, offs)
        reqs.append((t, ref, data, offs, out))
    res = wait_all(srv, [r[0] for r in reqs])
    for t, ref, data, offs, out in reqs:
        rc, st = res[t]
        assert rc == S.SA_OK
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
        assert st["nreads"] == len(offs) - 1
        assert (out == echo_expect(offs, t, ref, data)).all()
    srv.destroy()


@pytest.mark.parametrize("pool", [-1, 4096, 0])
def test_host_pool_full_and_absent(pool):
    """Reads reach the executor intact whether submit copies them into the
    pinned pool, into pageable memory (pool full or absent), or both; pool
    space comes back when requests finish."""
    rng = np.random.default_rng(9)
    srv = S.Server([None], test_echo=1, host_pool_bytes=pool, max_batch_reads=50, nstreams=2)
    for _ in range(3):
        reqs = []
        for i in range(40):
            data, offs = make_request(rng, int(rng.integers(0, 80)), 1, 120)
            t, out = srv.submit(0, data, offs)
            reqs.append((t, data, offs, out))
        res = wait_all(srv, [r[0] for r in reqs])
        for t, data, offs, out in reqs:
            assert res[t][0] == S.SA_OK
            assert (out == echo_expect(offs, t, 0, data)).all()
    srv.destroy()


def test_budget_refuses_requests_that_never_fit():
    rng = np.random.default_rng(1)
    # arena budget = fake free - reserve = 4096 bytes
    srv = S.Server([None], test_echo=1, test_fake_free_hbm=(1 << 20) + 4096, hbm_reserve_bytes=1 << 20)
    big_data, big_offs = make_request(rng, 200, 30, 60)      # > 4096 bytes
    small_data, small_offs = make_request(rng, 20, 10, 20)   # < 4096 bytes
    tb, _ = srv.submit(0, big_data, big_offs)
    ts, out = srv.submit(0, small_data, small_offs)
    res = wait_all(srv, [tb, ts])
    assert res[tb][0] == S.SA_ENOSPC
    assert res[ts][0] == S.SA_OK
    assert (out == echo_expect(small_offs, ts, 0, small_data)).all()
    srv.destroy()


def test_budget_admits_in_turn():
    rng = np.random.default_rng(2)
    # room for about two requests at a time; all must still finish, admitted in arrival order
    srv = S.Server([None], test_echo=1, test_fake_free_hbm=(1 << 20) + 3 * 1024, hbm_reserve_bytes=1 << 20,
                   max_batch_reads=16)
    reqs = [srv.submit(0, *make_request(rng, 30, 20, 30)) for _ in range(12)]
    res = wait_all(srv, [t for t, _ in reqs])
    admits = [res[t][1]["t_admit_ns"] for t, _ in reqs]
    assert all(res[t][0] == S.SA_OK for t, _ in reqs)
    assert admits == sorted(admits)
    srv.destroy()


def test_inflight_read_cap():
    rng = np.random.default_rng(3)
    srv = S.Server([None], test_echo=1, max_inflight_reads=50, max_batch_reads=10)
    reqs = [srv.submit(0, *make_request(rng, 40)) for _ in range(5)]
    res = wait_all(srv, [t for t, _ in reqs])
    assert all(rc == S.SA_OK for rc, _ in res.values())
    big = srv.submit(0, *make_request(rng, 51))[0]
    assert wait_all(srv, [big])[big][0] == S.SA_ENOSPC
    srv.destroy()


def test_failed_batch_only_fails_its_requests():
    rng = np.random.default_rng(4)
    srv = S.Server([None], test_echo=1, test_fail_batch=3, max_batch_reads=10, nstreams=1)
    reqs = []
    for _ in range(8):
        data, offs = make_request(rng, 10)
        t, out = srv.submit(0, data, offs)
        reqs.append((t, data, offs, out))
    res = wait_all(srv, [r[0] for r in reqs])
    codes = [res[t][0] for t, _, _, _ in reqs]
    assert codes.count(S.SA_EDEVICE) >= 1
    for (t, data, offs, out), rc in zip(reqs, codes):
        if rc == S.SA_OK:
            assert (out == echo_expect(offs, t, 0, data)).all()
        else:
            assert rc == S.SA_EDEVICE
    srv.destroy()


def test_submit_validation_and_unknown_ticket():
    srv = S.Server([None], test_echo=1)
    data = np.frombuffer(b"A" * 1100, dtype=np.uint8)
    with pytest.raises(S.SaError) as e:
        srv.submit(0, data, np.array([0, S.SA_MAX_READ + 1]))
    assert e.value.code == S.SA_ETOOBIG
    with pytest.raises(S.SaError) as e:
        srv.submit(5, data, np.array([0, 4]))
    assert e.value.code == S.SA_EINVAL
    with pytest.raises(S.SaError) as e:
        srv.submit(0, data, np.array([4, 2]))
    assert e.value.code == S.SA_EINVAL
    with pytest.raises(S.SaError) as e:
        srv.poll(12345)
    assert e.value.code == S.SA_ENOTFOUND
    t, _ = srv.submit(0, data, np.array([0]))  # zero reads
    assert wait_all(srv, [t])[t][0] == S.SA_OK
    srv.destroy()


def test_batch_linger_waits_for_a_full_batch_or_its_deadline():
    """With batch_linger_us, a batch starts once it holds max_batch_reads
    reads or its oldest read has waited that long; results are unchanged."""
    rng = np.random.default_rng(11)
    linger_ns = 300_000_000
    srv = S.Server([None, None], test_echo=1, max_batch_reads=1000, batch_linger_us=linger_ns // 1000)
    # a lone small request waits out the deadline
    data, offs = make_request(rng, 10)
    t, out = srv.submit(0, data, offs)
    rc, st = wait_all(srv, [t])[t]
    assert rc == S.SA_OK and (out == echo_expect(offs, t, 0, data)).all()
    assert st["t_done_ns"] - st["t_admit_ns"] >= linger_ns
    # a request that fills a batch by itself starts at once
    data, offs = make_request(rng, 1000)
    t, out = srv.submit(1, data, offs)
    rc, st = wait_all(srv, [t])[t]
    assert rc == S.SA_OK and (out == echo_expect(offs, t, 1, data)).all()
    assert st["t_done_ns"] - st["t_admit_ns"] < linger_ns // 2
    # small requests that fill a batch together start as soon as the last arrives
    reqs = []
    for i in range(4):
        data, offs = make_request(rng, 250)
        reqs.append((srv.submit(0, data, offs), data, offs))
    res = wait_all(srv, [r[0][0] for r in reqs])
    for (t, out), data, offs in reqs:
        rc, st = res[t]
        assert rc == S.SA_OK and (out == echo_expect(offs, t, 0, data)).all()
    last_admit = max(res[r[0][0]][1]["t_admit_ns"] for r in reqs)
    assert max(res[r[0][0]][1]["t_done_ns"] for r in reqs) - last_admit < linger_ns // 2
    srv.destroy()
    for bad in (-1, 1_000_001):
        with pytest.raises(S.SaError) as e:
            S.Server([None], test_echo=1, batch_linger_us=bad)
        assert e.value.code == S.SA_EINVAL


def test_destroy_with_pending_requests():
    rng = np.random.default_rng(5)
    srv = S.Server([None, None], test_echo=1, max_inflight_reads=20, max_batch_reads=5)
    outs = [srv.submit(i % 2, *make_request(rng, 20))[1] for i in range(50)]
    srv.destroy()  # must not hang or crash; unfinished outputs stay untouched
    assert all(o.shape[1] == 4 for o in outs)


def test_replay_submits_open_loop_from_native_threads():
    """sa_server_replay (the load-test client): every request submitted at
    or after its scheduled time, in time order per client thread, each
    getting its own ticket and its results, the timestamps ordered."""
    rng = np.random.default_rng(5)
    srv = S.Server([None, None, None], test_echo=1, max_batch_reads=300, nstreams=2)
    n = 120
    reqs = [make_request(rng, int(rng.integers(0, 80))) for _ in range(n)]
    refs = [i % 3 for i in range(n)]
    arrival = np.sort(rng.integers(0, 30_000_000, size=n))  # within 30 ms
    outs, sched, stats = srv.replay(refs, [r[0] for r in reqs], [r[1] for r in reqs], arrival, nthreads=4)
    tickets = set()
    for i, ((data, offs), out, st) in enumerate(zip(reqs, outs, stats)):
        assert st["status"] == S.SA_OK
        assert sched[i] <= st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
        assert st["nreads"] == len(offs) - 1
        if len(offs) > 1:
            ticket = int(out[0, 1] - out[0, 0])
            tickets.add(ticket)
            assert (out == echo_expect(offs, ticket, refs[i], data)).all()
    assert len(tickets) == sum(1 for d, o in reqs if len(o) > 1) and min(tickets) >= 1 and max(tickets) <= n
    assert (np.diff(sched) == np.diff(arrival)).all()
    srv.destroy()


def test_replay_rejects_bad_arguments():
    srv = S.Server([None], test_echo=1)
    L = S.lib()
    assert L.sa_server_replay(None, 0, None, None, None, None, None, None, 1, None, None) == S.SA_EINVAL
    assert L.sa_server_replay(srv._p, 0, None, None, None, None, None, None, 0, None, None) == S.SA_EINVAL
    assert L.sa_server_replay(srv._p, 1, None, None, None, None, None, None, 1, None, None) == S.SA_EINVAL
    srv.destroy()
