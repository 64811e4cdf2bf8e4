"""The request loop on the GPU: requests over two resident references,
submitted together and in an open-loop stream, each result identical to
the same reads matched alone (tolerance 0) and to the oracle."""
import time

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def refs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    out = []
    for cfg, n in (("c2", 1_500_000), ("c4", 2_500_000)):
        ref = gen.make_reference(cfg, n=n)
        text = ref.ascii()
        out.append((ref, text, oracle.sa_build(text), S.sa_upload(S.sa_build(text), 0)))
    return out


def wait_all(srv, tickets, timeout_s=120.0):
    end = time.time() + timeout_s
    res = {}
    for t in tickets:
        while True:
            rc, st = srv.poll(t, timeout_us=200_000)
            if rc != S.SA_PENDING:
                res[t] = (rc, st)
                break
            assert time.time() < end, "request did not finish"
    return res


def test_requests_alone_and_in_the_mix(refs):
    print("case: serving mix", flush=True)
    rng = np.random.default_rng(12)
    sizes = gen.request_sizes(60, rng, max_reads=20_000)
    reqs = []
    for i, size in enumerate(sizes):
        which = int(rng.integers(0, 2))
        ref = refs[which][0]
        spec = gen.ReadSpec(900 + i, int(size), 30, 300, 0.3, 0.0, 0.02)
        reqs.append((which, gen.make_reads(ref, spec)))
    # small batches and three streams: many requests share batches and run concurrently
    srv = S.Server([r[3] for r in refs], max_batch_reads=4096, nstreams=3)
    tickets = [srv.submit(which, r.data, r.offs) for which, r in reqs]
    res = wait_all(srv, [t for t, _ in tickets])
    for (t, out), (which, r) in zip(tickets, reqs):
        rc, st = res[t]
        assert rc == S.SA_OK, rc
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
        _, text, sa, d = refs[which]
        alone = S.match_batch(d, r.data, r.offs)
        assert (out == alone).all()
        want = oracle.match(text, sa, r.data, r.offs)
        assert (out[:, :3] == want[:, :3]).all() and ((out[:, 3] & 1) == want[:, 3]).all()
    srv.destroy()


@pytest.mark.parametrize("pool", [-1, 0])
def test_open_loop_stream_and_budget(refs, pool):
    """Every request is admitted into the device arena under a 4 MB budget
    (requests wait for admission; one that can never fit is refused), with
    no pinned pool (pool -1: pageable copies) and with the default mapped
    pool (pool 0: copied to the arena by the upload kernel)."""
    print("case: serving stream, pool", pool, flush=True)
    rng = np.random.default_rng(13)
    reqs = []
    for i in range(40):
        which = int(rng.integers(0, 2))
        spec = gen.ReadSpec(1900 + i, int(rng.integers(1, 3000)), 30, 300, 0.2, 0.01, 0.01)
        reqs.append((which, gen.make_reads(refs[which][0], spec)))
    # a device budget of about 3.7 MB for read data (4 MB less the per-stream
    # buffers)
    free_now = torch.cuda.mem_get_info()[0]
    srv = S.Server([r[3] for r in refs], test_fake_free_hbm=free_now, hbm_reserve_bytes=free_now - (4 << 20),
                   max_batch_reads=1024, nstreams=2, host_pool_bytes=pool)
    big = gen.make_reads(refs[0][0], gen.ReadSpec(2999, 30_000, 200, 200, 0.0, 0.0, 0.0))
    tickets = []
    for which, r in reqs:
        tickets.append(srv.submit(which, r.data, r.offs))
        time.sleep(0.001)
    t_big, out_big = srv.submit(0, big.data, big.offs)
    res = wait_all(srv, [t for t, _ in tickets] + [t_big])
    assert res[t_big][0] == S.SA_ENOSPC
    for (t, out), (which, r) in zip(tickets, reqs):
        assert res[t][0] == S.SA_OK
        alone = S.match_batch(refs[which][3], r.data, r.offs)
        assert (out == alone).all()
    srv.destroy()


@pytest.mark.parametrize("linger", [0, 2000])
def test_replayed_stream(refs, linger):
    """The native load-test client on the device: an open-loop stream over
    both references, every result identical to the same reads matched alone
    (batches starting at once, or waiting up to 2 ms to fill)."""
    print("case: serving replay, linger", linger, flush=True)
    rng = np.random.default_rng(14)
    stream = []
    for i in range(80):
        which = int(rng.integers(0, 2))
        spec = gen.ReadSpec(2900 + i, int(rng.integers(0, 5000)), 30, 300, 0.3, 0.0, 0.02)
        stream.append((which, gen.make_reads(refs[which][0], spec)))
    arrival = np.cumsum(rng.exponential(200_000, size=len(stream))).astype(np.int64)  # ~5,000 requests/s
    srv = S.Server([r[3] for r in refs], max_batch_reads=1 << 16, nstreams=2, batch_linger_us=linger)
    outs, sched, stats = srv.replay([w for w, _ in stream], [r.data for _, r in stream], [r.offs for _, r in stream],
                                    arrival, nthreads=4)
    srv.destroy()
    for (which, r), out, t, st in zip(stream, outs, sched, stats):
        assert st["status"] == S.SA_OK
        assert t <= st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
        if r.count:
            assert (out == S.match_batch(refs[which][3], r.data, r.offs)).all()


@pytest.mark.parametrize("measure", [1, 2])
def test_measured_serving(refs, measure):
    """Measurement mode: the same results as the reads matched alone, every
    request image counted as uploaded to the arena, search time and (with
    the instrumented kernels) bytes touched reported."""
    print("case: measured serving", measure, flush=True)
    rng = np.random.default_rng(15 + measure)
    reqs = []
    for i in range(24):
        which = int(rng.integers(0, 2))
        spec = gen.ReadSpec(3100 + i, int(rng.integers(1, 4000)), 30, 300, 0.2, 0.0, 0.02)
        reqs.append((which, gen.make_reads(refs[which][0], spec)))
    srv = S.Server([r[3] for r in refs], max_batch_reads=2048, nstreams=2, measure=measure)
    tickets = [srv.submit(which, r.data, r.offs) for which, r in reqs]
    res = wait_all(srv, [t for t, _ in tickets])
    st = srv.stats()
    srv.destroy()
    for (t, out), (which, r) in zip(tickets, reqs):
        assert res[t][0] == S.SA_OK
        assert (out == S.match_batch(refs[which][3], r.data, r.offs)).all()
    nreads = sum(r.count for _, r in reqs)
    images = sum(((len(r.data) + 7) // 8) * 8 + 8 * (r.count + 1) for _, r in reqs)
    assert st["reads"] == nreads and st["batches"] >= 1
    assert st["upload_bytes"] == images
    assert st["search_ms"] > 0
    if measure == 2:
        assert st["touched_bytes"] > 16 * nreads
    else:
        assert st["touched_bytes"] == 0
