"""The seeded input generators: chunked and parallel generation give the
same reads as one serial pass; offsets without reads; the read classes and
their recorded substitutions are what the reads hold."""
import numpy as np
import pytest

import gen

FIELDS = ("data", "offs", "cls", "pos", "first_sub")


@pytest.fixture(scope="module")
def ref():
    return gen.make_reference("c4", n=400_000)


@pytest.mark.parametrize("spec_name", ["c1", "c2", "c3", "c4"])
def test_parallel_and_chunked_equal_serial(ref, spec_name):
    spec = gen.READ_SPECS[spec_name]
    count = 3 * gen.CHUNK + 1234
    a = gen.make_reads(ref, spec, count)
    b = gen.make_reads_parallel(ref, spec, count, workers=3)
    for f in FIELDS:
        assert (getattr(a, f) == getattr(b, f)).all(), f
    assert (gen.read_offsets(spec, count) == a.offs).all()
    lo, hi = gen.CHUNK - 7, 2 * gen.CHUNK + 11
    c = gen.make_reads(ref, spec, count, lo, hi)
    assert c.data.tobytes() == a.data[a.offs[lo]:a.offs[hi]].tobytes()
    assert (c.pos == a.pos[lo:hi]).all() and (c.first_sub == a.first_sub[lo:hi]).all()


@pytest.mark.parametrize("spec_name", ["c2", "c4"])
def test_recorded_substitutions(ref, spec_name):
    """Sampled reads equal the reference up to first_sub; random reads have
    pos -1; the random fraction is the recipe's."""
    spec = gen.READ_SPECS[spec_name]
    r = gen.make_reads(ref, spec, 20_000)
    assert abs((r.cls == gen.RANDOM).mean() - spec.frac_random) < 1e-3
    assert ((r.pos == -1) == (r.cls == gen.RANDOM)).all()
    text = gen.to_ascii(ref.codes)
    for i in np.nonzero(r.cls != gen.RANDOM)[0][:3000]:
        m = r.offs[i + 1] - r.offs[i]
        read = r.data[r.offs[i]:r.offs[i + 1]]
        src = text[r.pos[i]:r.pos[i] + m]
        diff = np.nonzero(read != src)[0]
        assert (diff[0] if len(diff) else m) == r.first_sub[i]


def test_request_pool_is_deterministic(ref):
    refs = [ref, ref]
    a = gen.request_pool(refs, 12, max_reads=500)
    b = gen.request_pool(refs, 12, max_reads=500)
    for (ra, xa), (rb, xb) in zip(a, b):
        assert ra == rb and xa.data.tobytes() == xb.data.tobytes()
    s = gen.request_stream(refs, 50, 1000.0, pool=a)
    t = [x.t_arrival for x in s]
    assert t == sorted(t) and t[0] == 0.0
    assert all(any(x.reads is p for _, p in a) for x in s)
