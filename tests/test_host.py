"""Host-side parts of the library, on the CPU: the exported C-ABI, the DC3
suffix array against the oracle's comparison sort, index files, and
argument errors."""
import ctypes
import itertools
import os
import re
import subprocess

import numpy as np
import pytest

import gen
import paper_1303_3692_amd as S
from oracle import oracle
from tests.golden import paper

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def header_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 18
    assert sorted(names) == sorted(S.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in names:
        assert n in exported, n
        assert hasattr(S.lib(), n)


def test_dc3_paper_example():
    p = paper.load()
    assert list(S.sa_build(p["text"]).suffix_array()) == p["sa"]


def test_dc3_exhaustive_small_texts():
    for n in range(1, 8):
        for tup in itertools.product("ACGT", repeat=n):
            t = "".join(tup)
            assert (S.sa_build(t).suffix_array() == oracle.sa_build(t)).all(), t


def test_dc3_repetitive_texts():
    texts = ["A" * 5000, "AC" * 2501, "ACG" * 1700 + "A", "AAAAC" * 900, ("ACGTTGCA" * 400)[:3001],
             "T" * 3 + "A" * 4000 + "T"]
    rng = np.random.default_rng(1)
    for _ in range(20):
        unit = "".join(rng.choice(list("ACGT"), size=rng.integers(1, 9)))
        texts.append((unit * 600)[: int(rng.integers(100, 3000))])
    for t in texts:
        assert (S.sa_build(t).suffix_array() == oracle.sa_build(t)).all()


def test_dc3_every_length_residue():
    """Texts of 16-400 bases over one to four letters, every length residue
    mod 3 (the sample and non-sample groups end differently), periodic and
    random: the recursion on tied triples runs several levels deep."""
    rng = np.random.default_rng(5)
    for n in list(range(16, 80)) + [97, 128, 129, 130, 255, 256, 257, 400]:
        for letters in ("A", "AC", "ACG", "ACGT"):
            t = "".join(rng.choice(list(letters), size=n))
            assert (S.sa_build(t).suffix_array() == oracle.sa_build(t)).all(), (n, letters)
        period = "".join(rng.choice(list("ACGT"), size=int(rng.integers(1, 6))))
        t = (period * n)[:n]
        assert (S.sa_build(t).suffix_array() == oracle.sa_build(t)).all(), (n, period)


@pytest.mark.parametrize("cfg,n", [("c1", 300_000), ("c2", 1_000_000), ("c4", 600_000)])
def test_dc3_generated_references(cfg, n):
    t = gen.make_reference(cfg, n=n).ascii()
    sa = S.sa_build(t).suffix_array()
    assert oracle.sa_check(t, sa) == 0
    assert (sa == oracle.sa_build(t)).all()


def test_lower_case_reference_is_accepted():
    assert (S.sa_build("acgtACGTacgt").suffix_array() == oracle.sa_build("ACGTACGTACGT")).all()


def test_build_errors():
    with pytest.raises(S.SaError) as e:
        S.sa_build("ACGN")
    assert e.value.code == S.SA_EALPHABET
    with pytest.raises(S.SaError) as e:
        S.sa_build("")
    assert e.value.code == S.SA_EINVAL
    out = ctypes.c_void_p()
    assert S.lib().sa_build(None, 5, ctypes.byref(out)) == S.SA_EINVAL
    assert S.lib().sa_build(b"ACGT", 3_000_000_000, ctypes.byref(out)) == S.SA_ETOOBIG
    with pytest.raises(S.SaError) as e:
        S.sa_build_from_sa("ACGT", np.array([0, 1, 2, 9], dtype=np.int32))
    assert e.value.code == S.SA_EINVAL
    assert S.lib().sa_strerror(S.SA_EDEVICE).decode() == "HIP device error"


def test_save_load_roundtrip(tmp_path):
    t = gen.make_reference("c1", n=50_000).ascii()
    ix = S.sa_build(t)
    path = str(tmp_path / "ix.bin")
    S.sa_save(ix, path)
    back = S.sa_load(path)
    assert len(back) == len(ix)
    assert (back.suffix_array() == ix.suffix_array()).all()
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0x40
    open(tmp_path / "bad.bin", "wb").write(bytes(raw))
    with pytest.raises(S.SaError) as e:
        S.sa_load(str(tmp_path / "bad.bin"))
    assert e.value.code == S.SA_EFORMAT
    open(tmp_path / "short.bin", "wb").write(bytes(raw[:50]))
    with pytest.raises(S.SaError) as e:
        S.sa_load(str(tmp_path / "short.bin"))
    assert e.value.code == S.SA_EFORMAT
    with pytest.raises(S.SaError) as e:
        S.sa_load(str(tmp_path / "missing.bin"))
    assert e.value.code == S.SA_EIO


def test_build_from_sa_matches_build():
    t = gen.make_reference("c1", n=20_000).ascii()
    a = S.sa_build(t).suffix_array()
    b = S.sa_build_from_sa(t, oracle.sa_build(t)).suffix_array()
    assert (a == b).all()


def test_null_handles_are_rejected():
    L = S.lib()
    assert L.sa_index_length(None) == -1
    assert L.sa_dindex_length(None) == -1
    assert L.match_batch(None, None, None, 0, None, None, None) == S.SA_EINVAL
    assert L.match_batch_dev(None, None, None, 0, None, None, None) == S.SA_EINVAL
    assert L.sa_upload(None, 0, ctypes.byref(ctypes.c_void_p())) == S.SA_EINVAL
    L.sa_free(None)
    L.sa_dfree(None)
    assert L.sa_server_destroy(None) == S.SA_OK


def test_random_read_rate_rejects_bad_arguments():
    """Checked before any device call: a table size out of range, no output."""
    L = S.lib()
    r = ctypes.c_double(-1.0)
    assert L.sa_random_read_rate(0, 7, ctypes.byref(r)) == S.SA_EINVAL
    assert L.sa_random_read_rate(0, 29, ctypes.byref(r)) == S.SA_EINVAL
    assert L.sa_random_read_rate(0, 20, None) == S.SA_EINVAL
    assert r.value == -1.0
