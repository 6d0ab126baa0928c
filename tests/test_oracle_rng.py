"""Pins of the oracle's random streams (Philox4x32-10, Box-Muller, accept uniform).

The Philox block function is pinned to rocRAND's Philox4x32-10 engine (a
library implementation written independently of the oracle; its header is
host-callable, so it runs here on the CPU).  The distribution transforms are
pinned by goodness-of-fit and independence tests: a wrong scale, a swapped
word or a biased mapping moves one of the statistics far outside its bound.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or g++ unavailable")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_ref")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])

    def run(keys, ctrs):
        rec = np.concatenate([keys, ctrs], axis=1).astype(np.uint32)
        out = subprocess.run([exe], input=rec.tobytes(), capture_output=True, check=True).stdout
        return np.frombuffer(out, dtype=np.uint32).reshape(-1, 4)
    return run


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(123)
    n = 4000
    keys = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctrs = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctrs[:, 1] &= (1 << 30) - 1
    # structured counters as the sampler uses them: (chain, t, block, tag)
    keys[:64] = 0
    ctrs[:64] = np.stack([np.arange(64), np.arange(64) % 7, np.arange(64) // 8, np.arange(64) % 2], 1)
    ref = rocrand_ref(keys, ctrs)
    got = np.stack([oracle.philox(ctrs[i:i + 1], keys[i])[0] for i in range(n)])
    assert np.array_equal(got, ref)


def test_box_muller_radius_and_key_split():
    # Box-Muller invariants: z0^2 + z1^2 = -2 log u1 and atan2(z1, z0) = 2 pi u2 (mod 2 pi),
    # with (u1, u2) from words 0 and 1 of the block keyed by the seed split
    # (low word, high word).
    seed = 0x0123456789ABCDEF
    for c0 in range(50):
        z = oracle.normal4(seed, c0, 6, 7, 0)
        w = oracle.philox(np.array([[c0, 6, 7, 0]], np.uint32), (0x89ABCDEF, 0x01234567))[0]
        for pair in range(2):
            u1 = ((int(w[2 * pair]) >> 9) + 0.5) / 2**23
            u2 = ((int(w[2 * pair + 1]) >> 9) + 0.5) / 2**23
            r2 = z[2 * pair] ** 2 + z[2 * pair + 1] ** 2
            assert r2 == pytest.approx(-2 * np.log(u1), rel=1e-13)
            ang = np.arctan2(z[2 * pair + 1], z[2 * pair]) % (2 * np.pi)
            assert ang == pytest.approx(2 * np.pi * u2, abs=1e-9)


def test_momentum_is_standard_normal():
    p = oracle.momentum(seed=0, C=20000, t=3, D=10).ravel()   # 200k draws
    ks = stats.kstest(p, "norm")
    assert ks.pvalue > 1e-4, ks
    assert abs(p.mean()) < 5 * 1 / np.sqrt(p.size)
    assert abs(p.var() - 1) < 5 * np.sqrt(2 / p.size)
    # fourth moment (a wrong radius law shows up here)
    assert abs(np.mean(p ** 4) - 3) < 5 * np.sqrt(96 / p.size)


def test_momentum_components_independent():
    p = oracle.momentum(seed=1, C=50000, t=0, D=8)
    c = np.corrcoef(p.T)
    off = c[~np.eye(8, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(50000)
    # the two normals of one Box-Muller pair are uncorrelated in square too
    s = np.corrcoef(p[:, 0] ** 2, p[:, 1] ** 2)[0, 1]
    assert abs(s) < 5 / np.sqrt(50000) * 2


def test_momentum_streams_depend_on_chain_step_and_seed():
    a = oracle.momentum(0, 64, 0, 5)
    b = oracle.momentum(0, 64, 1, 5)
    c = oracle.momentum(7, 64, 0, 5)
    assert len(np.unique(a[:, 0])) == 64
    assert not np.any(a == b)
    assert not np.any(a == c)
    # a chain's momentum does not depend on how many chains run (batch semantics)
    assert np.array_equal(oracle.momentum(0, 3, 0, 5), a[:3])


def test_accept_uniform_distribution():
    u = np.concatenate([oracle.accept_uniform(0, 100000, t) for t in range(3)])
    assert np.all(u > 0) and np.all(u < 1)
    ks = stats.kstest(u, "uniform")
    assert ks.pvalue > 1e-4, ks
    # -log u is Exp(1): the accept test compares log u with -dH
    e = -np.log(u)
    assert abs(e.mean() - 1) < 5 / np.sqrt(u.size)
    # momentum and accept streams of the same (chain, t) differ (distinct tags)
    z = oracle.momentum(0, 1000, 0, 4)
    uu = oracle.accept_uniform(0, 1000, 0)
    assert abs(np.corrcoef(z[:, 0], uu)[0, 1]) < 0.15


def test_philox_known_answer_vectors():
    # the published known-answer vectors of Philox4x32-10 (tests/golden/philox4x32_10_kat.txt)
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        key, ctr, want = (v[0], v[1]), np.array([v[2:6]], np.uint32), v[6:10]
        assert list(oracle.philox(ctr, key)[0]) == want
