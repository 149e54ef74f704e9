"""Pins of the oracle's sketch generator (Philox4x32-10 + Box-Muller).

The paper only says the sketch is GIID (Sec. 2.1, Fig. 1 step 1); the
generator is fixed by its published definition.  Pins: published known-answer
vectors, an independent implementation (PyTorch's header-only engine, compiled
here), exact edge values of the uniform map, and the distribution facts the
paper relies on (N(0,1) entries; Lemma in Sec. 3.1: E = l, Var = 2l).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*r[:6])
        assert [int(x) for x in out] == r[6:]


@pytest.fixture(scope="module")
def torch_ref(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.fail("g++ is required for the Philox cross-check")
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("ref") / "philox_ref")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I", inc, "-o", exe,
                           os.path.join(HERE, "ref", "philox_torch_ref.cpp")])
    return exe


@pytest.mark.parametrize("seed,sid,batch,offset,count", [
    (0x5EED0000, 0, 0, 0, 512),
    (0x123456789ABCDEF0, 3, 0, 1000, 64),
    (1, 6, 7, 0xFFFFFFF0, 40),            # counter crosses 2^32
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, (1 << 64) - 8, 8),
])
def test_matches_independent_engine(torch_ref, seed, sid, batch, offset, count):
    # torch's engine: key = seed words, counter = (offset lo, offset hi,
    # subsequence lo, subsequence hi); our stream id is c2 and batch is c3.
    subseq = sid | (batch << 32)
    out = subprocess.check_output([torch_ref, str(seed), str(subseq),
                                   str(offset), str(count)], text=True)
    ref = np.array([[int(x) for x in ln.split()] for ln in out.splitlines()],
                   dtype=np.uint64)
    got = philox.raw_words(seed, sid, offset, count, batch).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_uniform_map_edges():
    w = np.array([[0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],
                  [0, 0, 0, 0],
                  [1 << 5, 0, 0, 1 << 6]], dtype=np.uint32)
    u1, u2 = philox.uniforms(w)
    assert u1[0] == 1.0                      # largest u1 is exactly 1
    assert u2[0] == 1.0 - 2.0 ** -53         # largest u2 stays below 1
    assert u1[1] == 2.0 ** -53 and u2[1] == 0.0
    assert u1[2] == (2.0 ** 26 + 1) * 2.0 ** -53
    assert u2[2] == 2.0 ** -53


def test_box_muller_pairs_and_layout():
    seed, n, l = 77, 37, 5
    om = philox.sketch(seed, n, l)
    assert om.shape == (n, l)
    z = philox.normals(seed, 0, 0, n * l)
    # Omega[i, j] is normal number j*n + i
    for j in range(l):
        assert np.array_equal(om[:, j], z[j * n:(j + 1) * n])
    # numbers 2t and 2t+1 are the cos / sin of one Box-Muller pair
    u1, u2 = philox.uniforms(philox.raw_words(seed, 0, 0, 4))
    r = np.sqrt(-2.0 * np.log(u1))
    th = philox.TWO_PI * u2
    assert np.array_equal(z[0:8:2], r * np.cos(th))
    assert np.array_equal(z[1:8:2], r * np.sin(th))
    # an odd start is the second half of a pair
    assert np.array_equal(philox.normals(seed, 0, 3, 4), z[3:7])
    # the sketch for a smaller l is a column prefix
    assert np.array_equal(philox.sketch(seed, n, 3), om[:, :3])


def test_gaussian_moments_and_ks():
    z = philox.normals(0x5EED0001, 0, 0, 1 << 20)
    N = len(z)
    assert abs(z.mean()) < 5.0 / np.sqrt(N)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / N)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the two halves of each pair are uncorrelated
    c = np.corrcoef(z[0::2], z[1::2])[0, 1]
    assert abs(c) < 5.0 / np.sqrt(N / 2)


def test_column_norm_lemma():
    """Lemma of Sec. 3.1: for an l x m GIID Omega and a fixed a,
    ||Omega a||^2 / ||a||^2 has mean l and variance 2l (chi-square_l)."""
    m, l, draws = 40, 12, 3000
    a = np.linspace(-1.0, 2.0, m)
    ratios = np.empty(draws)
    for d in range(draws):
        om = philox.sketch(0xABC000 + d, m, l).T        # l x m
        ratios[d] = np.sum((om @ a) ** 2) / np.sum(a * a)
    assert abs(ratios.mean() - l) < 4.0 * np.sqrt(2 * l / draws)
    # sample variance of a chi-square_l: its sd is ~ sqrt((8l + 24... ) / N);
    # use a 15% band, far outside the 2.5% sampling spread at N=3000
    assert abs(ratios.var() - 2 * l) < 0.15 * 2 * l
    assert scipy.stats.kstest(ratios, "chi2", args=(l,)).pvalue > 1e-4


def test_streams_and_seeds_differ():
    a = philox.normals(5, 0, 0, 1000)
    b = philox.normals(5, 1, 0, 1000)
    c = philox.normals(6, 0, 0, 1000)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.15
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.15
