"""Gaussian test matrix of the range finder, from a counter-based generator.

Test infrastructure (see the package header): only tests, smoke() and the
bench's cpu_baseline leg may use it.

The paper draws the n x (k+p) sketch with Matlab's ``randn`` (Fig. 1 step 1;
Sec. 2.1 "GIID matrix"; Alg. 4/5 line 1) and names no generator.  Both the
oracle and the GPU library use the same published counter-based generator so
that they see the same sketch:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key, ten rounds of
  two 32x32->64 multiplies with xor mixing, the key bumped by two Weyl
  constants between rounds.
* Box-Muller (1958): two uniforms give two independent N(0,1) values
  r*cos(theta), r*sin(theta) with r = sqrt(-2 ln u1), theta = 2 pi u2.

Stream layout (all values FP64):

* key = (seed & 0xffffffff, seed >> 32);
* normal number t of stream ``sid`` uses counter (c0, c1) = t // 2 as a 64-bit
  integer (low word first), c2 = sid, c3 = batch;
* from the four output words x0..x3:
  u1 = ((x0 >> 5) * 2^26 + (x1 >> 6) + 1) * 2^-53   in (0, 1],
  u2 = ((x2 >> 5) * 2^26 + (x3 >> 6)) * 2^-53       in [0, 1);
* theta = fl(TWO_PI * u2) with TWO_PI the double nearest 2 pi;
  t even -> r cos(theta), t odd -> r sin(theta);
* sketch entry Omega[i, j] (i < n rows, j < l columns) is number t = j*n + i
  of stream 0, so the sketch for a smaller l is a column prefix.
"""

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
TWO_PI = 6.283185307179586  # nearest double to 2*pi

STREAM_SKETCH = 0      # Omega (n x l) of the range finder
STREAM_QB = 5          # Omega_i (n x b) of block i of the blocked QB (batch = i)
STREAM_LEFT = 6        # Omega~^T (m x l) of the left-sketch ID


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on uint32 arrays (c0..c3) with key (k0, k1).

    One round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit
    products), new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key
    is bumped by (W0, W1) modulo 2^32 before every round but the first.
    Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = c0 * np.uint64(PHILOX_M0)
        p1 = c2 * np.uint64(PHILOX_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def raw_words(seed, sid, first_pair, count, batch=0):
    """Philox outputs for counters first_pair .. first_pair+count-1 of stream
    ``sid``: a (count, 4) uint32 array."""
    idx = np.arange(count, dtype=np.uint64) + np.uint64(first_pair)
    lo = idx & np.uint64(MASK32)
    hi = idx >> np.uint64(32)
    seed = int(seed)
    x = philox4x32_10(lo, hi, np.uint64(sid), np.uint64(batch),
                      seed & MASK32, (seed >> 32) & MASK32)
    return np.stack(x, axis=1)


def uniforms(words):
    """Box-Muller inputs (u1 in (0,1], u2 in [0,1)) from Philox words."""
    w = words.astype(np.uint64)
    a = (w[:, 0] >> np.uint64(5)).astype(np.float64) * 67108864.0 \
        + (w[:, 1] >> np.uint64(6)).astype(np.float64)
    b = (w[:, 2] >> np.uint64(5)).astype(np.float64) * 67108864.0 \
        + (w[:, 3] >> np.uint64(6)).astype(np.float64)
    u1 = (a + 1.0) * 2.0 ** -53
    u2 = b * 2.0 ** -53
    return u1, u2


def normals(seed, sid, t0, count, batch=0):
    """Normal numbers t0 .. t0+count-1 of stream ``sid`` (FP64)."""
    if count <= 0:
        return np.zeros(0)
    p0 = t0 // 2
    p1 = (t0 + count - 1) // 2
    u1, u2 = uniforms(raw_words(seed, sid, p0, p1 - p0 + 1, batch))
    r = np.sqrt(-2.0 * np.log(u1))
    theta = TWO_PI * u2
    pair = np.empty(2 * len(r))
    pair[0::2] = r * np.cos(theta)
    pair[1::2] = r * np.sin(theta)
    off = t0 - 2 * p0
    return pair[off:off + count]


def sketch(seed, n, l, sid=STREAM_SKETCH, batch=0):
    """The n x l GIID sketch Omega: Omega[i, j] = normal number j*n + i."""
    z = normals(seed, sid, 0, n * l, batch)
    return z.reshape(l, n).T.copy()
