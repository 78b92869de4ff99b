"""Philox4x32-10 and the random maps used by the sampler (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Philox4x32 with R = 10 rounds is the counter-based bijection of Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1); each round
multiplies c0 and c2 by the constants M0, M1 into 64-bit products and mixes
hi/lo halves with the other two words and the key; the key is bumped by the
Weyl constants W0, W1 between rounds.  Written here from that definition with
Python integers, so there is no overflow subtlety to get wrong.

The paper only says that a random permutation m of the orbital indices is
drawn first (text after Eq. (2)) and that each x_k is then drawn from its
conditional; it fixes no generator.  The stream layout below is this
project's reading (it is the same on the GPU side):
  key     = (seed mod 2^32, seed >> 32)
  counter = (sample mod 2^32, sample >> 32, step, 0),   step = k - 1 (0-based)
(word 3 = 1 is the eigenvector-selection stream of the DPP front end, dpp.py)
One Philox block per (sample, step) gives four words w0..w3:
  * column draw (lazy Fisher-Yates): j = step + floor(((w1<<32)|w0) * R / 2^64)
    with R = N - step candidates left (64-bit multiply-high, no rejection;
    bias at most R/2^64);
  * uniform for the inverse-CDF draw: u = (((w3<<32)|w2) >> 11) * 2^-53,
    a 53-bit dyadic number in [0, 1).
"""

MASK32 = 0xFFFFFFFF
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC'11).  Returns 4 words."""
    c0, c1, c2, c3 = (int(c) & MASK32 for c in ctr)
    k0, k1 = (int(k) & MASK32 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK32,
                          (p0 >> 32) ^ c3 ^ k1, p0 & MASK32)
    return c0, c1, c2, c3


def stream_words(seed, sample, step, stream):
    """The Philox block with counter (sample lo, sample hi, step, stream)."""
    seed = int(seed)
    sample = int(sample)
    return philox4x32_10((sample & MASK32, sample >> 32, int(step), int(stream)),
                         (seed & MASK32, seed >> 32))


def step_words(seed, sample, step):
    """The Philox block owned by (seed, sample, step): the sampler's stream 0."""
    return stream_words(seed, sample, step, 0)


def fisher_yates_index(words, step, n):
    """Index j in [step, n) of the lazy Fisher-Yates swap at `step`."""
    r = n - step
    v = (words[1] << 32) | words[0]
    return step + ((v * r) >> 64)


def uniform53(words):
    """u in [0, 1) with 53 random bits, exactly representable in float64."""
    v = (words[3] << 32) | words[2]
    return float(v >> 11) * (2.0 ** -53)
