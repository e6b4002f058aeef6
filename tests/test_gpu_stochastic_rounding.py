"""Stochastic rounding of the 16-bit g stores (lbm_encode16_stochastic, the
encoder the step kernels use) against its definition: the random bits of
the "lowbias32" counter-based hash of C. Wellons, keyed by step, node and
direction (written here from the published hash, not from the library), and
the rounding rule (add the top bits of r below the last kept bit of the
float, cut there).  Plus the statistics that make it worth having: every
result is one of the two neighbours of the input, and the error has mean
zero."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

M32 = np.uint64(0xFFFFFFFF)


def lowbias32(x):
    x = np.asarray(x, dtype=np.uint64) & M32
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & M32
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & M32
    x ^= x >> np.uint64(16)
    return x


def random_bits(step, n, direction):
    sk = lowbias32((np.uint64(step) * np.uint64(0x9E3779B9) + np.uint64(0x6A09E667)) & M32)
    nk = lowbias32(np.arange(n, dtype=np.uint64) ^ sk)
    return (nk + np.uint64(direction) * np.uint64(0x9E3779B9)) & M32


def expected(storage, x, step, direction):
    r = random_bits(step, x.size, direction)
    b = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    if storage == "bf16":
        return (((b + (r >> np.uint64(16))) & M32) >> np.uint64(16)).astype(np.uint16)
    t = ((b + (r >> np.uint64(19))) & np.uint64(0xFFFFE000)).astype(np.uint32)
    return t.view(np.float32).astype(np.float16).view(np.uint16)


def neighbours(storage, x):
    """The two format values around x (equal when x is exact), as floats."""
    if storage == "bf16":
        b = x.view(np.uint32)
        lo = (b & np.uint32(0xFFFF0000)).view(np.float32)
        hi = ((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
        hi = np.where(lo == x, lo, hi)
        return np.minimum(lo, hi), np.maximum(lo, hi)
    h = x.astype(np.float16)
    up = np.nextafter(h, np.float16(np.inf))
    dn = np.nextafter(h, np.float16(-np.inf))
    exact = h.astype(np.float32) == x
    lo = np.where(exact, h, np.where(h.astype(np.float32) < x, h, dn)).astype(np.float32)
    hi = np.where(exact, h, np.where(h.astype(np.float32) > x, h, up)).astype(np.float32)
    return lo, hi


def decode(storage, bits):
    bits = np.asarray(bits).view(np.uint16)
    if storage == "bf16":
        return (bits.astype(np.uint32) << np.uint32(16)).view(np.float32)
    return bits.view(np.float16).astype(np.float32)


@pytest.fixture(scope="module")
def hip():
    import torch
    assert torch.cuda.is_available()
    import paper_1110_5004_amd as P
    return P


def run(hip, storage, x, step, direction):
    import torch
    return hip.encode16_stochastic(storage, torch.from_numpy(x).cuda(), step,
                                   direction).cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_bits_match_definition(hip, storage):
    rng = np.random.default_rng(7)
    n = 200_003
    x = (rng.standard_normal(n) * np.exp(rng.uniform(-12, 9, n))).astype(np.float32)
    x[:6] = [0.0, -0.0, 1.0, np.inf, -np.inf, 3e-9]
    for step, direction in ((0, 0), (1, 5), (123456789, 18), (2**32 - 1, 1)):
        got = run(hip, storage, x, step, direction)
        want = expected(storage, x, step, direction)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (storage, step, direction, bad[:5], x[bad[:5]], got[bad[:5]],
                               want[bad[:5]])


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_neighbours_and_mean_zero(hip, storage):
    rng = np.random.default_rng(11)
    n = 1 << 20
    # normal-range values of the format, and Inf / NaN
    x = (rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n) *
         np.exp2(rng.integers(-10, 12, n))).astype(np.float32)
    got = decode(storage, run(hip, storage, x, 42, 3))
    lo, hi = neighbours(storage, x)
    assert np.all((got == lo) | (got == hi))
    # one value repeated: P(up) equals the fractional distance, the mean the value
    lo1, hi1 = neighbours(storage, np.array([1.0 + 0.3 * (2.0 ** -10 if storage == "fp16"
                                                          else 2.0 ** -7)], np.float32))
    v = np.float32(lo1[0] + 0.3 * (hi1[0] - lo1[0]))
    ups = np.zeros(4)
    for s in range(4):
        d = decode(storage, run(hip, storage, np.full(n, v, np.float32), 1000 + s, s))
        assert np.all((d == lo1[0]) | (d == hi1[0]))
        ups[s] = np.mean(d == hi1[0])
    p = (v - lo1[0]) / (hi1[0] - lo1[0])
    sigma = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(ups - p) < 5 * sigma), (ups, p, sigma)
    special = np.array([np.inf, -np.inf, np.nan, 0.0], np.float32)
    d = decode(storage, run(hip, storage, special, 9, 2))
    assert d[0] == np.inf and d[1] == -np.inf and np.isnan(d[2]) and d[3] == 0.0
