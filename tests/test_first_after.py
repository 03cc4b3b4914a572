"""Host model of the row passes' division (first_after in edt_internal.h): the
first pixel past an intersection of Eq. eq_intersection, floor(num / den) + 1
clamped to [0, W], computed from a float estimate of the quotient (num and
the reciprocal of den rounded to fp32, their product rounded to fp32,
clamped to [-1, W], then truncated) and one integer correction step.  The hardware
reciprocal is accurate to about one ulp; here it is modelled as the correctly
rounded reciprocal moved by -2 .. +2 ulp, and the result must equal the exact floor
for every denominator 2 <= den < 2^16, for W up to 2^15 - 1, at the numerators
where an error would show: each multiple of den and its neighbours, for
quotients across the whole clamped range, and the largest numerators below
2^31."""
import numpy as np
import pytest


def model(num, den, W, ulps):
    """first_after with the reciprocal of den moved by `ulps` ulp."""
    num = np.asarray(num, np.int64)
    den = np.asarray(den, np.int64)
    rcp = (np.float32(1.0) / den.astype(np.float32)).astype(np.float32)
    if ulps:
        toward = np.float32(np.inf) if ulps > 0 else np.float32(0.0)
        for _ in range(abs(ulps)):
            rcp = np.nextafter(rcp, toward).astype(np.float32)
    qf = (num.astype(np.float32) * rcp).astype(np.float32)
    q = np.trunc(np.clip(qf, np.float32(-1.0), np.float32(W))).astype(np.int64)
    r = num - q * den
    q = q + (r >= den) - (r < 0)
    return np.where(num < 0, 0, np.minimum(q + 1, W))


def exact(num, den, W):
    num = np.asarray(num, np.int64)
    den = np.asarray(den, np.int64)
    return np.clip(np.floor_divide(num, den) + 1, 0, W)


DENS = np.arange(2, 1 << 16, dtype=np.int64)


@pytest.mark.parametrize("W", [1, 2, 64, 1023, 1024, 4097, 16384, 32767])
@pytest.mark.parametrize("ulps", [-2, -1, 0, 1, 2])
def test_first_after_is_the_exact_floor(W, ulps):
    # quotients spread over [0, W + 2] (denser at the top, where the float
    # estimate's absolute error is largest), each with remainders 0, 1,
    # den - 1 and the neighbouring multiples
    qs = np.unique(np.concatenate([np.arange(0, min(W + 3, 40)),
                                   np.linspace(0, W + 2, 24).astype(np.int64),
                                   np.arange(max(0, W - 6), W + 3)]))
    for q in qs:
        base = q * DENS
        for off in (-1, 0, 1):
            for num in (base + off, base + DENS - 1 + off):
                ok = (num >= -(1 << 16)) & (num < (1 << 31))
                n, d = num[ok], DENS[ok]
                got = model(n, d, W, ulps)
                want = exact(n, d, W)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (W, ulps, int(n[bad[0]]), int(d[bad[0]]))


@pytest.mark.parametrize("ulps", [-2, 0, 2])
def test_first_after_at_the_largest_numerators(ulps):
    # numerators up to (H - 1)^2 + (W - 1)^2 - 1 for sides of 32767, against
    # every denominator: the quotient then lies far past any W and clamps
    W = 32767
    for num in ((1 << 31) - 1, 2 * 32766 * 32766, (1 << 30) + 12345):
        n = np.full(DENS.shape, num, np.int64)
        assert np.array_equal(model(n, DENS, W, ulps), exact(n, DENS, W))
    # and quotients just below W for the largest denominators
    d = DENS[-4096:]
    for q in (W - 2, W - 1, W):
        for r in (0, 1):
            n = q * d + r
            n = n[n < (1 << 31)]
            dd = d[: n.size]
            assert np.array_equal(model(n, dd, W, ulps), exact(n, dd, W))
