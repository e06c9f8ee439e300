"""The approximate passes' bands (bf16 rows or 8-bit codes, float32
accumulation) against an emulation of that arithmetic on the CPU: a point
inside the radius must never compute above the band's upper edge, whatever
the summation order, for squared L2 and for the negated inner product."""
import numpy as np


def bf16_round(x):
    """float32 -> bfloat16 -> float32 with round-to-nearest-even."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def approx_sq(xb, q, rng):
    """float32 sum of squared differences in a random order (FMA emulated by
    rounding each product-sum once)."""
    order = rng.permutation(len(q))
    acc = np.float32(0)
    for i in order:
        t = np.float32(xb[i] - q[i])
        acc = np.float32(np.float64(t) * np.float64(t) + np.float64(acc))
    return acc


def band_hi(r2, maxnorm, d, margin):
    r = np.sqrt(r2)
    gamma = (d + 2) * 2.0 ** -24
    delta = max(margin * r, 2.0 ** -8 * maxnorm * (1 + 1e-6))
    return (1 + gamma) * (r + delta) ** 2


def test_band_never_rejects_an_inside_point():
    rng = np.random.default_rng(0)
    worst = 0.0
    for d in (8, 96, 768):
        for _ in range(300):
            q = rng.standard_normal(d).astype(np.float32)
            q /= np.linalg.norm(q)
            x = (q + rng.standard_normal(d).astype(np.float32) * rng.uniform(0.001, 0.2)).astype(np.float32)
            x /= np.linalg.norm(x)
            d64 = float(((x.astype(np.float64) - q) ** 2).sum())
            s = float(approx_sq(bf16_round(x), q, rng))
            # radius exactly at the point: the hardest case for the upper edge
            hi = band_hi(d64, 1.0, d, margin=0.0)
            assert s <= hi, (d, s, hi, d64)
            worst = max(worst, (s - d64) / max(hi - d64, 1e-30))
    assert worst < 1.0


def test_bf16_rounding_matches_definition():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: round to even gives 1
    assert bf16_round(np.array([1 + 2 ** -8], np.float32))[0] == 1.0
    assert bf16_round(np.array([1 + 3 * 2 ** -8], np.float32))[0] == 1 + 2 ** -6
    x = np.random.default_rng(1).standard_normal(1000).astype(np.float32)
    assert np.all(np.abs(bf16_round(x) - x) <= 2 ** -8 * np.abs(x))


def approx_ip(xb, q, rng):
    """float32 sum of products in a random order (one rounding per FMA)."""
    acc = np.float32(0)
    for i in rng.permutation(len(q)):
        acc = np.float32(np.float64(xb[i]) * np.float64(q[i]) + np.float64(acc))
    return acc


def band_ip(r, maxnorm, qnorm, d, margin):
    gamma = (d + 2) * 2.0 ** -24
    delta = max(margin * abs(r), (2.0 ** -8 + gamma * (1 + 2.0 ** -8)) * maxnorm * qnorm * (1 + 1e-6))
    return r - delta, r + delta


def test_inner_product_band_brackets_the_exact_distance():
    """d = -<x, q>: with r = d exactly, the approximate value lies inside
    [lo, hi] for rows of any norm and for cancelling sums."""
    rng = np.random.default_rng(2)
    worst = 0.0
    for d in (8, 96, 768):
        for k in range(300):
            q = (rng.standard_normal(d) * rng.uniform(0.1, 3.0)).astype(np.float32)
            x = (rng.standard_normal(d) * rng.uniform(0.1, 3.0)).astype(np.float32)
            if k % 3 == 0:  # nearly orthogonal: the sum cancels
                x = (x - q * np.float32(np.dot(x, q) / np.dot(q, q))).astype(np.float32)
            d64 = -float(np.dot(x.astype(np.float64), q.astype(np.float64)))
            s = -float(approx_ip(bf16_round(x), q, rng))
            maxnorm = float(np.linalg.norm(x.astype(np.float64)))
            lo, hi = band_ip(d64, maxnorm, float(np.linalg.norm(q.astype(np.float64))), d, 0.0)
            assert lo <= s <= hi, (d, s, lo, hi, d64)
            worst = max(worst, abs(s - d64) / (hi - d64))
    assert worst < 1.0


def sq8_params(base):
    """One affine map for all coordinates: lo rounded down and scale rounded
    up to float32 so that [lo, lo + 255 scale] covers every value."""
    mn, mx = float(base.min()), float(base.max())
    lo = np.float32(mn)
    if float(lo) > mn:
        lo = np.nextafter(lo, np.float32(-np.inf))
    span = (mx - float(lo)) / 255.0 if mx > mn else 1.0
    sc = np.float32(span)
    if float(sc) < span:
        sc = np.nextafter(sc, np.float32(np.inf))
    codes = np.clip(np.rint((base.astype(np.float64) - float(lo)) / float(sc)), 0, 255)
    return lo, sc, codes.astype(np.uint8)


def sq8_approx_l2(code, q, lo, sc, rng):
    qp = ((q.astype(np.float64) - float(lo)) / float(sc)).astype(np.float32)
    acc = np.float32(0)
    for i in rng.permutation(len(q)):
        t = np.float32(np.float32(code[i]) - qp[i])
        acc = np.float32(np.float64(t) * np.float64(t) + np.float64(acc))
    return np.float32(acc * np.float32(sc * sc))


def sq8_approx_ip(code, q, sc, rng):
    acc = np.float32(0)
    for i in rng.permutation(len(q)):
        acc = np.float32(np.float64(np.float32(code[i])) * np.float64(q[i]) + np.float64(acc))
    return np.float32(acc * np.float32(-sc))


def test_sq8_bands_bracket_the_exact_distance():
    rng = np.random.default_rng(3)
    u = 2.0 ** -24
    for d in (8, 96, 768):
        base = (rng.standard_normal((200, d)) * rng.uniform(0.05, 2.0, (200, 1))).astype(np.float32)
        lo, sc, codes = sq8_params(base)
        xh = float(lo) + float(sc) * codes.astype(np.float64)
        assert np.all(np.abs(xh - base) <= float(sc) / 2 * (1 + 1e-12))
        for k in range(100):
            q = (rng.standard_normal(d) * rng.uniform(0.05, 2.0)).astype(np.float32)
            i = k % len(base)
            x = base[i].astype(np.float64)
            # squared L2 at r = the exact distance
            e2 = float(((x - q) ** 2).sum())
            s = float(sq8_approx_l2(codes[i], q, lo, sc, rng))
            dl2 = float(((q.astype(np.float64) - float(lo)) ** 2).sum())
            delta = (0.5 * float(sc) * np.sqrt(d) + u * np.sqrt(dl2)) * (1 + 1e-6)
            g = (d + 4) * u
            r = np.sqrt(e2)
            hi = (1 + g) * (r + delta) ** 2
            lo_e = (1 - g) * (r - delta) ** 2 if r > delta else -1.0
            assert lo_e <= s <= hi, (d, s, lo_e, hi, e2)
            # negated inner product, in keys shifted by lo * sum(q)
            dip = -float(np.dot(x, q.astype(np.float64)))
            shift = float(lo) * float(q.astype(np.float64).sum())
            s = float(sq8_approx_ip(codes[i], q, sc, rng))
            delta = float(sc) * float(np.abs(q.astype(np.float64)).sum()) * (0.5 + 255 * (d + 2) * u) * (1 + 1e-6)
            assert dip + shift - delta <= s <= dip + shift + delta, (d, s, dip + shift, delta)
