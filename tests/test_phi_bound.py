"""The trilinear fraction phi = log2(m), m in [1, 2), as the kernels evaluate
it in float32 -- s = (m - 1) rcp(m + 1), then eight odd terms of
(2 / ln 2) atanh(s) by Horner's rule -- stays within the 4e-7 absolute bar
of the GPU trace test for every float32 mantissa, even when the reciprocal
is off by a whole ulp either way (the hardware reciprocal's accuracy).
Likewise 1 - phi = log2(2 / m) from (2 - m) / (2 + m)."""
import numpy as np

F = np.float32


def _series(num, den, rcp_ulps):
    r = (F(1.0) / den).astype(np.float32)
    r = np.nextafter(r, np.float32(np.inf) if rcp_ulps > 0 else np.float32(0)) \
        if rcp_ulps else r
    s = (num * r).astype(np.float32)
    s2 = (s * s).astype(np.float32)
    c = [F(2.0 / np.log(2.0) / (2 * i + 1)) for i in range(8)]
    p = np.full_like(s, c[7])
    for i in range(6, -1, -1):
        # fused multiply-add: one rounding of the exact p * s2 + c
        p = (p.astype(np.float64) * s2.astype(np.float64) + np.float64(c[i])).astype(np.float32)
    return (s * p).astype(np.float32)


def test_phi_within_bound_for_every_mantissa():
    m = (np.arange(1 << 23, dtype=np.uint32) | np.uint32(0x3F800000)).view(np.float32)
    exact = np.log2(m.astype(np.float64))
    for ulps in (0, 1, -1):
        phi = _series((m - F(1)).astype(np.float32), (m + F(1)).astype(np.float32), ulps)
        om0 = _series((F(2) - m).astype(np.float32), (F(2) + m).astype(np.float32), ulps)
        assert np.abs(phi - exact).max() <= 4e-7
        assert np.abs(om0 - (1.0 - exact)).max() <= 4e-7
    # and the coefficients are the series' own terms
    c = [2.0 / np.log(2.0) / (2 * i + 1) for i in range(8)]
    assert abs(c[0] - 2.885390082) < 1e-9 and abs(c[7] - 0.1923593388) < 1e-9
