"""The seeded texel fills: the Perlin gradient noise fill, in exact integer
arithmetic, against Perlin's formula evaluated in float64 (fade
6t^5 - 15t^4 + 10t^3, dot products of lattice gradients with corner
offsets); its range; the fade table's symmetry; mirrored boundary
content."""
import numpy as np

from htexgen import texels as T


def test_fade_table_is_perlins_quintic_and_symmetric():
    t = (2 * np.arange(8) + 1) / 16.0
    np.testing.assert_array_equal(T.FADE, np.round((6 * t ** 5 - 15 * t ** 4 + 10 * t ** 3)
                                                   * 2 ** 20).astype(np.int64))
    # fade(1 - t) = 1 - fade(t), exactly
    np.testing.assert_array_equal(T.FADE + T.FADE[::-1], np.full(8, 1 << 20))


def test_perlin_fill_equals_the_float_formula_to_its_rounding():
    n = 64
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for e in (0, 3, 17, 396965):
        for c in range(4):
            v = T.texel_values(T.PERLIN, 202, e, n, False, i, j, c).astype(np.float64)
            ref = T.perlin_reference(202, e, c, i, j)
            # v = 1/64 + (62/64)(1/2 + noise/2), noise rounded down to 2^-18
            noise = ((v * 2 ** 24 - 2 ** 18) / 31 - 2 ** 18) / 2 ** 18
            assert np.all(noise <= ref + 1e-12)
            assert np.all(noise >= ref - 2.0 ** -18 - 1e-12)
            assert v.min() >= 1 / 64 and v.max() <= 63 / 64


def test_perlin_noise_is_smooth_and_varies():
    """Gradient noise is continuous across cells: neighbouring texels differ
    far less than the spread of values, and a cell corner's value is
    reached from both sides."""
    n = 64
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v = T.texel_values(T.PERLIN, 5, 11, n, False, i, j, 0).astype(np.float64)
    assert v.std() > 0.05
    assert np.abs(np.diff(v, axis=1)).max() < 0.25 * (v.max() - v.min())
    assert np.abs(np.diff(v, axis=0)).max() < 0.25 * (v.max() - v.min())


def test_boundary_edges_mirror_their_lower_left_half():
    n = 16
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for kind in (T.UNIFORM, T.SMOOTH, T.PERLIN):
        v = T.texel_values(kind, 9, 4, n, True, i, j, 1)
        np.testing.assert_array_equal(v, v[::-1, ::-1].T)
