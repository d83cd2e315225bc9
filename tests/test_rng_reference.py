"""Pins of the Philox4x32-10 reference used to check the device white draws:
the known-answer vectors of the generator's authors (SC 2011 release), and the
first two moments of the Box-Muller draws built on it."""
import numpy as np

from tests.philox_ref import box_muller, philox4x32_10, white_alm, white_map


def test_philox_known_answers():
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = tuple(int(v) for v in philox4x32_10(*ctr, *key))
        assert got == want, (ctr, [hex(v) for v in got])


def test_box_muller_moments_and_white_layouts():
    n = 400_000
    g0, g1 = box_muller(philox4x32_10(np.arange(n), 7, 3, 0, 12345, 678))
    for g in (g0, g1):
        assert abs(g.mean()) < 5.0 / np.sqrt(n)
        assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
        assert abs(np.mean(g ** 4) - 3.0) < 0.05
    assert abs(np.mean(g0 * g1)) < 5.0 / np.sqrt(n)
    ms = np.concatenate([np.full(200 - m + 1, m) for m in range(201)])
    a = white_alm(ms, 0, 99, 5)
    assert np.all(a[ms == 0].imag == 0.0)
    re, im = a[ms > 0].real, a[ms > 0].imag
    assert abs(re.var() - 0.5) < 0.02 and abs(im.var() - 0.5) < 0.02
    w = white_map(1001, 2, 99, 5)
    assert w.size == 1001 and abs(w.var() - 1.0) < 0.2
    # columns, counters and the two purposes are different streams
    assert not np.allclose(white_map(64, 0, 99, 5), white_map(64, 1, 99, 5))
    assert not np.allclose(white_map(64, 0, 99, 5), white_map(64, 0, 99, 6))
    assert not np.allclose(white_alm(ms[:32], 0, 99, 5).real, white_map(64, 0, 99, 5)[:32])
