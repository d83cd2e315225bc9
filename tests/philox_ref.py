"""Plain reference of the Philox4x32-10 generator (Salmon, Moraes, Dror and
Shaw, SC 2011) and of the Box-Muller white draws built on it, for checking the
device draws. Vectorised over counters with numpy uint64 arithmetic."""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten rounds on counter words (arrays or ints) with key (k0, k1)."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(k0 & MASK), np.uint64(k1 & MASK)
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c


def box_muller(b):
    a = (b[0] << np.uint64(32)) | b[1]
    c = (b[2] << np.uint64(32)) | b[3]
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = ((c >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def white_alm(ms, col, seed, counter):
    """w0 column `col` (ms: m of every coefficient)."""
    i = np.arange(ms.size, dtype=np.uint64)
    g0, g1 = box_muller(philox4x32_10(i, col, counter & MASK, counter >> 32, seed & MASK, seed >> 32))
    h = np.sqrt(0.5)
    return np.where(ms == 0, g0 + 0j, (g0 + 1j * g1) * h)


def white_map(npix, col, seed, counter):
    j = np.arange((npix + 1) // 2, dtype=np.uint64)
    g0, g1 = box_muller(philox4x32_10(j, col | 0x80000000, counter & MASK, counter >> 32, seed & MASK, seed >> 32))
    out = np.empty(2 * j.size)
    out[0::2], out[1::2] = g0, g1
    return out[:npix]
