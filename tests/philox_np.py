"""A second, independent Philox4x32-10 written for the tests in vectorised NumPy.

Written from the round definition in Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): each round multiplies counter words
0 and 2 by two fixed odd constants, forms the four output words from the high
halves xor-ed with the other counter words and the round key, and the low halves;
the key advances by two Weyl constants per round.  Ten rounds.
"""
import numpy as np

_MUL_A = np.uint64(0xD2511F53)
_MUL_B = np.uint64(0xCD9E8D57)
_WEYL_A = 0x9E3779B9
_WEYL_B = 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised over numpy arrays of uint32 counters; scalar key words."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        pa = _MUL_A * c0
        pb = _MUL_B * c2
        new0 = (pb >> np.uint64(32)) ^ c1 ^ np.uint64(ka)
        new1 = pb & _LO
        new2 = (pa >> np.uint64(32)) ^ c3 ^ np.uint64(kb)
        new3 = pa & _LO
        c0, c1, c2, c3 = new0, new1, new2, new3
        ka = (ka + _WEYL_A) & 0xFFFFFFFF
        kb = (kb + _WEYL_B) & 0xFFFFFFFF
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32), c3.astype(np.uint32))


def site_keys(seed: int, sample: int, sites, tag: int = 0):
    """64-bit keys of sites i: the Philox block of counter (i // 2, lo(sample),
    hi(sample), tag) under key (lo(seed), hi(seed)) gives K = (word1 << 32) |
    word0 to even i and (word3 << 32) | word2 to odd i."""
    sites = np.asarray(sites, dtype=np.uint64)
    n = sites.shape
    o0, o1, o2, o3 = philox4x32_10(
        sites >> np.uint64(1),
        np.full(n, sample & 0xFFFFFFFF, dtype=np.uint64),
        np.full(n, (sample >> 32) & 0xFFFFFFFF, dtype=np.uint64),
        np.full(n, tag, dtype=np.uint64),
        seed & 0xFFFFFFFF,
        (seed >> 32) & 0xFFFFFFFF,
    )
    even = (o1.astype(np.uint64) << np.uint64(32)) | o0.astype(np.uint64)
    odd = (o3.astype(np.uint64) << np.uint64(32)) | o2.astype(np.uint64)
    return np.where((sites & np.uint64(1)) == 0, even, odd)
