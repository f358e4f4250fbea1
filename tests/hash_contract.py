"""The biclique hash written out in plain Python integers, for pinning the oracle's C version.

It is the library's hash contract: with mix the SplitMix64 output function (Steele, Lea and
Flood, OOPSLA 2014) and K = 0x9E3779B97F4A7C15, all arithmetic mod 2^64,

    hu(a) = mix(K (2a + 1))   for a in U,      hv(b) = mix(K (2b + 2))   for b in V,
    h(A, B) = mix(sum_{a in A} hu(a) + mix(sum_{b in B} hv(b) + K)),
    H = sum of h over the maximal bicliques.

The tests check ``mix`` here against the published first outputs of SplitMix64 before they
use it; this module imports nothing from the oracle or the library.
"""
M64 = (1 << 64) - 1
K = 0x9E3779B97F4A7C15


def mix(z: int) -> int:
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def hu(a: int) -> int:
    return mix(K * (2 * a + 1))


def hv(b: int) -> int:
    return mix(K * (2 * b + 2))


def h(A, B) -> int:
    sa = sum(hu(a) for a in A) & M64
    sb = sum(hv(b) for b in B) & M64
    return mix(sa + mix(sb + K))


def total(records) -> int:
    """H of a list of (A, B) records."""
    s = 0
    for a, b in records:
        s = (s + h(a, b)) & M64
    return s
