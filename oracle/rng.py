"""Random parameters of the two projections, from a 64-bit seed.

The paper draws the SEM hash h and signs (Section 2.2) and the SRFT diagonal
and column selection (Section 2.1) at random but fixes no generator.  Both
this oracle and the GPU library use one counter-based rule, each implemented
independently from its published definition:

* mix64 is the SplitMix64 output function (Steele, Lea & Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014; variant 13 of
  Stafford's 64-bit finalizers), gamma = 0x9E3779B97F4A7C15.
* stream key     K_t  = mix64(seed + t * gamma)   (t = 1 SEM, 2 signs d, 3 selection
                 of Omega_1; t = 4, 5, 6 the same three of Omega_2)
* draw i         r_t(i) = mix64(K_t + (i + 1) * gamma)       (all mod 2^64)
* SEM bucket     h(j)  = r_1(j) >> (64 - log2 s)   (uniform over [0, s))
* SEM sign       sgn(j) = 1 - 2 * (r_1(j) & 1)
* SRFT sign      d_b   = 1 - 2 * (r_2(b) >> 63)
* SRFT selection partial Fisher-Yates on [0, s): for i < l,
                 j = i + floor(r_3(i) * (s - i) / 2^64)  (multiply-high,
                 Lemire 2019, no rejection), swap idx[i], idx[j], sel[i] = idx[i].

Pure Python integers: slow, obviously exact.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
STREAM_SEM = 1
STREAM_SIGNS = 2
STREAM_SELECT = 3
STREAM_SEM2 = 4      # Omega_2 = Pi_2 S_2 of Algorithm 1 step 4: its SEM over the m rows,
STREAM_SIGNS2 = 5    # the SRFT diagonal and
STREAM_SELECT2 = 6   # the SRFT selection


def mix64(z: int) -> int:
    """SplitMix64 output function on a 64-bit integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(seed: int, count: int) -> list[int]:
    """Outputs of the classic SplitMix64 generator started at state ``seed``."""
    out, state = [], seed & MASK64
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(mix64(state))
    return out


def stream_key(seed: int, stream: int) -> int:
    return mix64((seed + stream * GAMMA) & MASK64)


def draw(key: int, i: int) -> int:
    return mix64((key + (i + 1) * GAMMA) & MASK64)


def _log2_exact(s: int) -> int:
    if s < 2 or s & (s - 1):
        raise ValueError("s must be a power of two >= 2")
    return s.bit_length() - 1


def sem_hash(seed: int, n: int, s: int, stream: int = STREAM_SEM):
    """Bucket h(j) in [0, s) and sign sgn(j) in {+1, -1} of every column j < n.

    Section 2.2: S = Phi D with Phi_{h(j), j} = 1 and D = diag(sgn).
    """
    b = _log2_exact(s)
    key = stream_key(seed, stream)
    h = np.empty(n, dtype=np.int64)
    sgn = np.empty(n, dtype=np.int64)
    for j in range(n):
        r = draw(key, j)
        h[j] = r >> (64 - b)
        sgn[j] = 1 - 2 * (r & 1)
    return h, sgn


def srft_signs(seed: int, s: int, stream: int = STREAM_SIGNS) -> np.ndarray:
    """Diagonal d_b in {+1, -1}, b < s (the real form of D in Section 2.1)."""
    _log2_exact(s)
    key = stream_key(seed, stream)
    return np.array([1 - 2 * (draw(key, b) >> 63) for b in range(s)], dtype=np.int64)


def srft_select(seed: int, s: int, l: int, stream: int = STREAM_SELECT) -> np.ndarray:
    """l distinct coordinates of [0, s) in draw order (the matrix S of Section 2.1)."""
    _log2_exact(s)
    if not 1 <= l <= s:
        raise ValueError("need 1 <= l <= s")
    key = stream_key(seed, stream)
    idx = list(range(s))
    sel = np.empty(l, dtype=np.int64)
    for i in range(l):
        j = i + ((draw(key, i) * (s - i)) >> 64)
        idx[i], idx[j] = idx[j], idx[i]
        sel[i] = idx[i]
    return sel
