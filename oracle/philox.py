"""Counter-based random numbers for the test matrices the method draws.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

The randomized range finders draw a random test matrix Omega: a standard
Gaussian n x l matrix for Algorithm 4.1 (Section 4.1), or the SRFT
Omega = sqrt(n/l) D F R of Section 4.6, whose random parts are the diagonal D
and the column sampler R.  The GPU library draws the same numbers on the
device from its own, independently written implementation of the same
published generator, so both sides consume identical test matrices without one
ever reading the other's output.

Generator contract (written out here and implemented twice)
------------------------------------------------------------
* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 10 rounds of the 4x64 Philox S-box with multipliers
  0xD2E7470EE14C6C93, 0xCA5A826395121157 and Weyl key increments
  0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B.  Key (k0, k1) = (seed, 0).  The
  bijection is applied to the counter as given (nothing is incremented first).
* Uniform: u(w) = ((w >> 12) + 1/2) * 2^-52.  Every step is exact in FP64
  (w >> 12 < 2^52), so u lies strictly inside (0, 1) on any machine.
* Gaussian Omega (n x l, row-major) for stream s: entry (i, j) belongs to quad
  t = i * ceil(l/4) + floor(j/4); counter (t, s, 0, 0) gives words w0..w3 and
  uniforms u0..u3; the Box-Muller pairs are
      g0, g1 = sqrt(-2 ln u0) * (cos th, sin th),  th = TWO_PI * u1
      g2, g3 = sqrt(-2 ln u2) * (cos th', sin th'), th' = TWO_PI * u3
  with TWO_PI the double nearest 2*pi, and Omega[i, 4*floor(j/4) + r] = g_r.
  Entries of a quad that fall past column l - 1 are dropped.
* SRFT diagonal (real +-1 signs): d_p = 1 - 2 * (w0 & 1) with w0 from counter
  (p, s, 1, 0).
* SRFT sampler: a partial Fisher-Yates shuffle of [0, n).  Step t = 0..l-1 takes
  w0 from counter (t, s, 2, 0), sets j = min(t + floor(u(w0) * (n - t)), n - 1)
  (the product can round up to n - t when u is within an ulp of 1) and swaps
  perm[t] with perm[j]; R[t] = perm[t].  R lists l distinct coordinates in draw
  order, so the sample is uniform without replacement as Section 4.6 requires.
* GSRFT (the Givens-chain transform of the remark on random Givens rotations in
  Section 4.6), chain c = 0 (Theta, D') and c = 1 (Theta', D''):
    - signs: d_p = 1 - 2 * (w0 & 1), w0 from counter (p, s, 3, c) (D' for c = 0,
      D'' for c = 1);
    - angles: theta_j = TWO_PI * u(w0), w0 from counter (j, s, 4, c),
      j = 0..n-2 (the rotation in the coordinate plane (j, j + 1));
    - permutation: key_p = ((w0 >> 16) << 16) | p with w0 from counter
      (p, s, 5, c); pi lists the indices p in increasing order of key_p (the top
      48 bits of w0, ties broken by p), a uniformly random permutation of [0, n)
      for n <= 2^16.
* Streams: s = 0 for a single matrix, s = 10 + b for matrix b of a batch.
"""

import numpy as np

PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
ROUNDS = 10

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)
TWO_PI = 2.0 * np.pi  # doubling is exact, so this is the double nearest 2*pi

KIND_GAUSS = 0
KIND_SRFT_SIGN = 1
KIND_SRFT_SAMPLE = 2
KIND_GIVENS_SIGN = 3
KIND_GIVENS_ANGLE = 4
KIND_GIVENS_PERM = 5


def _mulhilo(a, b):
    """Full 64x64 -> 128 bit product of a Python-int constant a and uint64 array b.

    Returns (hi, lo), both uint64 arrays.  Plain schoolbook on 32-bit limbs.
    """
    a = np.uint64(a)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    # The middle column: at most (2^32-1) + (2^32-1) + (2^32-1)^2 < 2^64.
    mid = (ll >> _S32) + (hl & _M32) + lh
    hi = hh + (hl >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (ll & _M32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1=0):
    """Philox4x64-10 of counter (c0..c3) under key (k0, k1).

    Arguments broadcast as uint64 arrays; returns the four output words.
    """
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        x0, x1, x2, x3 = (v.copy() for v in (x0, x1, x2, x3))
        key0 = int(k0) & 0xFFFFFFFFFFFFFFFF
        key1 = int(k1) & 0xFFFFFFFFFFFFFFFF
        for _ in range(ROUNDS):
            hi0, lo0 = _mulhilo(PHILOX_M0, x0)
            hi1, lo1 = _mulhilo(PHILOX_M1, x2)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(key0), lo1,
                              hi0 ^ x3 ^ np.uint64(key1), lo0)
            key0 = (key0 + PHILOX_W0) & 0xFFFFFFFFFFFFFFFF
            key1 = (key1 + PHILOX_W1) & 0xFFFFFFFFFFFFFFFF
    return x0, x1, x2, x3


def uniform_from_word(w):
    """u = ((w >> 12) + 1/2) * 2^-52: 52 random bits centred in their bin, exact in FP64."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def gaussian_omega(n, l, seed, stream=0):
    """Standard Gaussian n x l test matrix (Algorithm 4.1, step 1), FP64.

    Follows the Gaussian part of the generator contract in the module
    docstring: one Philox call per quad of four horizontally adjacent entries,
    Box-Muller on two uniform pairs.
    """
    n, l = int(n), int(l)
    quads_per_row = (l + 3) // 4
    t = np.arange(n * quads_per_row, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x64(t, np.uint64(stream), np.uint64(KIND_GAUSS), 0, seed)
    u0, u1, u2, u3 = (uniform_from_word(w) for w in (w0, w1, w2, w3))
    r01 = np.sqrt(-2.0 * np.log(u0))
    r23 = np.sqrt(-2.0 * np.log(u2))
    th01 = TWO_PI * u1
    th23 = TWO_PI * u3
    g = np.stack([r01 * np.cos(th01), r01 * np.sin(th01),
                  r23 * np.cos(th23), r23 * np.sin(th23)], axis=1)
    g = g.reshape(n, quads_per_row * 4)
    return np.ascontiguousarray(g[:, :l])


def srft_signs(n, seed, stream=0):
    """Random +-1 diagonal D of the SRFT (Section 4.6), as a length-n FP64 vector."""
    p = np.arange(int(n), dtype=np.uint64)
    w0, _, _, _ = philox4x64(p, np.uint64(stream), np.uint64(KIND_SRFT_SIGN), 0, seed)
    return 1.0 - 2.0 * (w0 & np.uint64(1)).astype(np.float64)


def srft_sample(n, l, seed, stream=0):
    """l coordinates of [0, n) drawn uniformly without replacement (the R of Section 4.6).

    Partial Fisher-Yates shuffle, one plain Python step per draw.
    """
    n, l = int(n), int(l)
    if l > n:
        raise ValueError("cannot sample more coordinates than n")
    t = np.arange(l, dtype=np.uint64)
    w0, _, _, _ = philox4x64(t, np.uint64(stream), np.uint64(KIND_SRFT_SAMPLE), 0, seed)
    u = uniform_from_word(w0)
    perm = list(range(n))
    out = []
    for step in range(l):
        j = min(step + int(np.floor(u[step] * float(n - step))), n - 1)
        perm[step], perm[j] = perm[j], perm[step]
        out.append(perm[step])
    return np.array(out, dtype=np.int64)


def givens_signs(n, seed, chain, stream=0):
    """The +-1 diagonal of GSRFT chain `chain` (D' for 0, D'' for 1), length-n FP64."""
    p = np.arange(int(n), dtype=np.uint64)
    w0, _, _, _ = philox4x64(p, np.uint64(stream), np.uint64(KIND_GIVENS_SIGN), np.uint64(chain), seed)
    return 1.0 - 2.0 * (w0 & np.uint64(1)).astype(np.float64)


def givens_angles(n, seed, chain, stream=0):
    """theta_0 .. theta_{n-2} of GSRFT chain `chain`, uniform on [0, 2 pi), FP64."""
    j = np.arange(max(int(n) - 1, 0), dtype=np.uint64)
    w0, _, _, _ = philox4x64(j, np.uint64(stream), np.uint64(KIND_GIVENS_ANGLE), np.uint64(chain), seed)
    return TWO_PI * uniform_from_word(w0)


def givens_permutation(n, seed, chain, stream=0):
    """pi of GSRFT chain `chain`: the indices p ordered by ((w0 >> 16) << 16) | p (n <= 2^16)."""
    n = int(n)
    if n > 1 << 16:
        raise ValueError("the permutation key holds the index in 16 bits")
    p = np.arange(n, dtype=np.uint64)
    w0, _, _, _ = philox4x64(p, np.uint64(stream), np.uint64(KIND_GIVENS_PERM), np.uint64(chain), seed)
    keys = ((w0 >> np.uint64(16)) << np.uint64(16)) | p
    return (np.sort(keys) & np.uint64(0xFFFF)).astype(np.int64)


def round_to_dtype(x, dtype):
    """Round an FP64 array to the working dtype by IEEE round-to-nearest-even."""
    return np.asarray(x, dtype=np.float64).astype(dtype).astype(np.float64)
