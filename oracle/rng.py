"""Random numbers for the recycled sketch operator G (oracle side; test infrastructure).

The paper draws G once and reuses it in every iteration (Alg. 1, "Generate a sketch
matrix"; §3.2.1).  It uses Gaussian entries in its experiments (§3.4, last paragraph)
and names the sparse-sign matrix as a cheaper alternative (§2.1 and §3.4).  It fixes
neither a generator nor a scaling; the reading used here (and, independently
implemented, on the GPU) is:

* counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11), written from that published definition;
* Gaussian entries: Box-Muller on two 53-bit uniforms, evaluated in FP64, rounded to
  FP32 and then to BF16 (round to nearest even), so G holds the same values in every
  precision form.  The scale is 1 (the estimator rho is invariant to scaling G);
* sparse-sign entries: zeta distinct rows per column of G drawn by Floyd's sampling
  algorithm (Bentley and Floyd, "A sample of brilliance", CACM 1987), each with a
  random sign.  Scale 1.
* subsampled randomized trigonometric transform (SRTT, named in §3.4 for very large m):
  G = sqrt(m/c) R F D with D a diagonal of random signs, F the orthonormal DCT-II of
  length m, and R keeping c distinct rows of F D drawn by Floyd's algorithm and listed
  in increasing order.  With this scale E ||G x||^2 = ||x||^2.

Counter layout (shared definition, implemented separately on each side):
  Gaussian entry G[r, i]     : ctr = (lo32(i), hi32(i), r, 0x47415553), key = (lo32(seed), hi32(seed))
  sparse-sign draw t, col i  : ctr = (lo32(i), hi32(i), t, 0x53505253), key = (lo32(seed), hi32(seed))
  SRTT sign d_i              : ctr = (lo32(i), hi32(i), 0, 0x53525444), bit 0 of x0 set = -1
  SRTT row draw t            : ctr = (t, 0, 0, 0x53525452), v = (x1 * 2^32 + x0) mod (j + 1)
"""
import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint32(0x9E3779B9)
PHILOX_W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

TAG_GAUSS = 0x47415553
TAG_SIGN = 0x53505253
TAG_SRTT_SIGN = 0x53525444
TAG_SRTT_ROWS = 0x53525452


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of 32-bit counters and a 2x32 key.

    One round maps (x0, x1, x2, x3) to (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2),
    hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); between rounds the key is bumped by the Weyl
    constants (W0, W1).  Returns four uint32 arrays.
    """
    x0 = np.asarray(c0, dtype=np.uint64) & MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & MASK32
    ka = np.uint32(k0)
    kb = np.uint32(k1)
    for rnd in range(10):
        if rnd > 0:
            ka = np.uint32((int(ka) + int(PHILOX_W0)) & 0xFFFFFFFF)
            kb = np.uint32((int(kb) + int(PHILOX_W1)) & 0xFFFFFFFF)
        p0 = PHILOX_M0 * x0          # exact: both factors < 2**32
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(ka), lo1, hi0 ^ x3 ^ np.uint64(kb), lo0)
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def _seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def round_to_bf16(x):
    """FP64 -> FP32 (IEEE round to nearest even) -> BF16 (round to nearest even on the
    FP32 bit pattern), returned as FP64 values.  Inputs are finite."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    out = (bits << np.uint64(16)).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def gaussian_entries(seed, rows, cols):
    """G[r, i] for r in rows, i in cols (outer grid): Box-Muller standard normal from
    one Philox block, z = sqrt(-2 ln u1) cos(2 pi u2), rounded to BF16 values."""
    rows = np.asarray(rows, dtype=np.uint64)
    cols = np.asarray(cols, dtype=np.uint64)
    R, C = np.meshgrid(rows, cols, indexing="ij")
    k0, k1 = _seed_key(seed)
    x0, x1, x2, x3 = philox4x32_10(C & MASK32, C >> np.uint64(32), R,
                                   np.full(R.shape, TAG_GAUSS, np.uint64), k0, k1)
    a = ((x1.astype(np.uint64) << np.uint64(32)) | x0.astype(np.uint64)) >> np.uint64(11)
    b = ((x3.astype(np.uint64) << np.uint64(32)) | x2.astype(np.uint64)) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53          # (0, 1]
    u2 = b.astype(np.float64) * 2.0 ** -53                  # [0, 1)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
    return round_to_bf16(z)


def gaussian_G(seed, c, m):
    """Dense c x m Gaussian sketch operator (FP64 array holding BF16 values)."""
    return gaussian_entries(seed, np.arange(c), np.arange(m))


def sparse_sign_pattern(seed, c, m, zeta=8):
    """For each column i of G (one per row of A): zeta' = min(zeta, c) distinct row
    indices in [0, c) and signs in {+1, -1}.

    Floyd's algorithm: for t = 0 .. zeta'-1 with j = c - zeta' + t, draw v uniform on
    [0, j] (as the Philox word x0 modulo j+1); insert v unless it is already chosen,
    in which case insert j.  The sign of the t-th inserted row is + when bit 0 of the
    Philox word x1 is 0.  Returns (rows int64 [m, zeta'], signs float64 [m, zeta']).
    """
    z = min(int(zeta), int(c))
    k0, k1 = _seed_key(seed)
    i = np.arange(m, dtype=np.uint64)
    rows = np.zeros((m, z), dtype=np.int64)
    signs = np.zeros((m, z), dtype=np.float64)
    for t in range(z):
        j = c - z + t
        x0, x1, _, _ = philox4x32_10(i & MASK32, i >> np.uint64(32),
                                     np.full(m, t, np.uint64), np.full(m, TAG_SIGN, np.uint64),
                                     k0, k1)
        v = (x0.astype(np.int64)) % (j + 1)
        taken = np.zeros(m, dtype=bool)
        for s in range(t):
            taken |= rows[:, s] == v
        rows[:, t] = np.where(taken, j, v)
        signs[:, t] = np.where((x1 & np.uint32(1)) == 0, 1.0, -1.0)
    return rows, signs


def sparse_sign_G(seed, c, m, zeta=8):
    """Dense c x m materialisation of the sparse-sign operator."""
    rows, signs = sparse_sign_pattern(seed, c, m, zeta)
    G = np.zeros((c, m), dtype=np.float64)
    for t in range(rows.shape[1]):
        G[rows[:, t], np.arange(m)] = signs[:, t]
    return G


def srtt_signs(seed, m):
    """Diagonal of D: d_i = -1 when bit 0 of the Philox word x0 for column i is set."""
    k0, k1 = _seed_key(seed)
    i = np.arange(m, dtype=np.uint64)
    x0, _, _, _ = philox4x32_10(i & MASK32, i >> np.uint64(32), np.zeros(m, np.uint64),
                                np.full(m, TAG_SRTT_SIGN, np.uint64), k0, k1)
    return np.where((x0 & np.uint32(1)) == 0, 1.0, -1.0)


def srtt_rows(seed, c, m):
    """The c distinct kept rows of F D in increasing order (Floyd's algorithm: for
    t = 0 .. c-1 with j = m - c + t draw v uniform on [0, j] from the 64-bit Philox value
    x1 * 2^32 + x0 modulo j + 1; insert v unless already chosen, else insert j)."""
    if c > m:
        raise ValueError("SRTT needs c <= m")
    k0, k1 = _seed_key(seed)
    chosen = set()
    for t in range(c):
        j = m - c + t
        x0, x1, _, _ = philox4x32_10(np.uint64(t), np.uint64(0), np.uint64(0),
                                     np.uint64(TAG_SRTT_ROWS), k0, k1)
        v = ((int(x1) << 32) | int(x0)) % (j + 1)
        chosen.add(j if v in chosen else v)
    return np.array(sorted(chosen), dtype=np.int64)


def srtt_G(seed, c, m):
    """Dense c x m SRTT operator sqrt(m/c) R F D (FP64), from the DCT-II definition
    F[r, i] = s_r cos(pi r (2 i + 1) / (2 m)), s_0 = sqrt(1/m), s_r = sqrt(2/m).  The
    angle is reduced exactly as q = r (2 i + 1) mod 4 m before the cosine."""
    rows = srtt_rows(seed, c, m)
    d = srtt_signs(seed, m)
    i = np.arange(m, dtype=np.int64)
    q = (rows[:, None] * (2 * i[None, :] + 1)) % (4 * m)
    F = np.cos(np.pi * q.astype(np.float64) / (2.0 * m))
    scale = np.where(rows == 0, np.sqrt(1.0 / m), np.sqrt(2.0 / m)) * np.sqrt(m / c)
    return F * scale[:, None] * d[None, :]


def make_G(seed, c, m, kind, zeta=8):
    """The recycled sketch operator G (c x m).  kind 0: Gaussian, 1: sparse-sign,
    2: SRTT."""
    if kind == 0:
        return gaussian_G(seed, c, m)
    if kind == 1:
        return sparse_sign_G(seed, c, m, zeta)
    if kind == 2:
        return srtt_G(seed, c, m)
    raise ValueError("unknown sketch kind %r" % (kind,))


def g_scale(kind, c, zeta=8):
    """s with E ||G x||^2 = s^2 ||x||^2 for the operator make_G returns: sqrt(c) for the
    unscaled Gaussian, sqrt(min(zeta, c)) for the sparse-sign operator, 1 for SRTT."""
    if kind == 0:
        return float(np.sqrt(c))
    if kind == 1:
        return float(np.sqrt(min(int(zeta), int(c))))
    if kind == 2:
        return 1.0
    raise ValueError("unknown sketch kind %r" % (kind,))
