"""Gaussian test matrices from a counter-based generator (oracle side).

The paper draws the sketching matrix Omega with i.i.d. entries from a
prescribed distribution, Gaussian for the random-projection HOSVD
(Section 3.1, eq. proj and Algorithm 1 step 1; Algorithm 6 step 3 names a
Gaussian matrix).  It does not say how the numbers are produced.  This
package fixes a reproducible definition so that the CPU oracle and the GPU
kernels can draw the *same* Omega without storing it:

* Generator: Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw,
  "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter,
  a 2x32-bit key, ten rounds, round multipliers 0xD2511F53 / 0xCD9E8D57 and
  Weyl key increments 0x9E3779B9 / 0xBB67AE85.
* Key = (low 32 bits of seed, high 32 bits of seed).
* Omega_n has J rows and K columns; entry (c, k) (0-based) has linear index
  e = k*J + c (column-major, so a larger oversampling keeps the smaller
  Omega as its leading columns).
* Row c of the generated matrix belongs to the unfolding column whose
  position in the *cyclic* order of the remaining modes is c: with the tensor
  of shape (I_1, ..., I_N) and mode n, the remaining indices are enumerated
  as i_{n+1}, ..., i_N, i_1, ..., i_{n-1}, the first of them fastest (the
  unfolding of De Lathauwer, De Moor and Vandewalle, SIMAX 2000).  The
  paper's n-unfolding (Section 2) orders the same columns with i_1 fastest;
  for a column j = l + L t of it (l over the modes before n, L their size,
  t over the modes after n, T their size) the cyclic position is
  c = t + T l.  This is a fixed row permutation of an i.i.d. Gaussian
  matrix, so Omega keeps its distribution; omega_unfolding() returns Omega
  in the paper's row order.
* Counter for entry e = (low32(e >> 2), high32(e >> 2), mode, tag); the
  generator output word used is e & 3.  tag = 1 for RP-HOSVD sketches,
  tag = 2 for R-STHOSVD sketches.
* Uniform: u = ((x >> 9) + 0.5) * 2**-23 = (2m + 1) * 2**-24 with m < 2**23,
  so every value is exact in binary32 and lies in [2**-24, 1 - 2**-24].
* Box-Muller (Box & Muller, 1958): words (x0, x1) give
  z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1);
  words (x2, x3) give z2, z3 the same way.  Omega(e) = z_{e & 3}.

The oracle evaluates log, sqrt, sin and cos in float64.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

TAG_RP_HOSVD = 1
TAG_R_STHOSVD = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on arrays of counters with one key.

    c0..c3: integer arrays (values < 2**32) of equal shape; k0, k1: ints.
    Each round maps (c0, c1, c2, c3) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
    then the key is bumped by the Weyl constants (Salmon et al., SC'11).
    Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    lo_mask = np.uint64(MASK32)
    for _ in range(10):
        p0 = m0 * c0          # < 2**64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & lo_mask
        hi1, lo1 = p1 >> s32, p1 & lo_mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniform01(x):
    """Map uint32 words to ((x >> 9) + 0.5) * 2**-23, a float64 in (0, 1)
    that binary32 represents exactly."""
    x = np.asarray(x, dtype=np.uint32)
    return ((x >> np.uint32(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def box_muller(ua, ub):
    """Two independent N(0,1) variables from two uniforms (Box-Muller)."""
    r = np.sqrt(-2.0 * np.log(ua))
    t = 2.0 * np.pi * ub
    return r * np.cos(t), r * np.sin(t)


def normals_for_quads(quads, seed, mode, tag):
    """The four normals produced by the counters (quad, mode, tag).

    quads: int array of quad indices (e >> 2).  Returns a (len, 4) float64
    array whose column w is Omega at e = 4*quad + w.
    """
    quads = np.asarray(quads, dtype=np.uint64)
    seed = int(seed)
    x0, x1, x2, x3 = philox4x32_10(quads & np.uint64(MASK32),
                                    quads >> np.uint64(32),
                                    np.full(quads.shape, mode, np.uint64),
                                    np.full(quads.shape, tag, np.uint64),
                                    seed & MASK32, (seed >> 32) & MASK32)
    z0, z1 = box_muller(uniform01(x0), uniform01(x1))
    z2, z3 = box_muller(uniform01(x2), uniform01(x3))
    return np.stack([z0, z1, z2, z3], axis=-1)


def omega_entries(seed, mode, tag, J, j, k):
    """Omega(j, k) for arrays of 0-based row / column indices."""
    e = np.asarray(k, dtype=np.uint64) * np.uint64(J) + np.asarray(j, dtype=np.uint64)
    z = normals_for_quads(e >> np.uint64(2), seed, mode, tag)
    w = (e & np.uint64(3)).astype(np.int64)
    return np.take_along_axis(z, w[..., None], axis=-1)[..., 0]


def omega(seed, mode, tag, J, K):
    """The J x K Gaussian test matrix in generator row order (row c = cyclic
    column position), float64."""
    total = int(J) * int(K)
    if total == 0:
        return np.zeros((J, K))
    nquads = (total + 3) // 4
    z = normals_for_quads(np.arange(nquads, dtype=np.uint64), seed, mode, tag)
    flat = z.reshape(-1)[:total]          # flat[e] = Omega at linear index e
    return flat.reshape(K, J).T           # e = k*J + c


def cyclic_position(j, L, T):
    """Cyclic position c = t + T l of the n-unfolding column j = l + L t."""
    j = np.asarray(j, dtype=np.int64)
    return (j // L) + T * (j % L)


def omega_unfolding(seed, mode, tag, shape, K):
    """Omega for the n-unfolding (mode = n) of a tensor of the given shape,
    rows in the paper's column order: row j = l + L t holds generator row
    c = t + T l."""
    shape = tuple(int(d) for d in shape)
    L = int(np.prod(shape[:mode], dtype=np.int64))
    T = int(np.prod(shape[mode + 1:], dtype=np.int64))
    om = omega(seed, mode, tag, L * T, K)
    # generator rows indexed (t, l) with t fastest -> paper rows (l, t), l fastest
    return om.reshape(T, L, K, order="F").transpose(1, 0, 2).reshape(L * T, K, order="F")
