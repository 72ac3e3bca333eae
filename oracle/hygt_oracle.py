"""FP64 CPU oracle for the Hypercube-Givens transform (HyGT).

TEST INFRASTRUCTURE ONLY. This module is the plain, slow, obviously correct
statement of what the GPU library computes. It exists so that the tests, the
smoke check and the benchmark's CPU-baseline leg can compare the HIP path
against it. The product path never imports it, and it imports nothing from the
product: the two share no kernels, helpers, tables or constants.

Source: Said, Zhao, Karczewicz, Egilmez, Seregin, Chen, "Highly Efficient
Non-Separable Transforms for Next Generation Video Coding" (arXiv 2505.21728).

Conventions fixed here (the paper's figures are not available; each reading is
listed with its justification in the design notes):

* A block is a vector of N = 2**d residuals (Sec. II, signal-adaptive model).
* The Givens rotation G(m, n, theta) is the identity except
  G[m,m] = G[n,n] = cos(theta), G[m,n] = +sin(theta), G[n,m] = -sin(theta)
  (Sec. IV, element definition). Applied as y = G x this is
  y_m = cos*x_m + sin*x_n,  y_n = -sin*x_m + cos*x_n.
* Pass k of a round pairs every index with its neighbour along hypercube
  dimension k, i.e. (i, i XOR 2**k) (Sec. IV, Fig. 3 caption and Fig. 5).
  Angle j of pass k belongs to pair number j in the enumeration of Fig. 5:
  m = j with a zero bit inserted at position k, n = m + 2**k.
* A round applies passes k = 0, 1, ..., d-1; the transform applies rounds
  0..R-1; the first pass applied is F_1 of eq. (5).
* Angle table layout: angles[class, round, pass, j], radians.
* The inverse applies the passes in reverse order with negated angles
  (eq. (6), eq. (9), Sec. IV).
* Class indices are 0-based.

* Variants: 8-bit angle codes (Fig. 6) map code q to (q - 128) pi / 128, and
  the integer transform uses 14-bit fixed-point multipliers with outputs
  rounded by an arithmetic shift. The paper gives neither the map nor the
  word length and rounding, so those choices are parity unpinned; the
  arithmetic built on them is pinned.

Every function states the passage it follows. Parity pins for each function
live in tests/test_oracle.py.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "pair_indices",
    "forward",
    "inverse",
    "givens_matrix",
    "parallel_givens_matrix",
    "transform_matrix_from_passes",
    "transform_matrix_from_columns",
    "num_parameters",
    "klt_parameters",
    "memory_usage_ratio",
    "round_to_bf16",
    "dense_transform",
    "rel_l2_per_block",
    "rel_l2_global",
    "class_log_variance_loss",
    "class_log_variance_grad",
    "backward",
    "angles_from_codes",
    "codes_from_angles",
    "INT_FRAC_BITS",
    "int_multipliers",
    "forward_int",
    "inverse_int",
    "int_error_bound",
    "forward_permuted",
    "inverse_permuted",
    "variance_order",
]


# ---------------------------------------------------------------------------
# Hypercube index pairs (Sec. IV, Fig. 5)
# ---------------------------------------------------------------------------

def pair_indices(d: int, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Index vectors (m, n) of pass k on a d-dimensional hypercube.

    Sec. IV: the passes of a round take the hypercube edges one dimension at a
    time. For pair number j (0 <= j < N/2) the lower index m is j with a zero
    bit inserted at bit position k, and n = m + 2**k (the same pairs Fig. 5
    enumerates). The pairs cover {0, ..., N-1} exactly once (eq. (7)).
    """
    if not (1 <= d) or not (0 <= k < d):
        raise ValueError("need d >= 1 and 0 <= k < d")
    half = 1 << (d - 1)
    m = np.empty(half, dtype=np.int64)
    n = np.empty(half, dtype=np.int64)
    low_mask = (1 << k) - 1
    for j in range(half):
        high = j >> k          # bits of j at and above position k
        low = j & low_mask     # bits of j below position k
        mj = (high << (k + 1)) | low
        m[j] = mj
        n[j] = mj + (1 << k)
    return m, n


# ---------------------------------------------------------------------------
# Batched transform (eq. (5), (6), (8), (9); Sec. IV)
# ---------------------------------------------------------------------------

def _check(x: np.ndarray, cls: np.ndarray | None, angles: np.ndarray):
    x = np.asarray(x, dtype=np.float64)
    angles = np.asarray(angles, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("x must be [nblocks, N]")
    if angles.ndim != 4:
        raise ValueError("angles must be [C, R, d, N/2]")
    nclasses, rounds, d, half = angles.shape
    n_elems = 1 << d
    if x.shape[1] != n_elems or half != n_elems // 2:
        raise ValueError("shape mismatch between x and angles")
    if cls is None:
        if nclasses != 1:
            raise ValueError("cls may be omitted only when there is one class")
        cls = np.zeros(x.shape[0], dtype=np.int64)
    cls = np.asarray(cls, dtype=np.int64)
    if cls.shape != (x.shape[0],):
        raise ValueError("cls must be [nblocks]")
    if cls.size and (cls.min() < 0 or cls.max() >= nclasses):
        raise ValueError("class index out of range")
    return x, cls, angles, rounds, d


def forward(x, cls, angles) -> np.ndarray:
    """y[b] = T_{cls[b]} x[b] in FP64.

    T_c = F_P ... F_1 (eq. (5)), F for round r and pass k being the
    parallel-Givens matrix G(m, n, theta_{c,r,k}) of eq. (8) with the
    hypercube pairs of pass k. Rounds go 0..R-1, passes 0..d-1 inside each
    round (Sec. IV). Each pair is rotated with the element definition of G:
    y_m = cos*x_m + sin*x_n, y_n = -sin*x_m + cos*x_n.
    """
    x, cls, angles, rounds, d = _check(x, cls, angles)
    v = x.copy()
    for r in range(rounds):
        for k in range(d):
            m, n = pair_indices(d, k)
            theta = angles[cls, r, k, :]          # [B, N/2]
            c = np.cos(theta)
            s = np.sin(theta)
            xm = v[:, m].copy()
            xn = v[:, n].copy()
            v[:, m] = c * xm + s * xn
            v[:, n] = -s * xm + c * xn
    return v


def inverse(y, cls, angles) -> np.ndarray:
    """z[b] = T_{cls[b]}^{-1} y[b] in FP64.

    eq. (6): the inverse is the product of the inverse passes in reverse
    order. eq. (9): the inverse of a parallel-Givens pass is the same pass with
    negated angles. So rounds run R-1..0, passes d-1..0, and each pair gets
    y_m = cos*x_m - sin*x_n, y_n = sin*x_m + cos*x_n.
    """
    y, cls, angles, rounds, d = _check(y, cls, angles)
    v = y.copy()
    for r in reversed(range(rounds)):
        for k in reversed(range(d)):
            m, n = pair_indices(d, k)
            theta = -angles[cls, r, k, :]
            c = np.cos(theta)
            s = np.sin(theta)
            xm = v[:, m].copy()
            xn = v[:, n].copy()
            v[:, m] = c * xm + s * xn
            v[:, n] = -s * xm + c * xn
    return v


# ---------------------------------------------------------------------------
# Dense matrices built from the definitions (for tiny N)
# ---------------------------------------------------------------------------

def givens_matrix(n_elems: int, m: int, n: int, theta: float) -> np.ndarray:
    """G(m, n, theta) written out element by element (Sec. IV definition)."""
    g = np.zeros((n_elems, n_elems), dtype=np.float64)
    for i in range(n_elems):
        for j in range(n_elems):
            if i == j and (i == m or i == n):
                g[i, j] = math.cos(theta)
            elif i == m and j == n:
                g[i, j] = math.sin(theta)
            elif i == n and j == m:
                g[i, j] = -math.sin(theta)
            elif i == j:
                g[i, j] = 1.0
    return g


def parallel_givens_matrix(d: int, k: int, thetas) -> np.ndarray:
    """G(m, n, theta) of eq. (8): the product of the N/2 rotations of pass k."""
    n_elems = 1 << d
    m, n = pair_indices(d, k)
    out = np.eye(n_elems)
    for j in range(n_elems // 2):
        out = out @ givens_matrix(n_elems, int(m[j]), int(n[j]), float(thetas[j]))
    return out


def transform_matrix_from_passes(angles_c) -> np.ndarray:
    """T = F_P ... F_2 F_1 (eq. (5)) as a product of dense pass matrices.

    angles_c is one class's table [R, d, N/2]; F_1 is round 0, pass 0.
    """
    angles_c = np.asarray(angles_c, dtype=np.float64)
    rounds, d, _ = angles_c.shape
    t = np.eye(1 << d)
    for r in range(rounds):
        for k in range(d):
            t = parallel_givens_matrix(d, k, angles_c[r, k]) @ t
    return t


def transform_matrix_from_columns(angles_c) -> np.ndarray:
    """T built column by column: column i is forward(e_i)."""
    angles_c = np.asarray(angles_c, dtype=np.float64)
    n_elems = 1 << angles_c.shape[1]
    eye = np.eye(n_elems)
    cols = forward(eye, np.zeros(n_elems, dtype=np.int64), angles_c[None])
    return cols.T


# ---------------------------------------------------------------------------
# Parameter counts and Table II memory ratios (Sec. IV, Sec. VI)
# ---------------------------------------------------------------------------

def num_parameters(n_elems: int, rounds: int) -> int:
    """Angles in one HyGT: R * N * log2(N) / 2 (Sec. IV)."""
    d = int(round(math.log2(n_elems)))
    if 1 << d != n_elems:
        raise ValueError("N must be a power of two")
    return rounds * n_elems * d // 2


def klt_parameters(n_elems: int) -> int:
    """Entries of one dense N x N KLT matrix (eq. (3))."""
    return n_elems * n_elems


def memory_usage_ratio(scheme_4x4: str, scheme_8x8: str, which: str) -> float:
    """Memory used by KLTs divided by memory used by the scheme (Table II).

    A scheme name is "K" (dense KLT) or "H(R)" (HyGT with R rounds). The same
    number of transforms is stored for each block size (105 per size), so the
    ratios depend only on per-transform parameter counts. `which` selects the
    4x4 set, the 8x8 set or both ("avg", the average row of Table II, taken as
    the ratio of totals over the two sizes).
    """
    def count(name: str, n_elems: int) -> int:
        if name == "K":
            return klt_parameters(n_elems)
        if name.startswith("H(") and name.endswith(")"):
            return num_parameters(n_elems, int(name[2:-1]))
        raise ValueError(name)

    klt4, klt8 = klt_parameters(16), klt_parameters(64)
    s4, s8 = count(scheme_4x4, 16), count(scheme_8x8, 64)
    if which == "4x4":
        return klt4 / s4
    if which == "8x8":
        return klt8 / s8
    if which == "avg":
        return (klt4 + klt8) / (s4 + s8)
    raise ValueError(which)


# ---------------------------------------------------------------------------
# Dense per-class matrix transform, the KLT-shaped comparison (eq. (3))
# ---------------------------------------------------------------------------

def round_to_bf16(a) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of an IEEE binary32. Rounding adds half an ulp of the kept part (plus the
    kept lowest bit for ties-to-even) before truncation. Inputs must be finite.
    """
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = a32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def dense_transform(x, cls, mats) -> np.ndarray:
    """y[b] = K_{cls[b]} x[b] (eq. (3)) in FP64 for dense per-class matrices."""
    x = np.asarray(x, dtype=np.float64)
    mats = np.asarray(mats, dtype=np.float64)
    cls = np.asarray(cls, dtype=np.int64)
    y = np.empty_like(x)
    for b in range(x.shape[0]):
        y[b] = mats[cls[b]] @ x[b]
    return y


# ---------------------------------------------------------------------------
# Angle gradients for the parameter optimisation of Sec. V
# ---------------------------------------------------------------------------

def class_log_variance_loss(y, cls, nclasses: int, eps: float = 1e-6) -> float:
    """sum over classes c and coefficients i of log(var_{c,i} + eps).

    Sec. V rates a transform by the variances of its coefficients, the
    diagonal of T Phi T^T (eq. (10)), under the high-rate model of eq. (11),
    in which the rate of a coefficient grows with the log of its variance.
    Here var_{c,i} is the mean of y_{b,i}^2 over the blocks b of class c (the
    variances with Phi estimated from those blocks). A class with no blocks
    adds nothing.
    """
    y = np.asarray(y, dtype=np.float64)
    cls = np.asarray(cls, dtype=np.int64)
    total = 0.0
    for c in range(nclasses):
        rows = y[cls == c]
        if rows.shape[0] == 0:
            continue
        var = np.mean(rows * rows, axis=0)
        total += float(np.sum(np.log(var + eps)))
    return total


def class_log_variance_grad(y, cls, nclasses: int, eps: float = 1e-6) -> np.ndarray:
    """dL/dy of class_log_variance_loss: 2 y_{b,i} / (n_c (var_{c,i} + eps))."""
    y = np.asarray(y, dtype=np.float64)
    cls = np.asarray(cls, dtype=np.int64)
    g = np.zeros_like(y)
    for c in range(nclasses):
        sel = cls == c
        n_c = int(np.count_nonzero(sel))
        if n_c == 0:
            continue
        var = np.mean(y[sel] * y[sel], axis=0)
        g[sel] = 2.0 * y[sel] / (n_c * (var + eps))
    return g


def backward(y, gy, cls, angles, with_mass=False):
    """Reverse-mode derivative of forward().

    Given the outputs y = forward(x, cls, angles) and gy = dL/dy, returns
    (gx, gangles): gx = dL/dx for every block and gangles = dL/dangles with
    the same layout as angles, summed over the blocks of each class.

    The passes are walked in reverse order (last round first, pass d-1 first
    inside it). Each pass's inputs are recovered from its outputs by the
    inverse rotation (eq. (9)) instead of being stored. For one rotation
    y_m = c x_m + s x_n, y_n = -s x_m + c x_n:
        dy_m/dtheta = y_n and dy_n/dtheta = -y_m, so dL/dtheta = g_m y_n - g_n y_m;
        (dL/dx_m, dL/dx_n) = (c g_m - s g_n, s g_m + c g_n), the inverse rotation of g.

    With with_mass, also returns the summed magnitudes of the terms behind
    each angle's gradient, sum over the class's blocks of |g_m y_n| + |g_n y_m|
    (same layout as gangles): the scale against which a floating-point sum
    of those terms has its error bounded.
    """
    y, cls, angles, rounds, d = _check(y, cls, angles)
    g = np.array(gy, dtype=np.float64, copy=True)
    if g.shape != y.shape:
        raise ValueError("gy must have the shape of y")
    v = y.copy()
    gangles = np.zeros_like(angles)
    mass = np.zeros_like(angles)
    for r in reversed(range(rounds)):
        for k in reversed(range(d)):
            m, n = pair_indices(d, k)
            theta = angles[cls, r, k, :]
            c = np.cos(theta)
            s = np.sin(theta)
            contrib = g[:, m] * v[:, n] - g[:, n] * v[:, m]      # [B, N/2]
            np.add.at(gangles[:, r, k, :], cls, contrib)
            if with_mass:
                np.add.at(mass[:, r, k, :], cls,
                          np.abs(g[:, m] * v[:, n]) + np.abs(g[:, n] * v[:, m]))
            ym, yn = v[:, m].copy(), v[:, n].copy()
            v[:, m] = c * ym - s * yn
            v[:, n] = s * ym + c * yn
            gm, gn = g[:, m].copy(), g[:, n].copy()
            g[:, m] = c * gm - s * gn
            g[:, n] = s * gm + c * gn
    if with_mass:
        return g, gangles, mass
    return g, gangles


# ---------------------------------------------------------------------------
# Paper variants: 8-bit parameter codes (Fig. 6) and the permutation pass (Fig. 4)
# ---------------------------------------------------------------------------

def angles_from_codes(codes) -> np.ndarray:
    """Angle of each 8-bit code: (q - 128) * pi / 128.

    Fig. 6 stores one byte per parameter and a shared table of multipliers;
    the paper does not give the code-to-angle map (parity unpinned for the
    map itself). This reading spaces the 256 codes evenly over [-pi, pi),
    with q = 128 the zero angle.
    """
    q = np.asarray(codes, dtype=np.int64)
    return (q - 128).astype(np.float64) * (math.pi / 128.0)


def codes_from_angles(angles) -> np.ndarray:
    """Nearest 8-bit code of each angle (angles taken modulo 2 pi)."""
    a = np.asarray(angles, dtype=np.float64)
    q = np.rint(a * (128.0 / math.pi)).astype(np.int64) + 128
    return np.mod(q, 256).astype(np.uint8)


def forward_permuted(x, cls, angles, perm) -> np.ndarray:
    """forward() followed by the permutation pass of Fig. 4: output position
    i of a block of class c holds transform coefficient perm[c, i]."""
    y = forward(x, cls, angles)
    cls = np.zeros(y.shape[0], dtype=np.int64) if cls is None else np.asarray(cls, np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    out = np.empty_like(y)
    for b in range(y.shape[0]):
        out[b] = y[b, perm[cls[b]]]
    return out


def inverse_permuted(yp, cls, angles, perm) -> np.ndarray:
    """Inverse of forward_permuted(): undo the permutation, then inverse()."""
    yp = np.asarray(yp, dtype=np.float64)
    cls_i = np.zeros(yp.shape[0], dtype=np.int64) if cls is None else np.asarray(cls, np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    y = np.empty_like(yp)
    for b in range(yp.shape[0]):
        y[b, perm[cls_i[b]]] = yp[b]
    return inverse(y, cls, angles)


def variance_order(y, cls, nclasses: int) -> np.ndarray:
    """Per class, the coefficients sorted by decreasing variance (mean of
    y^2 over the class's blocks), ties by index: the sort of Fig. 4's
    optional permutation pass. Classes without blocks keep the identity."""
    y = np.asarray(y, dtype=np.float64)
    cls = np.asarray(cls, dtype=np.int64)
    n = y.shape[1]
    out = np.tile(np.arange(n, dtype=np.int64), (nclasses, 1))
    for c in range(nclasses):
        rows = y[cls == c]
        if rows.shape[0]:
            var = np.mean(rows * rows, axis=0)
            out[c] = np.lexsort((np.arange(n), -var))
    return out


# ---------------------------------------------------------------------------
# Integer arithmetic (Sec. IV, Fig. 6): integer blocks, multipliers from a
# shared table of fixed-point cosines and sines indexed by the 8-bit code
# ---------------------------------------------------------------------------

INT_FRAC_BITS = 14


def int_multipliers(codes) -> tuple[np.ndarray, np.ndarray]:
    """Fixed-point (C, S) = round(2^14 cos, 2^14 sin) of each code's angle.

    Fig. 6 converts each low-bit parameter to higher-precision multipliers
    through a table of sines and cosines shared by all transforms, and the
    text asks for well-defined integer arithmetic without giving the word
    length or the rounding (parity unpinned for those choices). This reading
    takes 14 fractional bits and rounds half to even in FP64.
    """
    th = angles_from_codes(codes)
    scale = float(1 << INT_FRAC_BITS)
    return (np.rint(scale * np.cos(th)).astype(np.int64),
            np.rint(scale * np.sin(th)).astype(np.int64))


def _int_rotate(xm, xn, c, s):
    """One integer butterfly: eq. (7) with fixed-point multipliers, each
    output rounded to the nearest integer (ties upwards) by an arithmetic
    shift. All operands are int64, so nothing overflows."""
    half = 1 << (INT_FRAC_BITS - 1)
    ym = (c * xm + s * xn + half) >> INT_FRAC_BITS
    yn = (c * xn - s * xm + half) >> INT_FRAC_BITS
    return ym, yn


def _check_int(x, cls, codes):
    x = np.asarray(x)
    if not np.issubdtype(x.dtype, np.integer):
        raise TypeError("integer blocks expected")
    codes = np.asarray(codes)
    if codes.dtype != np.uint8 or codes.ndim != 4:
        raise TypeError("codes must be uint8 [C, R, d, N/2]")
    nclasses, rounds, d, half = codes.shape
    if x.ndim != 2 or x.shape[1] != 2 * half or 1 << d != x.shape[1]:
        raise ValueError("blocks do not match the codes")
    cls = np.zeros(x.shape[0], np.int64) if cls is None else np.asarray(cls, np.int64)
    if cls.size and (cls.min() < 0 or cls.max() >= nclasses):
        raise ValueError("class out of range")
    return x.astype(np.int64), cls, codes, rounds, d


def forward_int(x, cls, codes) -> np.ndarray:
    """Integer HyGT: R rounds of d passes in the order of eq. (5), each
    butterfly an integer rotation with the multipliers of its code."""
    y, cls, codes, rounds, d = _check_int(x, cls, codes)
    c_tab, s_tab = int_multipliers(codes)
    for r in range(rounds):
        for k in range(d):
            m, n = pair_indices(d, k)
            c = c_tab[cls, r, k, :]
            s = s_tab[cls, r, k, :]
            y[:, m], y[:, n] = _int_rotate(y[:, m], y[:, n], c, s)
    return y


def inverse_int(y, cls, codes) -> np.ndarray:
    """Integer inverse: the passes in reverse order with negated angles
    (eq. (9)), i.e. multipliers (C, -S). Not an exact inverse of
    forward_int(): each butterfly rounds."""
    x, cls, codes, rounds, d = _check_int(y, cls, codes)
    c_tab, s_tab = int_multipliers(codes)
    for r in reversed(range(rounds)):
        for k in reversed(range(d)):
            m, n = pair_indices(d, k)
            c = c_tab[cls, r, k, :]
            s = s_tab[cls, r, k, :]
            x[:, m], x[:, n] = _int_rotate(x[:, m], x[:, n], c, -s)
    return x


def int_error_bound(x_norm: float, n_elems: int, passes: int) -> float:
    """Bound on ||forward_int(x) - forward(x, angles of the codes)||_2 for a
    block of L2 norm x_norm. Per pass the rounding adds at most sqrt(N)/2
    and the multiplier quantisation (each entry within 2^-15) at most
    sqrt(2) 2^-15 times the current norm; the exact passes are orthogonal
    and so carry the earlier error unchanged."""
    delta = math.sqrt(2.0) * 2.0 ** -(INT_FRAC_BITS + 1)
    e = 0.0
    for _ in range(passes):
        e += delta * (x_norm + e) + 0.5 * math.sqrt(n_elems)
    return e


# ---------------------------------------------------------------------------
# Comparison metric
# ---------------------------------------------------------------------------

def rel_l2_per_block(approx, exact) -> np.ndarray:
    """||approx_b - exact_b||_2 / ||exact_b||_2 per block.

    A block whose exact value is all zeros reports its absolute error norm
    (which must be exactly zero for a pass).
    """
    approx = np.asarray(approx, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    num = np.sqrt(np.sum((approx - exact) ** 2, axis=1))
    den = np.sqrt(np.sum(exact ** 2, axis=1))
    out = num.copy()
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def rel_l2_global(approx, exact) -> float:
    """||approx - exact||_2 / ||exact||_2 over all blocks concatenated."""
    approx = np.asarray(approx, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    den = float(np.sqrt(np.sum(exact ** 2)))
    num = float(np.sqrt(np.sum((approx - exact) ** 2)))
    return num / den if den > 0 else num
