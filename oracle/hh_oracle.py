"""FP64 CPU oracle for adaptive mixed-precision H_h matrices (Khan & Carson,
"Hybrid hierarchical matrices with adaptive mixed precision storage").

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports or calls this
module: only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg use it. It shares no code with the HIP library (no kernels,
headers, tables or helpers); the only common input is the seeded generator
module ``workloads``.

Everything here is plain NumPy in float64, written for readability rather than
speed, following the paper's steps in its order:

* balanced 2^d-tree ............................ Sec. 2.1
* standard / weak / hybrid admissibility ....... eq:H_admiss, eq:HODLR_admiss,
                                                 eq:hybrid_admiss, Alg. 1
* low-rank compression (truncated SVD) ......... Sec. 2.2, Alg. 1, Def. H_h(p, eps)
* fast Frobenius norms ......................... Alg. 5 (Appendix B)
* adaptive precision choice .................... eq:amp_prec_choice, Alg. 3
* mat-vec with the mixed-precision matrix ..... Alg. 4
* switching-level choice ....................... eq:S1, eq:S2, Alg. 2 (Sec. 3.3)
* q43 and continuum storage (R10, R11) ......... Table tab:precisions, Sec. 4.3
* error bounds ................................. Lemma global_error, Thm amp,
                                                 Thm mvp, eq:standard_IL_size,
                                                 eq:standard_N_size, eq:weak_IL_size

Readings where the paper is silent or ambiguous (each also listed in the design
notes):

R1 tree depth: L is the smallest L >= 0 with leaf_size * 2^(dL) >= N
   (the perfectly-balanced formula of Sec. 2.1); leaves may hold more points.
R2 bounding cube: lower corner = coordinate-wise minimum of the points, side =
   the largest coordinate extent; leaf box k-coordinate =
   min(2^L - 1, floor(((p_k - lo_k) / side) * 2^L)).
R3 tree order: points sorted stably by the Morton key of their leaf box
   (axis 0 is the most significant bit inside each level).
R4 admissibility on tree boxes: diam = sqrt(d) h, dist = h sqrt(S) with
   S = sum_k max(0, |Delta_k| - 1)^2, so adm_s <=> d <= eta^2 S; exact ties count
   as admissible through a relative slack of 2^-40 (this is what reproduces the
   FMM list sizes 27/8 and 189/26 the paper states for eta = sqrt(d)).
R5 weak interaction list = the 2^d - 1 siblings (|IL_w| = 2^d - 1).
R6 compression: the truncated SVD of Sec. 2.2 (LAPACK SVD of the whole block)
   whenever min(m, n) <= 512. Larger blocks (the 2048^2 and 16384^2 blocks of
   the 3D benchmark, where a full SVD of every block is out of reach) use a
   randomized range finder instead: Rademacher sketch from SplitMix64, one
   power iteration, sketch width 64 doubling until rank + 16 <= width, and the
   truncation error ||H - QB||_F^2 summed directly, so the per-block bound
   ||H_b - H~_b|| <= eps ||H_b|| of Def. H_h(p, eps) stays certified. The
   paper fixes none of these randomized parameters (it uses the exact SVD);
   the tests pin the randomized path against the exact truncation on blocks of
   the benchmark's shapes. Rank k = smallest k whose discarded tail
   <= eps^2 ||H_b||_F^2 (the tail summed from the smallest singular value up).
R7 xi uses truncated norms (Alg. 5); the precision rule is evaluated squared:
   u^2 2^(dl) ||H~_b||^2 <= eps^2 ||H~||^2, ties pass; unit roundoffs are exact
   powers of two (2^-53, 2^-24, 2^-11, 2^-8).
R8 rounding: round-to-nearest-even straight from float64 to the storage format;
   each fp16 factor is first scaled by 2^-e with e = floor(log2 max|F|) - 14, each
   bf16 factor by 2^-e with e = floor(log2 max|F|); fp32 / fp64 are unscaled.
R9 singular kernels have H_ii = 0 and entries of coincident distinct points 0.
R10 q43 (8 bits: sign, 4 exponent bits, 3 fraction bits, normal exponents
   -6..7, largest value 240) has unit roundoff 2^-4, the value its 3 fraction
   bits give (the table's printed 2.5e-1 does not match them); rounding is
   ties-to-even with gradual underflow (spacing 2^-9 below 2^-6), and each q43
   factor is scaled by 2^-e with e = floor(log2 max|F|) - 6, so its largest
   entry lands in [64, 128) and nothing overflows.
R11 continuum storage (the accessor remark of Sec. 4.3, which names no format):
   each entry keeps its own 8-bit exponent (normal exponents -126..127, gradual
   underflow) and t fraction bits, ties to even, so u = 2^-(t+1) and an entry
   takes 9 + t bits; t = 7 is bf16 and t = 23 is fp32. A block takes the
   smallest t in [7, 23] whose u passes eq:amp_prec_choice (ties pass), else
   fp64. Rounding stays elementwise relative, so eq:need_mvp and Thm amp hold
   with the block's u as for the fixed formats. The t may also be restricted to
   a list (cont_ts), e.g. the byte-aligned widths t = 7, 15, 23 (16-, 24- and
   32-bit entries), with the same rule over that list.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from workloads import (LOG, INV_R, INV_R2, GAUSS, MATERN, DOUBLE_LAYER,
                       FMT_FP64, FMT_FP32, FMT_FP16, FMT_BF16, FMT_Q43)

# Unit roundoffs of the storage formats (Table tab:precisions, exact powers of two).
UNIT = {FMT_FP64: 2.0 ** -53, FMT_FP32: 2.0 ** -24, FMT_FP16: 2.0 ** -11,
        FMT_BF16: 2.0 ** -8, FMT_Q43: 2.0 ** -4}
BITS = {FMT_FP64: 64, FMT_FP32: 32, FMT_FP16: 16, FMT_BF16: 16, FMT_Q43: 8}
# q43 (R10): 4 significant bits, normal exponents -6..7, largest value 240.
Q43_EMIN, Q43_EMAX, Q43_SIG = -6, 7, 4
# Continuum storage (R11): a float with an 8-bit exponent and t fraction bits,
# CONT_TMIN <= t <= CONT_TMAX, chosen per block; 9 + t bits per entry.
FMT_CONT = 5
CONT_TMIN, CONT_TMAX = 7, 23

# Block types.
T_FAR, T_NEAR, T_WEAK, T_DIAG, T_DENSE_NEAR = 0, 1, 2, 3, 4
TYPE_NAMES = {T_FAR: "IL_s", T_NEAR: "N_s", T_WEAK: "IL_w", T_DIAG: "diag",
              T_DENSE_NEAR: "N_s dense"}

EXACT_SVD_MAX = 512      # R6
SKETCH_START = 64
OVERSAMPLE = 16
TIE_SLACK = 2.0 ** -40   # R4

SINGULAR = {LOG, INV_R, INV_R2, DOUBLE_LAYER}


# --------------------------------------------------------------------------
# Kernel matrix entries, eq:kernel_mat: H_ij = f(||x_i - x_j||_2), H_ii = 0 for
# singular f.
# --------------------------------------------------------------------------
@dataclass
class Kernel:
    kind: int
    scale: float = 1.0
    h: float = 1.0
    normals: np.ndarray | None = None     # user order, (N, d); double layer only


def kernel_entries(kern: Kernel, pi: np.ndarray, pj: np.ndarray,
                   gi: np.ndarray, gj: np.ndarray, nj: np.ndarray | None) -> np.ndarray:
    """Dense block of H for target points pi (m, d) and source points pj (n, d).

    gi / gj are the global indices of the points, used to detect the diagonal
    i == j. nj holds the normals of the source points (double layer only)."""
    diff = pi[:, None, :] - pj[None, :, :]
    same = gi[:, None] == gj[None, :]
    return _kernel_values(kern, diff, same, None if nj is None else nj[None, :, :])


def kernel_pairs(kern: Kernel, pi: np.ndarray, pj: np.ndarray,
                 gi: np.ndarray, gj: np.ndarray, nj: np.ndarray | None) -> np.ndarray:
    """Entries H[gi[k], gj[k]] for paired target points pi (K, d) and source
    points pj (K, d); nj holds the paired sources' normals (double layer)."""
    return _kernel_values(kern, pi - pj, gi == gj, nj)


def _kernel_values(kern: Kernel, diff: np.ndarray, same: np.ndarray,
                   nj: np.ndarray | None) -> np.ndarray:
    """Kernel values from the differences p_i - p_j (last axis = coordinates),
    the mask of equal indices and the (broadcastable) source normals."""
    r2 = np.sum(diff * diff, axis=-1)
    r = np.sqrt(r2)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        if kern.kind == LOG:
            v = np.log(r)
        elif kern.kind == INV_R:
            v = 1.0 / r
        elif kern.kind == INV_R2:
            v = 1.0 / r2
        elif kern.kind == GAUSS:
            v = np.exp(-r2 / (kern.h * kern.h))
        elif kern.kind == MATERN:
            v = np.exp(-r / kern.h)
        elif kern.kind == DOUBLE_LAYER:
            num = np.sum(nj * diff, axis=-1)
            v = num / (r2 * r)
        else:
            raise ValueError(f"unknown kernel {kern.kind}")
    v = kern.scale * v
    if kern.kind in SINGULAR:
        v[(r == 0.0) | same] = 0.0
    return v


def dense_matrix(points: np.ndarray, kern: Kernel) -> np.ndarray:
    """The full N x N kernel matrix in user order (small N only)."""
    n = points.shape[0]
    g = np.arange(n)
    return kernel_entries(kern, points, points, g, g, kern.normals)


def dense_matvec(points: np.ndarray, kern: Kernel, x: np.ndarray,
                 rows: np.ndarray | None = None, chunk: int = 512) -> np.ndarray:
    """y = H x (user order) with H never stored whole; optionally only `rows`."""
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    x2 = x.reshape(n, -1)
    g = np.arange(n)
    out = np.zeros((rows.size, x2.shape[1]))
    for a in range(0, rows.size, chunk):
        ri = rows[a:a + chunk]
        blk = kernel_entries(kern, points[ri], points, ri, g, kern.normals)
        out[a:a + chunk] = blk @ x2
    return out.reshape((rows.size,) + x.shape[1:])


def dense_matvec_t(points: np.ndarray, kern: Kernel, x: np.ndarray,
                   cols: np.ndarray | None = None, chunk: int = 512) -> np.ndarray:
    """y = H^T x (user order), optionally only entries `cols` of y."""
    n = points.shape[0]
    cols = np.arange(n) if cols is None else np.asarray(cols)
    x2 = x.reshape(n, -1)
    g = np.arange(n)
    out = np.zeros((cols.size, x2.shape[1]))
    for a in range(0, cols.size, chunk):
        cj = cols[a:a + chunk]
        nj = kern.normals[cj] if kern.normals is not None else None
        blk = kernel_entries(kern, points, points[cj], g, cj, nj)   # (N, c)
        out[a:a + chunk] = blk.T @ x2
    return out.reshape((cols.size,) + x.shape[1:])


# --------------------------------------------------------------------------
# Balanced 2^d-tree, Sec. 2.1 (readings R1-R3).
# --------------------------------------------------------------------------
def tree_depth(n: int, d: int, leaf_size: int) -> int:
    """Smallest L >= 0 with leaf_size * 2^(dL) >= n (R1)."""
    L = 0
    while leaf_size * (1 << (d * L)) < n:
        L += 1
    return L


def leaf_boxes(points: np.ndarray, L: int) -> np.ndarray:
    """Integer leaf-box coordinates of every point (R2)."""
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    side = float(np.max(hi - lo))
    if side == 0.0:
        side = 1.0
    c = np.floor(((points - lo) / side) * float(1 << L)).astype(np.int64)
    return np.minimum(c, (1 << L) - 1)


def morton(c: np.ndarray, L: int) -> np.ndarray:
    """Morton key of integer box coordinates c (n, d) on a 2^L grid (R3)."""
    n, d = c.shape
    key = np.zeros(n, dtype=np.int64)
    for b in range(L - 1, -1, -1):
        for k in range(d):
            key = key * 2 + ((c[:, k] >> b) & 1)
    return key


def box_coords(box: int, level: int, d: int) -> tuple:
    """Integer coordinates of box `box` (a Morton index) at `level`."""
    c = [0] * d
    for b in range(level):
        digit = (box >> (d * (level - 1 - b))) & ((1 << d) - 1)
        for k in range(d):
            bit = (digit >> (d - 1 - k)) & 1
            c[k] = c[k] * 2 + bit
    return tuple(c)


@dataclass
class Tree:
    n: int
    d: int
    L: int
    perm: np.ndarray            # tree position -> user index
    keys: np.ndarray            # sorted Morton keys (tree order)
    ranges: list                # ranges[l] : (2^(dl), 2) int64 [beg, end) per box

    def cluster(self, level: int, box: int) -> tuple:
        b, e = self.ranges[level][box]
        return int(b), int(e)


def build_tree(points: np.ndarray, leaf_size: int) -> Tree:
    n, d = points.shape
    L = tree_depth(n, d, leaf_size)
    c = leaf_boxes(points, L)
    keys = morton(c, L)
    perm = np.argsort(keys, kind="stable")
    skeys = keys[perm]
    ranges = []
    for level in range(L + 1):
        nb = 1 << (d * level)
        boxid = skeys >> (d * (L - level))
        beg = np.searchsorted(boxid, np.arange(nb), side="left")
        end = np.searchsorted(boxid, np.arange(nb), side="right")
        ranges.append(np.stack([beg, end], axis=1).astype(np.int64))
    return Tree(n, d, L, perm, skeys, ranges)


# --------------------------------------------------------------------------
# Admissibility and block partition: eq:H_admiss, eq:HODLR_admiss,
# eq:hybrid_admiss and Alg. 1 (readings R4, R5).
# --------------------------------------------------------------------------
def gap_S(ci: tuple, cj: tuple) -> int:
    return sum(max(0, abs(a - b) - 1) ** 2 for a, b in zip(ci, cj))


def adm_s(ci: tuple, cj: tuple, d: int, eta: float) -> bool:
    """Standard admissibility of two same-level tree boxes (R4)."""
    S = gap_S(ci, cj)
    return float(d) <= ((eta * eta) * float(S)) * (1.0 + TIE_SLACK)


@dataclass
class Block:
    level: int
    i: int                  # row box (Morton index at `level`)
    j: int                  # column box
    kind: int               # T_FAR / T_NEAR / T_WEAK / T_DIAG / T_DENSE_NEAR
    ib: int
    ie: int
    jb: int
    je: int

    @property
    def m(self) -> int:
        return self.ie - self.ib

    @property
    def n(self) -> int:
        return self.je - self.jb


def resolve_switch_level(switch_level: int, L: int) -> int:
    """switch_level = -1 selects the paper's default L - 1 (Sec. 3.3)."""
    if switch_level == -1:
        return max(L - 1, 0)
    return switch_level


def partition(tree: Tree, eta: float, switch_level: int) -> list:
    """All blocks of the H_h partition in canonical order (level, i, j).

    Levels 1..ell: IL_s (admissible, parents inadmissible). Level ell < L: the
    inadmissible non-self pairs N_s, compressed. ell == L: N_s kept dense.
    Levels ell+1..L: weak admissibility on siblings. Leaf diagonal dense.
    Blocks with an empty row or column cluster are dropped."""
    d, L = tree.d, tree.L
    ell = resolve_switch_level(switch_level, L)
    if not 0 <= ell <= L:
        raise ValueError("switch level outside [0, L]")
    blocks = []

    def nonempty(level):
        r = tree.ranges[level]
        return [b for b in range(r.shape[0]) if r[b, 1] > r[b, 0]]

    for level in range(1, L + 1):
        boxes = nonempty(level)
        if level <= ell:
            # standard admissibility: every pair whose parent pair is still
            # inadmissible (at level 1 the parent pair is the root with itself)
            coords = {b: box_coords(b, level, d) for b in boxes}
            pcoords = {b: box_coords(b >> d, level - 1, d) for b in boxes}
            for i in boxes:
                for j in boxes:
                    if level >= 2 and adm_s(pcoords[i], pcoords[j], d, eta):
                        continue
                    if adm_s(coords[i], coords[j], d, eta):
                        kind = T_FAR
                    elif level == ell and i != j:
                        kind = T_NEAR if ell < L else T_DENSE_NEAR
                    else:
                        continue
                    ib, ie = tree.cluster(level, i)
                    jb, je = tree.cluster(level, j)
                    blocks.append(Block(level, i, j, kind, ib, ie, jb, je))
        else:
            # weak admissibility below the switching level: the open pairs are
            # the children of a diagonal pair, i.e. siblings
            present = set(boxes)
            for i in boxes:
                first = (i >> d) << d
                for j in range(first, first + (1 << d)):
                    if j == i or j not in present:
                        continue
                    ib, ie = tree.cluster(level, i)
                    jb, je = tree.cluster(level, j)
                    blocks.append(Block(level, i, j, T_WEAK, ib, ie, jb, je))
    for i in nonempty(L):
        ib, ie = tree.cluster(L, i)
        blocks.append(Block(L, i, i, T_DIAG, ib, ie, ib, ie))
    blocks.sort(key=lambda b: (b.level, b.i, b.j))
    return blocks


# --------------------------------------------------------------------------
# Sparsity constants (eq:standard_IL_size, eq:standard_N_size, eq:weak_IL_size)
# and the global bounds (Thm amp_throrem, eq:err2_bound, Thm mvp).
# --------------------------------------------------------------------------
def constants_formula(d: int, eta: float) -> tuple:
    c1 = (2 ** d - 1) * (1.0 + 2.0 * math.sqrt(d) / eta) ** d
    c2 = (1.0 + 2.0 * math.sqrt(d) / eta) ** d - 1.0
    return c1, c2, float(2 ** d - 1)


def constants_enumerated(d: int, eta: float) -> tuple:
    """Largest |IL_s| and |N_s| of an interior box, by enumerating offsets."""
    R = 2 + int(math.ceil(math.sqrt(d) / eta))
    rng = range(-R, R + 1)
    import itertools
    zero = (0,) * d
    ns = sum(1 for off in itertools.product(rng, repeat=d)
             if off != zero and not adm_s(zero, off, d, eta))
    best = 0
    for pos in itertools.product((0, 1), repeat=d):
        cnt = 0
        for poff in itertools.product(rng, repeat=d):
            if adm_s(zero, poff, d, eta):
                continue
            for ch in itertools.product((0, 1), repeat=d):
                off = tuple(2 * po + c - p for po, c, p in zip(poff, ch, pos))
                if adm_s(zero, off, d, eta):
                    cnt += 1
        best = max(best, cnt)
    return best, ns, 2 ** d - 1


def global_bound(d: int, eta: float, L: int, ell: int, enumerated: bool = True) -> float:
    """Coefficient c with ||H - H^|| <~ c eps ||H|| (Thm amp_throrem; ell = L gives
    eq:err2_bound, ell = 0 drops C'' as the paper states)."""
    c1, c2, c3 = constants_enumerated(d, eta) if enumerated else constants_formula(d, eta)
    if ell == 0:
        c2 = 0.0
    return 2.0 * math.sqrt(ell * c1 + c2 + (L - ell) * c3) + 1.0


# --------------------------------------------------------------------------
# Counter-based sketch: SplitMix64 (Steele, Lea, Flood 2014), the k-th output
# of a stream started at state s is mix(s + k * gamma), arithmetic mod 2^64.
# --------------------------------------------------------------------------
M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 output function; z a Python int or a uint64 NumPy array."""
    if isinstance(z, np.ndarray):
        with np.errstate(over="ignore"):
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            return z ^ (z >> np.uint64(31))
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def rademacher_sketch(seed: int, uid: int, rnd: int, n: int, s: int) -> np.ndarray:
    """n x s matrix of +-1: entry (j, c) is the sign of output j*s + c + 1 of the
    stream keyed by (seed, block uid, sketch round)."""
    a = mix64((seed + GAMMA * (uid + 1)) & M64)
    b = mix64((a + GAMMA * (rnd + 1)) & M64)
    k = np.arange(1, n * s + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = mix64(np.uint64(b) + np.uint64(GAMMA) * k)
    sgn = np.where((z >> np.uint64(63)) == 0, 1.0, -1.0)
    return sgn.reshape(n, s)


# --------------------------------------------------------------------------
# Low-rank compression with target accuracy eps (Sec. 2.2, Alg. 1, R6).
# --------------------------------------------------------------------------
@dataclass
class Compressed:
    U: np.ndarray          # (m, k), orthonormal columns
    V: np.ndarray          # (n, k) = right singular vectors times sigma
    sigma: np.ndarray      # (k,)
    rank: int
    norm2: float           # ||H_b||_F^2 from the entries
    tail_prev: float       # discarded tail at rank - 1 (inf when rank == 0)
    tail: float            # discarded tail at the chosen rank
    thr: float             # eps^2 ||H_b||^2
    sketch: int            # final sketch width (0 = exact SVD)


def _tails(sig: np.ndarray, extra: float) -> np.ndarray:
    """t[k] = extra + sum_{r >= k} sig_r^2, summed from the smallest term up."""
    p = sig.size
    t = np.empty(p + 1)
    acc = 0.0
    t[p] = extra
    for r in range(p - 1, -1, -1):
        acc += sig[r] * sig[r]
        t[r] = extra + acc
    return t


def _choose_rank(t: np.ndarray, thr: float):
    for k in range(t.size):
        if t[k] <= thr:
            return k
    return None


def _sign_fix(U: np.ndarray, V: np.ndarray) -> None:
    for r in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, r])))
        if U[i, r] < 0:
            U[:, r] *= -1.0
            V[:, r] *= -1.0


def compress(H: np.ndarray, eps: float, seed: int = 0, uid: int = 0) -> Compressed:
    m, n = H.shape
    norm2 = float(np.sum(H * H))
    thr = (eps * eps) * norm2
    p = min(m, n)
    if norm2 == 0.0 or p == 0:
        return Compressed(np.zeros((m, 0)), np.zeros((n, 0)), np.zeros(0), 0, norm2,
                          math.inf, 0.0, thr, 0)
    if p <= EXACT_SVD_MAX:
        Uf, sig, Wt = np.linalg.svd(H, full_matrices=False)
        t = _tails(sig, 0.0)
        k = _choose_rank(t, thr)
        U = Uf[:, :k].copy()
        V = Wt[:k].T * sig[:k]
        _sign_fix(U, V)
        return Compressed(U, V, sig[:k].copy(), k, norm2,
                          t[k - 1] if k > 0 else math.inf, t[k], thr, 0)
    s = min(SKETCH_START, p)
    rnd = 0
    while True:
        Om = rademacher_sketch(seed, uid, rnd, n, s)
        Y = H @ Om
        Q, _ = np.linalg.qr(Y)
        Z = H.T @ Q
        Q2, _ = np.linalg.qr(Z)
        Y = H @ Q2
        Q, _ = np.linalg.qr(Y)
        B = Q.T @ H
        Ub, sig, Wt = np.linalg.svd(B, full_matrices=False)
        E = H - Q @ B
        e2 = float(np.sum(E * E))
        t = _tails(sig, e2)
        k = _choose_rank(t, thr)
        if k is None and s == p:
            k = s
        if k is not None and (k + OVERSAMPLE <= s or s == p):
            U = Q @ Ub[:, :k]
            V = Wt[:k].T * sig[:k]
            _sign_fix(U, V)
            return Compressed(U, V, sig[:k].copy(), k, norm2,
                              t[k - 1] if k > 0 else math.inf, t[k], thr, s)
        s = min(2 * s, p)
        rnd += 1


# --------------------------------------------------------------------------
# Rounding to storage formats (R8).
# --------------------------------------------------------------------------
def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each float64, returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    ax = np.abs(x[nz])
    _, q = np.frexp(ax)                      # ax = f 2^q, f in [0.5, 1)
    e = np.maximum(q - 1, -126)              # exponent of the leading bit
    ulp = np.ldexp(1.0, e - 7)               # 8 significant bits
    r = np.rint(ax / ulp) * ulp              # exact division, half-even rounding
    out[nz] = np.sign(x[nz]) * r
    big = np.float64(np.finfo(np.float32).max)
    out[np.abs(out) > big] = np.sign(out[np.abs(out) > big]) * np.inf
    return out


def round_q43(x: np.ndarray) -> np.ndarray:
    """Nearest q43 value (ties to even) of each float64, returned as float64;
    magnitudes from 248 (halfway between 240 and the next binade) up become inf."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    ax = np.abs(x[nz])
    _, q = np.frexp(ax)                          # ax = f 2^q, f in [0.5, 1)
    e = np.maximum(q - 1, Q43_EMIN)              # exponent of the leading bit
    ulp = np.ldexp(1.0, e - (Q43_SIG - 1))       # 2^-9 below the normal range
    r = np.rint(ax / ulp) * ulp
    out[nz] = np.sign(x[nz]) * r
    top = (2.0 - 2.0 ** -(Q43_SIG - 1)) * 2.0 ** Q43_EMAX
    out[np.abs(out) > top] = np.sign(out[np.abs(out) > top]) * np.inf
    return out


def round_fp(x: np.ndarray, t: int) -> np.ndarray:
    """Nearest value (ties to even) with t fraction bits and exponents >= -126
    (gradual underflow below 2^-126); magnitudes that round beyond
    (2 - 2^-t) 2^127 become inf (R11)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    ax = np.abs(x[nz])
    _, q = np.frexp(ax)
    e = np.maximum(q - 1, -126)
    ulp = np.ldexp(1.0, e - t)
    r = np.rint(ax / ulp) * ulp
    out[nz] = np.sign(x[nz]) * r
    top = (2.0 - 2.0 ** -t) * 2.0 ** 127
    out[np.abs(out) > top] = np.sign(out[np.abs(out) > top]) * np.inf
    return out


def q43_bits(v: np.ndarray) -> np.ndarray:
    """uint8 codes (sign, biased exponent, fraction) of q43 values held exactly
    in float64; exponent field 0 holds the subnormals."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(v.shape, dtype=np.uint8)
    a = np.abs(v)
    sign = (np.signbit(v)).astype(np.uint8) << 7
    _, q = np.frexp(np.where(a > 0, a, 1.0))
    e = q - 1
    normal = a >= 2.0 ** Q43_EMIN
    frac_n = np.rint((np.ldexp(a, -e) - 1.0) * 8.0).astype(np.int64)
    frac_s = np.rint(np.ldexp(a, 9)).astype(np.int64)
    field = np.where(normal, e + 7, 0)
    frac = np.where(normal, frac_n, frac_s)
    out[...] = sign | (field.astype(np.uint8) << 3) | frac.astype(np.uint8)
    return out


def bf16_bits(v: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of bfloat16 values held exactly in float64."""
    return (np.asarray(v, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def scale_exponent(F: np.ndarray, fmt: int) -> int:
    if fmt in (FMT_FP64, FMT_FP32) or F.size == 0:
        return 0
    mx = float(np.max(np.abs(F)))
    if mx == 0.0:
        return 0
    _, q = math.frexp(mx)
    top = q - 1                              # floor(log2 mx)
    if fmt == FMT_FP16:
        return top - 14
    if fmt == FMT_Q43:
        return top - 6
    return top


def round_to(G: np.ndarray, fmt: int) -> np.ndarray:
    """Nearest value of format `fmt` (ties to even), straight from float64."""
    G = np.asarray(G, dtype=np.float64)
    if fmt == FMT_FP64:
        return G.copy()
    if fmt == FMT_FP32:
        with np.errstate(over="ignore"):
            return G.astype(np.float32).astype(np.float64)
    if fmt == FMT_FP16:
        with np.errstate(over="ignore"):
            return G.astype(np.float16).astype(np.float64)
    if fmt == FMT_Q43:
        return round_q43(G)
    return round_bf16(G)


def quantize(F: np.ndarray, fmt: int) -> tuple:
    """(stored values as float64, stored raw array, exponent e); value = stored 2^e."""
    e = scale_exponent(F, fmt)
    G = np.ldexp(F, -e)
    if fmt == FMT_FP64:
        raw = G.copy()
    elif fmt == FMT_FP32:
        raw = G.astype(np.float32)
    elif fmt == FMT_FP16:
        raw = G.astype(np.float16)
    elif fmt == FMT_Q43:
        raw = q43_bits(round_q43(G))
    else:
        raw = bf16_bits(round_bf16(G))
    if fmt == FMT_BF16:
        stored = round_bf16(G)
    elif fmt == FMT_Q43:
        stored = round_q43(G)
    else:
        stored = raw.astype(np.float64)
    return stored, raw, e


# --------------------------------------------------------------------------
# Adaptive precision choice (eq:amp_prec_choice, Alg. 3, R7).
# --------------------------------------------------------------------------
def choose_format(nb2: float, total2: float, level: int, d: int, eps: float,
                  mask: int) -> int:
    """Largest available unit roundoff u with u <= eps / (2^(dl/2) xi_b)."""
    rhs = (eps * eps) * total2
    for fmt in (FMT_Q43, FMT_BF16, FMT_FP16, FMT_FP32):
        if mask & (1 << fmt):
            u = UNIT[fmt]
            if ((u * u) * (2.0 ** (d * level))) * nb2 <= rhs:
                return fmt
    return FMT_FP64


def choose_fraction_bits(nb2: float, total2: float, level: int, d: int, eps: float,
                         tmin: int = CONT_TMIN, tmax: int = CONT_TMAX, ts=None):
    """Continuum rule (R11): the smallest t in [tmin, tmax] (or in the list ts)
    whose unit roundoff 2^-(t+1) passes eq:amp_prec_choice, or None when even
    the largest fails (fp64)."""
    rhs = (eps * eps) * total2
    for t in (range(tmin, tmax + 1) if ts is None else sorted(ts)):
        u = 2.0 ** -(t + 1)
        if ((u * u) * (2.0 ** (d * level))) * nb2 <= rhs:
            return t
    return None


def format_margin(nb2: float, total2: float, level: int, d: int, eps: float, fmt: int) -> float:
    """Ratio lhs / rhs of the precision test for `fmt` (1.0 is an exact tie)."""
    u = UNIT[fmt]
    return ((u * u) * (2.0 ** (d * level))) * nb2 / ((eps * eps) * total2)


def beneficial(rank: int, m: int, n: int, fmt: int, bits: int | None = None) -> bool:
    """Low-rank storage of a leaf neighbour beats dense fp64 (Sec. 4.3 remark);
    `bits` overrides the format's width (continuum storage)."""
    b = BITS[fmt] if bits is None else bits
    return rank * (m + n) * b / 64.0 < m * n


# --------------------------------------------------------------------------
# Construction: Alg. 1 + Alg. 5 + Alg. 3.
# --------------------------------------------------------------------------
@dataclass
class StoredBlock:
    blk: Block
    uid: int
    lowrank: bool
    rank: int = 0
    fmt: int = FMT_FP64
    eU: int = 0
    eV: int = 0
    U: np.ndarray | None = None       # decoded stored factor (m, k) float64
    V: np.ndarray | None = None       # decoded stored factor (n, k) float64
    Ut: np.ndarray | None = None      # fp64 factors before rounding
    Vt: np.ndarray | None = None
    Uraw: np.ndarray | None = None
    Vraw: np.ndarray | None = None
    D: np.ndarray | None = None       # dense block (m, n) float64
    nb2: float = 0.0                  # ||H~_b||^2 (truncated) or ||H_b||^2 (dense)
    comp: Compressed | None = None
    t: int = -1                       # fraction bits when fmt == FMT_CONT


def block_unit(sb: StoredBlock) -> float:
    """Unit roundoff of a stored low-rank block's format."""
    return 2.0 ** -(sb.t + 1) if sb.fmt == FMT_CONT else UNIT[sb.fmt]


def block_bits(sb: StoredBlock) -> int:
    """Bits per stored factor entry of a low-rank block."""
    return 9 + sb.t if sb.fmt == FMT_CONT else BITS[sb.fmt]


@dataclass
class HMatrix:
    points: np.ndarray
    kern: Kernel
    tree: Tree
    eta: float
    ell: int
    eps: float
    mask: int
    uniform: bool
    blocks: list = field(default_factory=list)
    total2: float = 0.0

    @property
    def n(self):
        return self.tree.n

    @property
    def d(self):
        return self.tree.d


def block_entries(hm_points_tree: np.ndarray, kern: Kernel, normals_tree, b: Block) -> np.ndarray:
    gi = np.arange(b.ib, b.ie)
    gj = np.arange(b.jb, b.je)
    nj = normals_tree[b.jb:b.je] if normals_tree is not None else None
    return kernel_entries(kern, hm_points_tree[b.ib:b.ie], hm_points_tree[b.jb:b.je], gi, gj, nj)


def build(points: np.ndarray, kern: Kernel, eps: float, eta: float, switch_level: int,
          leaf_size: int, mask: int = 0xF, uniform: bool = False, seed: int = 0,
          keep_entries: bool = False, continuum: bool = False, cont_ts=None) -> HMatrix:
    tree = build_tree(points, leaf_size)
    ell = resolve_switch_level(switch_level, tree.L)
    blocks = partition(tree, eta, switch_level)
    pt = points[tree.perm]
    nt = kern.normals[tree.perm] if kern.normals is not None else None
    hm = HMatrix(points, kern, tree, eta, ell, eps, mask, uniform)

    # Alg. 1: compress admissible blocks; Alg. 5: accumulate ||H~||^2.
    for uid, b in enumerate(blocks):
        H = block_entries(pt, kern, nt, b)
        if b.kind == T_DIAG or (b.kind == T_DENSE_NEAR and uniform):
            sb = StoredBlock(b, uid, False, D=H, nb2=float(np.sum(H * H)))
        else:
            c = compress(H, eps, seed, uid)
            sb = StoredBlock(b, uid, True, rank=c.rank, Ut=c.U, Vt=c.V, comp=c,
                             nb2=float(np.sum(c.sigma * c.sigma)))
            if b.kind == T_DENSE_NEAR:
                sb.D = H
        hm.blocks.append(sb)
    total2 = 0.0
    for sb in hm.blocks:
        if sb.blk.kind == T_DENSE_NEAR:
            total2 += float(np.sum(sb.D * sb.D))          # Alg. 5, ell == L branch
        else:
            total2 += sb.nb2
    hm.total2 = total2

    # Alg. 3: precision per low-rank block, then round and store.
    for sb in hm.blocks:
        if not sb.lowrank:
            continue
        b = sb.blk
        t = -1
        if uniform:
            fmt = FMT_FP64
        elif continuum:
            tc = choose_fraction_bits(sb.nb2, total2, b.level, tree.d, eps, ts=cont_ts)
            fmt, t = (FMT_FP64, -1) if tc is None else (FMT_CONT, tc)
        else:
            fmt = choose_format(sb.nb2, total2, b.level, tree.d, eps, mask)
        bits = 9 + t if fmt == FMT_CONT else None
        if b.kind == T_DENSE_NEAR and not beneficial(sb.rank, b.m, b.n, fmt, bits):
            sb.lowrank = False
            sb.nb2 = float(np.sum(sb.D * sb.D))
            sb.Ut = sb.Vt = None
            continue
        sb.fmt = fmt
        sb.t = t
        if fmt == FMT_CONT:
            sb.U, sb.Uraw, sb.eU = round_fp(sb.Ut, t), None, 0
            sb.V, sb.Vraw, sb.eV = round_fp(sb.Vt, t), None, 0
            if b.kind == T_DENSE_NEAR:
                sb.D = None
            continue
        sb.U, sb.Uraw, sb.eU = quantize(sb.Ut, fmt)
        sb.V, sb.Vraw, sb.eV = quantize(sb.Vt, fmt)
        sb.U = np.ldexp(sb.U, sb.eU)
        sb.V = np.ldexp(sb.V, sb.eV)
        if b.kind == T_DENSE_NEAR:
            sb.D = None
    return hm


# --------------------------------------------------------------------------
# Mat-vec (Alg. 4) and its transpose, fp64 arithmetic on the stored factors.
# --------------------------------------------------------------------------
def matvec(hm: HMatrix, x: np.ndarray) -> np.ndarray:
    """b = H^ x in user order; x of shape (N,) or (N, nrhs)."""
    perm = hm.tree.perm
    x2 = np.asarray(x, dtype=np.float64).reshape(hm.n, -1)
    xt = x2[perm]
    yt = np.zeros_like(xt)
    for sb in hm.blocks:
        b = sb.blk
        if sb.lowrank:
            if sb.rank:
                yt[b.ib:b.ie] += sb.U @ (sb.V.T @ xt[b.jb:b.je])
        else:
            yt[b.ib:b.ie] += sb.D @ xt[b.jb:b.je]
    y = np.empty_like(yt)
    y[perm] = yt
    return y.reshape(x.shape)


def matvec_t(hm: HMatrix, x: np.ndarray) -> np.ndarray:
    """b = H^^T x in user order."""
    perm = hm.tree.perm
    x2 = np.asarray(x, dtype=np.float64).reshape(hm.n, -1)
    xt = x2[perm]
    yt = np.zeros_like(xt)
    for sb in hm.blocks:
        b = sb.blk
        if sb.lowrank:
            if sb.rank:
                yt[b.jb:b.je] += sb.V @ (sb.U.T @ xt[b.ib:b.ie])
        else:
            yt[b.jb:b.je] += sb.D.T @ xt[b.ib:b.ie]
    y = np.empty_like(yt)
    y[perm] = yt
    return y.reshape(x.shape)


def assemble(hm: HMatrix, which: str = "stored") -> np.ndarray:
    """Dense N x N matrix (user order) from the blocks: 'stored' = H^ (rounded
    factors), 'truncated' = H~ (fp64 factors). Also returns the coverage count."""
    n = hm.n
    A = np.zeros((n, n))
    cover = np.zeros((n, n), dtype=np.int32)
    perm = hm.tree.perm
    for sb in hm.blocks:
        b = sb.blk
        ri = perm[b.ib:b.ie]
        cj = perm[b.jb:b.je]
        if sb.lowrank:
            if which == "stored":
                blk = sb.U @ sb.V.T
            else:
                blk = sb.Ut @ sb.Vt.T
        else:
            blk = sb.D
        A[np.ix_(ri, cj)] += blk
        cover[np.ix_(ri, cj)] += 1
    return A, cover


# --------------------------------------------------------------------------
# Storage accounting (eq:LR_storage, Sec. 5.2).
# --------------------------------------------------------------------------
def storage(hm: HMatrix) -> dict:
    """Words of 64 bits: low-rank p(|I|+|J|) b/64 plus dense m n."""
    lr = 0.0
    dense = 0.0
    by_fmt = {f: 0 for f in list(UNIT) + [FMT_CONT]}
    for sb in hm.blocks:
        b = sb.blk
        if sb.lowrank:
            lr += sb.rank * (b.m + b.n) * block_bits(sb) / 64.0
            by_fmt[sb.fmt] += 1
        else:
            dense += b.m * b.n
    return {"lowrank": lr, "dense": dense, "total": lr + dense, "blocks_by_format": by_fmt}


def structure_arrays(hm: HMatrix) -> dict:
    """Flat arrays describing the structure, in canonical block order."""
    bl = hm.blocks
    return {
        "L": hm.tree.L, "ell": hm.ell, "perm": hm.tree.perm.astype(np.int64),
        "level": np.array([s.blk.level for s in bl], dtype=np.int32),
        "i": np.array([s.blk.i for s in bl], dtype=np.int64),
        "j": np.array([s.blk.j for s in bl], dtype=np.int64),
        "kind": np.array([s.blk.kind if (s.lowrank or s.blk.kind == T_DIAG) else
                          T_DENSE_NEAR for s in bl], dtype=np.int32),
        "lowrank": np.array([s.lowrank for s in bl], dtype=bool),
        "rank": np.array([s.rank if s.lowrank else 0 for s in bl], dtype=np.int32),
        "fmt": np.array([s.fmt if s.lowrank else FMT_FP64 for s in bl], dtype=np.int32),
        "eU": np.array([s.eU for s in bl], dtype=np.int32),
        "eV": np.array([s.eV for s in bl], dtype=np.int32),
    }


# --------------------------------------------------------------------------
# Choice of the switching level (Sec. 3.3: eq:S1, eq:S2, Alg. 2).
#
# H_s and H_h(ell) share the coarse interaction lists of levels 1..ell and the
# dense leaf diagonal; they differ in S1(ell) (what H_s stores below ell: its
# interaction lists of levels ell+1..L and its leaf neighbours N_s(L)) and
# S2(ell) (what H_h stores instead: the compressed neighbours N_s(ell) and the
# weak sibling lists of levels ell+1..L). Storage is counted in 64-bit words
# weighted by each block's storage bits, so the same sums serve the uniform
# scheme (every block fp64) and the mixed one.
# --------------------------------------------------------------------------
def block_words(sb: StoredBlock) -> float:
    """64-bit words of one stored block: k (m + n) bits / 64 low rank, m n dense."""
    b = sb.blk
    if sb.lowrank:
        return sb.rank * (b.m + b.n) * block_bits(sb) / 64.0
    return float(b.m * b.n)


def s1_by_level(hs: HMatrix) -> np.ndarray:
    """S1(ell) for ell = 0..L (eq:S1), read from the H_s representation
    (switching level L): interaction lists of levels ell+1..L plus the leaf
    neighbours, stored densely or, in the mixed scheme, as low rank where
    that is cheaper."""
    L = hs.tree.L
    if hs.ell != L:
        raise ValueError("S1 is read from the H_s representation (switching level L)")
    far = np.zeros(L + 2)
    near_leaf = 0.0
    for sb in hs.blocks:
        if sb.blk.kind == T_FAR:
            far[sb.blk.level] += block_words(sb)
        elif sb.blk.kind == T_DENSE_NEAR:
            near_leaf += block_words(sb)
    # S1(ell) = sum over levels l > ell of far[l], plus the leaf neighbours
    return np.array([far[ell + 1:].sum() + near_leaf for ell in range(L + 1)])


def s2_of(hh: HMatrix) -> float:
    """S2(ell) (eq:S2) of an H_h representation with switching level ell < L:
    its compressed neighbours N_s(ell) plus its sibling lists IL_w of levels
    ell+1..L."""
    if hh.ell >= hh.tree.L:
        raise ValueError("S2 is defined here for ell < L; S2(L) = S1(L)")
    return float(sum(block_words(sb) for sb in hh.blocks if sb.blk.kind in (T_NEAR, T_WEAK)))


def switch_level_search(L: int, s1: np.ndarray, s2_fn) -> tuple:
    """Alg. 2: start at ell = L with gain S1(L) - S2(L) = 0 and lower ell while
    the gain S1(ell - 1) - S2(ell - 1) strictly grows; S2 is asked for only at
    the levels the walk reaches. Returns (ell*, {ell: gain})."""
    ell, s = L, 0.0
    gains = {L: 0.0}
    while ell > 0:
        s_new = float(s1[ell - 1]) - float(s2_fn(ell - 1))
        gains[ell - 1] = s_new
        if s_new <= s:
            break
        s, ell = s_new, ell - 1
    return ell, gains


def optimal_switch_level(points: np.ndarray, kern: Kernel, eps: float, eta: float,
                         leaf_size: int, mask: int = 0xF, uniform: bool = False,
                         seed: int = 0) -> dict:
    """Build H_s, read S1 for every level, then walk Alg. 2 building H_h(ell)
    for each level it reaches."""
    hs = build(points, kern, eps, eta, build_tree(points, leaf_size).L, leaf_size,
               mask=mask, uniform=uniform, seed=seed)
    L = hs.tree.L
    s1 = s1_by_level(hs)
    s2 = {L: float(s1[L])}

    def s2_fn(ell):
        hh = build(points, kern, eps, eta, ell, leaf_size, mask=mask, uniform=uniform, seed=seed)
        s2[ell] = s2_of(hh)
        return s2[ell]

    ell, gains = switch_level_search(L, s1, s2_fn)
    return {"ell": ell, "L": L, "s1": s1, "s2": s2, "gains": gains,
            "storage_hs": storage(hs)["total"]}


# --------------------------------------------------------------------------
# Iterative solution with the H_h matrix (the closing remark of Sec. 5.3: the
# fast mixed-precision product serves iterative solvers). Restarted GMRES
# (Saad & Schultz, 1986) for (H^ + shift I) x = b, the Krylov basis made
# orthonormal by classical Gram-Schmidt applied twice, the small least-squares
# problem kept triangular with Givens rotations.
# --------------------------------------------------------------------------
def gmres(apply, b: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-10,
          restart: int = 30, max_iter: int = 300) -> tuple:
    """Returns (x, iterations, relative residual history) for the operator
    `apply` (a function v -> A v). The residual history holds the recurrence's
    residual norms divided by ||b||, one per iteration, after the initial one;
    the method stops when that ratio is <= rtol or after max_iter iterations."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return np.zeros(n), 0, [0.0]
    hist = []
    it = 0
    while True:
        r = b - apply(x)
        beta = float(np.linalg.norm(r))
        hist.append(beta / nb)
        if beta / nb <= rtol or it >= max_iter:
            return x, it, hist
        m = min(restart, max_iter - it)
        V = np.zeros((n, m + 1))
        Hs = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            w = apply(V[:, j])
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            Hs[:j + 1, j] = h
            Hs[j + 1, j] = hn
            if hn > 0.0:
                V[:, j + 1] = w / hn
            for i in range(j):                      # earlier rotations
                a, c = Hs[i, j], Hs[i + 1, j]
                Hs[i, j] = cs[i] * a + sn[i] * c
                Hs[i + 1, j] = -sn[i] * a + cs[i] * c
            a, c = Hs[j, j], Hs[j + 1, j]
            d = math.hypot(a, c)
            cs[j], sn[j] = (1.0, 0.0) if d == 0.0 else (a / d, c / d)
            Hs[j, j] = d
            Hs[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            res = abs(g[j + 1]) / nb
            if res <= rtol or hn == 0.0:
                break
            if j + 1 < m:
                hist.append(res)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):              # back substitution
            y[i] = (g[i] - Hs[i, i + 1:k] @ y[i + 1:]) / Hs[i, i]
        x = x + V[:, :k] @ y
