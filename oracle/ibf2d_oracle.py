"""Plain FP64 CPU oracle for the 2-D tensor IBF and the multiscale IBF (MIBF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this module; only the tests, the smoke check and the CPU-baseline
leg of the benchmark may.  It shares no code with the HIP implementation.

Passages followed:

* Sec. 5 (high dimensional extension): the multidimensional IBF on
  quadtrees with tensor Chebyshev grids, and the MIBF -- the corona
  decomposition of Omega (eq:domaindecomp), the multiscale sum (eq:mba) and
  its factorized form (eq:f1): one IBF per subdomain, the centre summed
  directly.
* Sec. 6.3: the 2-D FIO Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2).
* Secs. 3 and 4 for the blocks and the sweep-out compression, exactly as in
  the 1-D oracle with four children per box instead of two.

Readings (also in the design notes): child c of a box is (c1, c2) with
c = 2 c1 + c2 (c1 = upper half in the first coordinate); boxes are indexed
by Morton codes, so the children of code b are 4b + c and its parent b >> 2;
the tensor grid index is t = t1 r + t2; every coronal subdomain is the union
of the 12 dyadic boxes of side n / 2^(t+2) between the squares of half-width
n / 2^(t+1) and n / 2^(t+2) (half-open), and the centre is the square of
side `centre` (16, Sec. 6.3) at the origin; each box runs its own IBF.  In
a box of side w the pair (T_X box at level l, T_Omega box at level L - l),
L = log2 w, has width product 1 per coordinate; V pairs the Omega leaves
(side `leaf_side`, level L - lV) with the T_X boxes at level lV =
log2(leaf_side), U pairs the T_X boxes at level L with the box itself, and
the middle level is h = floor((lV + L) / 2).

Randomized low-rank approximation (Sec. 2.1, f2): the paper computes large
low-rank approximations by sampling the matrix randomly and defers the
algorithm to its references.  `sweep_out_2d(..., sample=(seed, S))` takes
the column-sampling reading: every block W (the middle M~, the W of eqn:GC,
the Z of eqn:HR) keeps each of its n real columns with probability
min(1, S / n), independently, by a counter-based draw (the (i + 1)-th
output of SplitMix64 started at `seed`, Steele, Lea and Flood 2014, for the
column's index i); the left singular vectors U and singular values of the
s kept columns, scaled by sqrt(n / s), stand for W's; the rank is the
tolerance rule on them, and the right factor is the projection of all of W,
V_k S_k = W^* U_k (linear in n).  With S >= n every column is kept and the
compression is the direct one.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .ibf_oracle import (TWO_PI, _keep, cheb_nodes, child_to_parent, lagrange,
                         rel_error, truncated_svd, two_product)

PHASE_DFT, PHASE_FIO2D, PHASE_SEPARABLE = 0, 2, 3


# ----------------------------------------------------------------------------
# 2-D phases with exact mod-1 reduction, dense product
# ----------------------------------------------------------------------------

def _frac_prod(a, b):
    p, e = two_product(a, b)
    t = (p - np.rint(p)) + e
    return t - np.rint(t)


def phase_frac_2d(kind, params, x, xi):
    """Phi(x, xi) mod 1 in [-1/2, 1/2] for x, xi of shape (..., 2) (broadcasting).

    kind 0: Phi = s (x1 xi1 + x2 xi2)
    kind 2: Phi = x.xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
            c1 = (p0 + p1 sin 2 pi x1 sin 2 pi x2) / p2,
            c2 = (p0 + p1 cos 2 pi x1 cos 2 pi x2) / p2          (Sec. 6.3)
    kind 3: Phi = p0 xi1 + p1 xi2 (independent of x: the IBF is exact)
    """
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    x1, x2 = x[..., 0], x[..., 1]
    k1, k2 = xi[..., 0], xi[..., 1]
    if kind == 0:
        s = params[0] if params else 1.0
        t = s * (_frac_prod(x1, k1) + _frac_prod(x2, k2))
    elif kind == 2:
        p0, p1, p2 = params
        s1, s2 = np.sin(TWO_PI * x1), np.sin(TWO_PI * x2)
        q1, q2 = np.cos(TWO_PI * x1), np.cos(TWO_PI * x2)
        c1 = (p0 + p1 * s1 * s2) / p2
        c2 = (p0 + p1 * q1 * q2) / p2
        root = np.sqrt((c1 * k1) ** 2 + (c2 * k2) ** 2)
        t = _frac_prod(x1, k1) + _frac_prod(x2, k2) + (root - np.rint(root))
    elif kind == 3:
        p0, p1 = params
        k1, k2 = np.broadcast_arrays(k1, k2 + 0.0 * x1)
        t = _frac_prod(np.full_like(k1, p0), k1) + _frac_prod(np.full_like(k2, p1), k2)
    else:
        raise ValueError(f"unsupported 2-D phase kind {kind}")
    return t - np.rint(t)


def kernel_2d(kind, params, x, xi):
    t = phase_frac_2d(kind, params, x, xi)
    return np.cos(TWO_PI * t) + 1j * np.sin(TWO_PI * t)


def dense_apply_2d(kind, params, x, xi, g, rows=None, chunk=None):
    """u(x_i) = sum_j K(x_i, xi_j) g_j (rows of x selected by `rows`)."""
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    g = np.asarray(g, dtype=np.complex128)
    if g.ndim == 1:
        g = g[:, None]
    if rows is not None:
        x = x[rows]
    if chunk is None:
        chunk = max(1, min(512, (1 << 22) // max(len(xi), 1)))
    out = np.empty((len(x), g.shape[1]), dtype=np.complex128)
    for i0 in range(0, len(x), chunk):
        K = kernel_2d(kind, params, x[i0:i0 + chunk, None, :], xi[None, :, :])
        out[i0:i0 + chunk] = K @ g
    return out


# ----------------------------------------------------------------------------
# Quadtree indexing (Morton codes), tensor grids
# ----------------------------------------------------------------------------

def morton_encode(i1, i2, level):
    """Code with child digit 2 c1 + c2 per level, the coarsest split most significant."""
    i1 = np.asarray(i1, dtype=np.int64)
    i2 = np.asarray(i2, dtype=np.int64)
    code = np.zeros(np.broadcast(i1, i2).shape, dtype=np.int64)
    for j in range(level):
        code |= (((i1 >> j) & 1) * 2 + ((i2 >> j) & 1)) << (2 * j)
    return code


def morton_decode(code, level):
    code = np.asarray(code, dtype=np.int64)
    i1 = np.zeros_like(code)
    i2 = np.zeros_like(code)
    for j in range(level):
        d = (code >> (2 * j)) & 3
        i1 |= (d >> 1) << j
        i2 |= (d & 1) << j
    return i1, i2


def tensor_nodes(z):
    """Tensor grid offsets (z_t1, z_t2) with t = t1 r + t2."""
    r = len(z)
    return np.stack([np.repeat(z, r), np.tile(z, r)], axis=-1)         # [r^2, 2]


def lagrange_2d(z, y):
    """M_t(y) = M_t1(y1) M_t2(y2) for y of shape (..., 2); returns (..., r^2)."""
    m1 = lagrange(z, y[..., 0])
    m2 = lagrange(z, y[..., 1])
    return (m1[..., :, None] * m2[..., None, :]).reshape(y.shape[:-1] + (len(z) ** 2,))


def child_to_parent_2d(z):
    """Lc[c][t, s] = M^B_t(g^{C_c}_s) for the four children, c = 2 c1 + c2."""
    L1 = child_to_parent(z)
    return np.stack([np.kron(L1[c >> 1], L1[c & 1]) for c in range(4)])


# ----------------------------------------------------------------------------
# One box: geometry and the problem description
# ----------------------------------------------------------------------------

@dataclass
class Box2DProblem:
    kind: int
    params: tuple
    x: np.ndarray            # (n, 2) all X points, caller order
    xi: np.ndarray           # (m, 2) this box's Omega points
    o: np.ndarray            # lower corner of the box
    w: float                 # side (a power of two)
    r: int
    leaf_side: int
    L: int
    lV: int
    h: int
    z: np.ndarray
    Lc: np.ndarray           # [4, r^2, r^2]
    perm_x: np.ndarray       # sorted -> caller
    xoff: np.ndarray         # X leaves at level L (Morton), CSR
    perm_xi: np.ndarray
    xioff: np.ndarray        # Omega leaves at level L - lV (Morton), CSR

    def K(self, x, xi):
        return kernel_2d(self.kind, self.params, x, xi)

    def cx(self, level):
        i1, i2 = morton_decode(np.arange(4 ** level), level)
        return np.stack([(i1 + 0.5), (i2 + 0.5)], axis=-1) / (1 << level)

    def wx(self, level):
        return 1.0 / (1 << level)

    def cxi(self, level):
        j1, j2 = morton_decode(np.arange(4 ** level), level)
        return self.o + np.stack([(j1 + 0.5), (j2 + 0.5)], axis=-1) * (self.w / (1 << level))

    def wxi(self, level):
        return self.w / (1 << level)


def _leaf_sort(codes, nleaf):
    perm = np.argsort(codes, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(codes, minlength=nleaf))])
    return perm, off


def make_box_problem(kind, params, x, xi, o, w, r, leaf_side=4):
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    L = int(round(math.log2(w)))
    lV = int(round(math.log2(leaf_side)))
    if (1 << L) != w or (1 << lV) != leaf_side or L < lV:
        raise ValueError("box side and leaf side must be powers of two with side >= leaf side")
    lO = L - lV
    h = (lV + L) // 2
    nx = 1 << L
    i = np.clip(np.floor(x * nx).astype(np.int64), 0, nx - 1)
    px, xoff = _leaf_sort(morton_encode(i[:, 0], i[:, 1], L), 4 ** L)
    no = 1 << lO
    j = np.clip(np.floor((xi - o) * no / w).astype(np.int64), 0, no - 1)
    pxi, xioff = _leaf_sort(morton_encode(j[:, 0], j[:, 1], lO), 4 ** lO)
    z = cheb_nodes(r)
    return Box2DProblem(kind, tuple(params), x, xi, np.asarray(o, dtype=np.float64), float(w),
                        r, leaf_side, L, lV, h, z, child_to_parent_2d(z), px, xoff, pxi, xioff)


def _slots(off):
    cnt = np.diff(off)
    smax = max(int(cnt.max()) if len(cnt) else 1, 1)
    idx = -np.ones((len(cnt), smax), dtype=np.int64)
    for s in range(smax):
        has = cnt > s
        idx[has, s] = off[:-1][has] + s
    return idx


# ----------------------------------------------------------------------------
# Preliminary factors (Sec. 3 blocks with four children), apply
# ----------------------------------------------------------------------------

@dataclass
class Prelim2D:
    prob: Box2DProblem
    Vs: np.ndarray           # [a @lV, b leaf, t, slot]
    xi_idx: np.ndarray       # [b, slot] sorted Omega index or -1
    H: dict                  # l -> [a @l, b @L-l, c, t, s]
    M: np.ndarray            # [a @h, b @L-h, t, s]
    G: dict                  # l -> [a @l, b @L-l, c, t, s]
    U: np.ndarray            # [a @L, slot, t]   (B = the box itself)
    x_idx: np.ndarray


def prelim_factors_2d(P: Box2DProblem) -> Prelim2D:
    """V^*: conj K(c_A, g^B_t) M^B_t(xi) K(c_A, xi)       (eqn:PIBF1)
    H^l: conj K(c_A, g^B_t) M^B_t(g^C_s) K(c_A, g^C_s)     (eqn:PIBF2)
    M^h: K(g^A_t, g^B_s)                                   (eqn:switchlocM)
    G^l: K(g^A_t, c_C) M^P_s(g^A_t) conj K(g^P_s, c_C)     (eqn:PIBF3)
    U  : K(x, c_B) M^A_t(x) conj K(g^A_t, c_B)             (eqn:PIBFbf3)"""
    z, Lc, L, lV, h = P.z, P.Lc, P.L, P.lV, P.h
    zt = tensor_nodes(z)
    lO = L - lV

    xi_idx = _slots(P.xioff)
    cA = P.cx(lV)
    cB, wB = P.cxi(lO), P.wxi(lO)
    gB = cB[:, None, :] + wB * zt[None]
    ok = xi_idx >= 0
    xiv = np.where(ok[..., None], P.xi[P.perm_xi[np.maximum(xi_idx, 0)]], cB[:, None, :])
    Mxi = lagrange_2d(z, (xiv - cB[:, None, :]) / wB) * ok[..., None]        # [b, slot, t]
    Vs = (np.conj(P.K(cA[:, None, None, None, :], gB[None, :, :, None, :])) *
          np.transpose(Mxi, (0, 2, 1))[None] *
          P.K(cA[:, None, None, None, :], xiv[None, :, None, :, :]))         # [a, b, t, slot]

    H = {}
    for l in range(lV + 1, h + 1):
        nb = 4 ** (L - l)
        cA = P.cx(l)
        gB = P.cxi(L - l)[:, None, :] + P.wxi(L - l) * zt[None]
        gC = P.cxi(L - l + 1)[:, None, :] + P.wxi(L - l + 1) * zt[None]
        left = np.conj(P.K(cA[:, None, None, :], gB[None, :, :, :]))         # [a, b, t]
        blk = np.empty((4 ** l, nb, 4) + Lc.shape[1:], dtype=np.complex128)
        for c in range(4):
            right = P.K(cA[:, None, None, :], gC[4 * np.arange(nb) + c][None])  # [a, b, s]
            blk[:, :, c] = left[..., :, None] * Lc[c][None, None] * right[..., None, :]
        H[l] = blk

    gA = P.cx(h)[:, None, :] + P.wx(h) * zt[None]
    gB = P.cxi(L - h)[:, None, :] + P.wxi(L - h) * zt[None]
    M = P.K(gA[:, None, :, None, :], gB[None, :, None, :, :])

    G = {}
    for l in range(h + 1, L + 1):
        na, nb = 4 ** l, 4 ** (L - l)
        gA = P.cx(l)[:, None, :] + P.wx(l) * zt[None]
        gP = P.cx(l - 1)[:, None, :] + P.wx(l - 1) * zt[None]
        cC = P.cxi(L - l + 1)
        par = np.arange(na) >> 2
        alpha = np.arange(na) & 3
        Mx = np.transpose(Lc[alpha], (0, 2, 1))                              # [a, t, s]
        blk = np.empty((na, nb, 4) + Lc.shape[1:], dtype=np.complex128)
        for c in range(4):
            ch = cC[4 * np.arange(nb) + c]
            left = P.K(gA[:, None, :, :], ch[None, :, None, :])              # [a, b, t]
            right = np.conj(P.K(gP[par][:, None, :, :], ch[None, :, None, :]))   # [a, b, s]
            blk[:, :, c] = left[..., :, None] * Mx[:, None] * right[..., None, :]
        G[l] = blk

    x_idx = _slots(P.xoff)
    cA, wA = P.cx(L), P.wx(L)
    gA = cA[:, None, :] + wA * zt[None]
    cB = P.o + P.w / 2.0
    ok = x_idx >= 0
    xv = np.where(ok[..., None], P.x[P.perm_x[np.maximum(x_idx, 0)]], cA[:, None, :])
    Mx = lagrange_2d(z, (xv - cA[:, None, :]) / wA) * ok[..., None]          # [a, slot, t]
    U = (P.K(xv[:, :, None, :], cB) * Mx *
         np.conj(P.K(gA[:, None, :, :], cB)))                                # [a, slot, t]
    return Prelim2D(P, Vs, xi_idx, H, M, G, U, x_idx)


def _stage_2d(blk, lam):
    """new[a, b] = sum_c blk[a, b, c] @ lam[a >> 2, 4b + c]."""
    na, nb = blk.shape[0], blk.shape[1]
    out = 0
    for c in range(4):
        src = lam[np.arange(na) >> 2][:, 4 * np.arange(nb) + c]
        out = out + np.einsum("abts,absn->abtn", blk[:, :, c], src)
    return out


def _gather_g(P, g):
    g = np.asarray(g, dtype=np.complex128)
    if g.ndim == 1:
        g = g[:, None]
    return g


def _leaf_gather(idx, v):
    out = v[np.maximum(idx, 0)]
    out[idx < 0] = 0
    return out


def _scatter_u(P, x_idx, u_leaf):
    u_s = np.zeros((len(P.x), u_leaf.shape[-1]), dtype=np.complex128)
    ok = x_idx >= 0
    u_s[x_idx[ok]] = u_leaf[ok]
    u = np.empty_like(u_s)
    u[P.perm_x] = u_s
    return u


def apply_prelim_2d(F: Prelim2D, g):
    """u = U G^L..G^{h+1} M H^h..H^{lV+1} V^* g over this box's points."""
    P = F.prob
    gs = _gather_g(P, g)[P.perm_xi]
    lam = np.einsum("abts,bsn->abtn", F.Vs, _leaf_gather(F.xi_idx, gs))
    for l in range(P.lV + 1, P.h + 1):
        lam = _stage_2d(F.H[l], lam)
    lam = np.einsum("abts,absn->abtn", F.M, lam)
    for l in range(P.h + 1, P.L + 1):
        lam = _stage_2d(F.G[l], lam)
    u_leaf = np.einsum("ait,atn->ain", F.U, lam[:, 0])
    return _scatter_u(P, F.x_idx, u_leaf)


# ----------------------------------------------------------------------------
# Sweep-out compression (Sec. 4.2) with four children, apply
# ----------------------------------------------------------------------------

@dataclass
class Optimal2D:
    prob: Box2DProblem
    Vbar: np.ndarray         # [a @lV, b leaf, k, slot]
    xi_idx: np.ndarray
    F: dict                  # l -> [a, b, c, k_out, k_in], lV < l <= h
    Gbar: dict               # l -> [a, b, c, k_out, k_in], h < l <= L
    Ubar: np.ndarray         # [a @L, slot, k]
    x_idx: np.ndarray
    ranks: dict              # level -> per-pair ranks [a, b]


_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_MUL1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_MUL2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(seed, index):
    """u in [0, 1) from the top 53 bits of the (index + 1)-th output of
    SplitMix64 started at `seed` (state seed + n gamma, then the mix
    function), elementwise over `index` (uint64 arithmetic modulo 2^64)."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_MUL1
        z = (z ^ (z >> np.uint64(27))) * _SM_MUL2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


# block families of the draws: the middle, the sweep toward U producing level
# l, the sweep toward V producing level l - 1
SAMPLE_TAG_MIDDLE = 0


def sample_tag_g(l):
    return 1 + l


def sample_tag_h(l):
    return 64 + l


def sample_columns(seed, S, tag, real):
    """Mask of the kept columns: real[..., n_cols] marks the block's real
    columns (pairs enumerated in C order over the leading axes, columns by
    their index j); column j of pair p is kept iff it is real and
    u(seed, j + 2^9 p + 2^41 tag) < min(1, S / n_real)."""
    real = np.asarray(real, dtype=bool)
    npair = int(np.prod(real.shape[:-1]))
    ncol = real.shape[-1]
    pidx = np.arange(npair, dtype=np.uint64).reshape(real.shape[:-1] + (1,))
    j = np.arange(ncol, dtype=np.uint64)
    index = j + (pidx << np.uint64(9)) + (np.uint64(tag) << np.uint64(41))
    u = splitmix64_uniform(seed, index)
    n = real.sum(axis=-1)
    rho = np.minimum(1.0, S / np.maximum(n, 1).astype(np.float64))
    return real & (u < rho[..., None])


def sampled_svd(W, real, tol, seed, S, tag):
    """Randomized low-rank approximation of the blocks W[..., R2, n] from
    their sampled columns: U, the scaled singular values, and the rank k by
    the tolerance rule on the sampled values (scale-free)."""
    mask = sample_columns(seed, S, tag, real)
    U, Sv, _ = np.linalg.svd(W * mask[..., None, :], full_matrices=False)
    s1 = Sv[..., :1]
    k = np.where(s1[..., 0] > 0, np.sum(Sv > tol * s1, axis=-1), 0)
    nreal = real.sum(axis=-1).astype(np.float64)
    nkept = mask.sum(axis=-1).astype(np.float64)
    f = np.where(nkept > 0, np.sqrt(nreal / np.maximum(nkept, 1.0)), 0.0)
    return U, Sv * f[..., None], k


def _proj(W, U, Ssc, keep):
    """V_k^* = S_k^-1 U_k^* W for the kept columns of U (zero rows otherwise)."""
    inv = np.where(keep > 0, 1.0 / np.where(Ssc > 0, Ssc, 1.0), 0.0)
    return (np.conj(np.swapaxes(U, -1, -2)) @ W) * inv[..., :, None]


def sweep_out_2d(F: Prelim2D, tol: float, sample=None) -> Optimal2D:
    """Middle SVDs (eq:KeqUMV with Sigma^(1/2) on both sides), then
    eqn:GC toward U (C^{l} = U_k S_k, Gbar = V_k^*) and eqn:HR toward V.
    sample = (seed, S): the randomized low-rank approximation by column
    sampling described in the module header, for every block."""
    P = F.prob
    L, lV, h = P.L, P.lV, P.h
    R2 = P.r * P.r
    ranks = {}
    if sample is None:
        Um, Sm, Vhm, km = truncated_svd(F.M, tol)
        keep = _keep(km, R2)
        sq = np.sqrt(Sm) * keep
        Cl = {h: Um * sq[..., None, :]}
        Rl = {h: np.conj(np.swapaxes(Vhm, -1, -2)) * sq[..., None, :]}
    else:
        real = np.ones(F.M.shape[:-2] + (R2,), dtype=bool)
        Um, Sm, km = sampled_svd(F.M, real, tol, sample[0], sample[1], SAMPLE_TAG_MIDDLE)
        keep = _keep(km, R2)
        sq = np.sqrt(Sm) * keep
        Cl = {h: Um * sq[..., None, :]}
        # V_k S_k^(1/2) = M^* U_k S_k^(-1/2)
        isq = np.where(keep > 0, 1.0 / np.where(sq > 0, sq, 1.0), 0.0)
        Rl = {h: (np.conj(np.swapaxes(F.M, -1, -2)) @ Um) * isq[..., None, :]}
    ranks[h] = km

    Gbar = {}
    for l in range(h + 1, L + 1):
        na, nb = 4 ** l, 4 ** (L - l)
        Cprev = Cl[l - 1]
        par = np.arange(na) >> 2
        W = np.concatenate([F.G[l][:, :, c] @ Cprev[par][:, 4 * np.arange(nb) + c]
                            for c in range(4)], axis=-1)                     # [a, b, R2, 4 R2]
        if sample is None:
            Uw, Sw, Vhw, kw = truncated_svd(W, tol)
            keep = _keep(kw, R2)
            Cl[l] = Uw[..., :R2] * (Sw[..., :R2] * keep)[..., None, :]
            Vk = Vhw[..., :R2, :] * keep[..., :, None]                       # [a, b, k, 4 R2]
        else:
            kprev = ranks[l - 1][par][:, 4 * np.arange(nb)[:, None] + np.arange(4)]   # [a, b, c]
            real = np.arange(R2)[None, None, None, :] < kprev[..., None]             # [a, b, c, m]
            real = real.reshape(na, nb, 4 * R2)
            Uw, Sw, kw = sampled_svd(W, real, tol, sample[0], sample[1], sample_tag_g(l))
            keep = _keep(kw, R2)
            Cl[l] = Uw[..., :R2] * (Sw[..., :R2] * keep)[..., None, :]
            Vk = _proj(W, Uw[..., :R2], Sw[..., :R2], keep)                  # [a, b, k, 4 R2]
        Gbar[l] = np.stack([Vk[..., c * R2:(c + 1) * R2] for c in range(4)], axis=2)
        ranks[l] = kw

    Fh = {}
    for l in range(h, lV, -1):
        na, nb = 4 ** l, 4 ** (L - l)
        Rcur = Rl[l]                                                         # [a, b, t, k]
        # input pair (p @ l-1, j @ L-l+1): outputs (4p + alpha, j >> 2), child j & 3
        npar, nin = na // 4, nb * 4
        p = np.arange(npar)[:, None]
        j = np.arange(nin)[None, :]
        parts = []
        for alpha in range(4):
            A = 4 * p + alpha
            Hs = np.conj(np.swapaxes(F.H[l][A, j >> 2, j & 3], -1, -2))     # [p, j, s, t]
            parts.append(Hs @ Rcur[A, j >> 2])
        Z = np.concatenate(parts, axis=-1)                                   # [p, j, R2, 4 R2]
        if sample is None:
            Uz, Sz, Vhz, kz = truncated_svd(Z, tol)
            keep = _keep(kz, R2)
            Rl[l - 1] = Uz[..., :R2] * (Sz[..., :R2] * keep)[..., None, :]
            Vk = np.conj(np.swapaxes(Vhz[..., :R2, :], -1, -2)) * keep[..., None, :]   # [p, j, 4 R2, k]
        else:
            kcur = np.stack([ranks[l][4 * p + alpha, j >> 2] for alpha in range(4)], -1)  # [p, j, 4]
            real = (np.arange(R2)[None, None, None, :] < kcur[..., None]).reshape(npar, nin, 4 * R2)
            Uz, Sz, kz = sampled_svd(Z, real, tol, sample[0], sample[1], sample_tag_h(l))
            keep = _keep(kz, R2)
            Rl[l - 1] = Uz[..., :R2] * (Sz[..., :R2] * keep)[..., None, :]
            Vk = np.conj(np.swapaxes(_proj(Z, Uz[..., :R2], Sz[..., :R2], keep), -1, -2))
        blk = np.empty((na, nb, 4, R2, R2), dtype=np.complex128)
        for alpha in range(4):
            blk[(4 * p + alpha), j >> 2, j & 3] = Vk[:, :, alpha * R2:(alpha + 1) * R2, :]
        Fh[l] = blk
        ranks[l - 1] = kz

    Vbar = np.conj(np.swapaxes(Rl[lV], -1, -2)) @ F.Vs                      # eqn:V0
    Ubar = F.U @ Cl[L][:, 0]                                                 # U C^L
    return Optimal2D(P, Vbar, F.xi_idx, Fh, Gbar, Ubar, F.x_idx, ranks)


def apply_optimal_2d(O: Optimal2D, g):
    P = O.prob
    gs = _gather_g(P, g)[P.perm_xi]
    mu = np.einsum("abks,bsn->abkn", O.Vbar, _leaf_gather(O.xi_idx, gs))
    for l in range(P.lV + 1, P.h + 1):
        mu = _stage_2d(O.F[l], mu)
    for l in range(P.h + 1, P.L + 1):
        mu = _stage_2d(O.Gbar[l], mu)
    u_leaf = np.einsum("aik,akn->ain", O.Ubar, mu[:, 0])
    return _scatter_u(P, O.x_idx, u_leaf)


def level_ranks_2d(O: Optimal2D):
    return {l: int(np.max(k)) for l, k in sorted(O.ranks.items())}


def nnz_prelim_2d(P: Box2DProblem):
    R2 = P.r * P.r
    npairs = 4 ** P.L
    return (len(P.xi) * 4 ** P.lV * R2 + len(P.x) * R2 +
            (P.L - P.lV) * npairs * 4 * R2 * R2 + npairs * R2 * R2)


def nnz_optimal_2d(O: Optimal2D):
    P = O.prob
    L, lV, h = P.L, P.lV, P.h
    rk = O.ranks
    tot = int(np.sum(rk[lV] * np.diff(P.xioff)[None, :]))                  # Vbar
    tot += int(np.sum(rk[L][:, 0] * np.diff(P.xoff)))                        # Ubar
    tot += int(np.sum(rk[h]))                                                # middle diagonal
    for l in range(lV + 1, L + 1):
        na, nb = 4 ** l, 4 ** (L - l)
        kin = rk[l - 1]
        ks = sum(kin[np.arange(na) >> 2][:, 4 * np.arange(nb) + c] for c in range(4))
        tot += int(np.sum(rk[l] * ks))
    return tot


def build_box(kind, params, x, xi, o, w, r, tol, leaf_side=4, sample=None):
    P = make_box_problem(kind, params, x, xi, o, w, r, leaf_side)
    F = prelim_factors_2d(P)
    return P, F, sweep_out_2d(F, tol, sample)


# ----------------------------------------------------------------------------
# MIBF: corona decomposition and multiscale sum (Sec. 5)
# ----------------------------------------------------------------------------

def mibf_boxes(n: int, centre: int = 16):
    """The boxes (lower corner, side) of every corona of [-n/2, n/2)^2, outermost
    first, and the centre square's half-side."""
    boxes = []
    t = 0
    while (n >> (t + 1)) > centre // 2:
        hw = n >> (t + 1)                      # half-width of the outer square
        w = n >> (t + 2)                       # box side
        for i1 in range(4):
            for i2 in range(4):
                if 1 <= i1 <= 2 and 1 <= i2 <= 2:
                    continue                   # the inner square
                boxes.append((np.array([-hw + i1 * w, -hw + i2 * w], dtype=np.float64), w))
        t += 1
    return boxes, centre // 2


def mibf_partition(xi, n: int, centre: int = 16):
    """Index of the box holding each xi (-1 for the centre, -2 outside)."""
    xi = np.asarray(xi, dtype=np.float64)
    boxes, hc = mibf_boxes(n, centre)
    part = np.full(len(xi), -2, dtype=np.int64)
    inside = np.all((xi >= -hc) & (xi < hc), axis=1)
    part[inside] = -1
    for i, (o, w) in enumerate(boxes):
        m = np.all((xi >= o) & (xi < o + w), axis=1)
        part[m] = i
    return part


def mibf_build(kind, params, x, xi, n, r, tol, leaf_side=4, centre=16, sample=None):
    part = mibf_partition(xi, n, centre)
    boxes, hc = mibf_boxes(n, centre)
    built = []
    for i, (o, w) in enumerate(boxes):
        idx = np.nonzero(part == i)[0]
        P, F, O = build_box(kind, params, x, xi[idx], o, w, r, tol, leaf_side, sample)
        built.append((idx, P, F, O))
    return part, built, np.nonzero(part == -1)[0]


def mibf_apply(kind, params, x, xi, g, built, centre_idx, which="optimal"):
    """eq:f1: K_C R_C g + sum over boxes of IBF_t R_t g."""
    g = np.asarray(g, dtype=np.complex128)
    if g.ndim == 1:
        g = g[:, None]
    u = dense_apply_2d(kind, params, x, xi[centre_idx], g[centre_idx])
    for idx, P, F, O in built:
        u = u + (apply_optimal_2d(O, g[idx]) if which == "optimal" else apply_prelim_2d(F, g[idx]))
    return u


def nnz_mibf(built, centre_idx, n_x):
    pre = sum(nnz_prelim_2d(P) for _, P, _, _ in built) + n_x * len(centre_idx)
    opt = sum(nnz_optimal_2d(O) for _, _, _, O in built) + n_x * len(centre_idx)
    return pre, opt


__all__ = ["splitmix64_uniform", "sample_columns", "sampled_svd", "phase_frac_2d", "kernel_2d", "dense_apply_2d", "morton_encode", "morton_decode",
           "make_box_problem", "prelim_factors_2d", "apply_prelim_2d", "sweep_out_2d",
           "apply_optimal_2d", "build_box", "mibf_boxes", "mibf_partition", "mibf_build",
           "mibf_apply", "nnz_mibf", "rel_error", "level_ranks_2d"]
