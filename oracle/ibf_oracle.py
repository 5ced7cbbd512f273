"""Plain FP64 CPU oracle for the interpolative butterfly factorization (IBF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this module; only the tests, the smoke check and the CPU-baseline
leg of the benchmark may.  It shares no code with the HIP implementation.

Everything is complex128 / float64, written for readability, vectorised over
box pairs with numpy (a library matmul, einsum and SVD serve as steps; there
is no blocking or fusion).  The passages followed are cited per function:

* Sec. 1    -- the kernel a(x, xi) exp(2 pi i Phi(x, xi)) of eqn:FIO; the
  paper then sets a == 1, here a general smooth amplitude is also kept
  (it enters only the switch blocks, see prelim_factors).
* Sec. 2.1  -- Chebyshev grid, Lagrange polynomials, the split of Phi
  (eqn:RAB, eqn:terms) and the interpolative factors (eqn:ab1, eqn:ab2).
* Sec. 2.2  -- Algorithm 2.1, the butterfly algorithm (eqn:1, eqn:2, the
  switch, eqn:3, eqn:bf3).
* Sec. 3    -- the preliminary IBF factors V^0, H^l, M^h, G^l, U^L
  (eqn:PIBF1, eqn:PIBF2, eqn:switchlocM, eqn:PIBF3, eqn:PIBFbf3).
* Sec. 4    -- structure-preserving compression, the sweep-out stage
  (middle factorization eq:KeqUMV, eqn:GC, eqn:HR, eqn:V0) and the sweep-in
  stage (eqn:IBFin); SVD rearrangements eq:lowrankSVD / 2 / 3 of Sec. 2.1.
* Sec. 6    -- the sampled relative error (eq:relativeerr) and R_comp
  (eq:compratio).

Readings of points where the paper is silent (each also listed in the design
notes): leaves hold `leaf` points while every box pair keeps w_A * w_B <= 1
(the butterfly runs from level l0 = log2(leaf) to L - l0, and the first and
last log2(leaf) levels collapse into exact leaf <-> grid blocks); boxes are
half-open with geometric centres; Chebyshev grids are 0-based with t = 0 at
+1/2; the middle level is h = floor(L/2); truncation keeps sigma_i >
tol * sigma_1 per block (optionally capped per level, cap_rank); the middle
block splits Sigma^(1/2) to both sides,
the sweep-out recursion keeps U_k Sigma_k on the basis side, the sweep-in
keeps Sigma_k V_k^* on the basis side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

TWO_PI = 2.0 * math.pi

# ----------------------------------------------------------------------------
# Phase functions with exact mod-1 reduction
# ----------------------------------------------------------------------------

_VELTKAMP = 134217729.0  # 2^27 + 1


def _split(a):
    """Veltkamp splitting a = hi + lo with 26-bit halves."""
    c = _VELTKAMP * a
    hi = c - (c - a)
    return hi, a - hi


def two_product(a, b):
    """Dekker's error-free product: a*b = p + e exactly (no FMA needed)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def _frac_of_product(a, b):
    """(a*b) mod 1 in [-1/2, 1/2], exact up to one final rounding."""
    p, e = two_product(a, b)
    t = (p - np.rint(p)) + e
    return t - np.rint(t)


def phase_frac(kind, params, x, xi):
    """Phi(x, xi) reduced mod 1 to [-1/2, 1/2] (float64, broadcasting).

    The kernel is K = exp(2 pi i Phi) (paper eqn:FIO with a == 1), so only
    Phi mod 1 matters.  Products of a coordinate with a frequency are reduced
    error-free, because Phi grows like N and a plain float64 product would
    lose the fractional part's low bits.

    kind 0: Phi = s x xi                         (Sec. 6.1, s = params[0])
    kind 1: Phi = x xi + c(x)|xi|, c = (p0 + p1 sin 2 pi x)/p2   (Sec. 6.2)
    kind 3: Phi = p0 x + p1 xi  (separable; R^{AB} == 0 in eqn:RAB)
    For kind 2 (2-D) see ibf2d_oracle.phase_frac_2d.
    """
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    if kind == 0:
        s = params[0] if params else 1.0
        t = _frac_of_product(x, xi)
        t = s * t
    elif kind == 1:
        p0, p1, p2 = params
        c = (p0 + p1 * np.sin(TWO_PI * x)) / p2
        t = _frac_of_product(x, xi) + _frac_of_product(c, np.abs(xi))
    elif kind == 3:
        p0, p1 = params
        x, xi = np.broadcast_arrays(x, xi)
        t = _frac_of_product(np.full_like(x, p0), x) + \
            _frac_of_product(np.full_like(xi, p1), xi)
    else:
        raise ValueError(f"unsupported 1-D phase kind {kind}")
    return t - np.rint(t)


def kernel(kind, params, x, xi):
    """K(x, xi) = exp(2 pi i Phi(x, xi)) evaluated from the reduced phase."""
    t = phase_frac(kind, params, x, xi)
    return np.cos(TWO_PI * t) + 1j * np.sin(TWO_PI * t)


# ----------------------------------------------------------------------------
# Amplitude a(x, xi) of eqn:FIO (Sec. 1)
# ----------------------------------------------------------------------------

AMP_NONE, AMP_SEPARABLE, AMP_WAVE = 0, 1, 2


def amplitude(amp, x, xi):
    """a(x, xi) of the kernel a(x, xi) exp(2 pi i Phi(x, xi)) (eqn:FIO).

    The paper assumes a == 1 after noting that a smooth symbol of order zero
    is numerically low-rank (Sec. 1).  amp = (kind, params) or None:
    kind 0: a == 1
    kind 1: a = (q0 + q1 sin 2 pi x + q2 cos 2 pi x) (q3 + q4 xi / sqrt(xi^2 + q5^2)),
            a product of a smooth function of x and an order-zero symbol in xi
    kind 2: a = q0 + q1 cos(2 pi (x + xi / q2)), smooth and not separable
            when q2 is at least the width of Omega
    """
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    x, xi = np.broadcast_arrays(x, xi)
    if amp is None or amp[0] == AMP_NONE:
        return np.ones(x.shape)
    kind, q = amp[0], amp[1]
    if kind == AMP_SEPARABLE:
        fx = q[0] + q[1] * np.sin(TWO_PI * x) + q[2] * np.cos(TWO_PI * x)
        fxi = q[3] + q[4] * xi / np.sqrt(xi * xi + q[5] * q[5])
        return fx * fxi
    if kind == AMP_WAVE:
        return q[0] + q[1] * np.cos(TWO_PI * (x + xi / q[2]))
    raise ValueError(f"unsupported amplitude kind {kind}")


# ----------------------------------------------------------------------------
# Dense direct product (the definition u = K g, eqn:DFIO)
# ----------------------------------------------------------------------------

def dense_apply(kind, params, x, xi, g, rows=None, chunk=None, amp=None):
    """u(x_i) = sum_j a(x_i, xi_j) K(x_i, xi_j) g_j for the selected rows (all
    by default); a == 1 unless `amp` is given.

    g has shape (n_xi,) or (n_xi, nrhs).  O(rows * n_xi) work, chunked so that
    one chunk of the kernel matrix holds about 2^22 entries.
    """
    if chunk is None:
        chunk = max(1, min(512, (1 << 22) // max(len(xi), 1)))
    g = np.asarray(g, dtype=np.complex128)
    squeeze = g.ndim == 1
    if squeeze:
        g = g[:, None]
    rows = np.arange(len(x)) if rows is None else np.asarray(rows)
    out = np.empty((len(rows), g.shape[1]), dtype=np.complex128)
    for s in range(0, len(rows), chunk):
        rr = rows[s:s + chunk]
        K = kernel(kind, params, x[rr][:, None], xi[None, :])
        if amp is not None:
            K = K * amplitude(amp, x[rr][:, None], xi[None, :])
        out[s:s + chunk] = K @ g
    return out[:, 0] if squeeze else out


# ----------------------------------------------------------------------------
# Chebyshev grid and Lagrange polynomials (Sec. 2.1)
# ----------------------------------------------------------------------------

def cheb_nodes(r):
    """z_t = cos(t pi/(r-1))/2, t = 0..r-1, on [-1/2, 1/2] (t = 0 at +1/2)."""
    t = np.arange(r, dtype=np.float64)
    return 0.5 * np.cos(t * math.pi / (r - 1))


def lagrange(z, y):
    """M_t(y) = prod_{j != t} (y - z_j)/(z_t - z_j) for every y (rows) and t.

    Product formula of Sec. 2.1 in normalised coordinates.  Returns an array of
    shape y.shape + (r,).
    """
    y = np.asarray(y, dtype=np.float64)
    r = len(z)
    out = np.ones(y.shape + (r,), dtype=np.float64)
    for t in range(r):
        for j in range(r):
            if j != t:
                out[..., t] *= (y - z[j]) / (z[t] - z[j])
    return out


def child_to_parent(z):
    """Lc[c][t, s] = M^B_t(g^{C_c}_s) for child c in {0,1} of a box B.

    In normalised coordinates the child grid point is (2c-1)/4 + z_s/2, the
    same for every box at every level (Sec. 3, eqn:PIBF2).
    """
    out = []
    for c in (0, 1):
        y = (2 * c - 1) / 4.0 + z / 2.0          # child grid in parent coords
        out.append(lagrange(z, y).T)             # [t, s]
    return np.stack(out)


# ----------------------------------------------------------------------------
# Geometry: dyadic trees, leaves, pair levels (Sec. 3 notation)
# ----------------------------------------------------------------------------

@dataclass
class Tree1D:
    """Dyadic trees T_X on [0,1) and T_Omega on [lo, lo + W).

    L = ceil(log2 W) so that a T_X box at level l (width 2^-l) and a T_Omega
    box at level L-l (width W 2^(l-L)) satisfy w_A w_B = W/2^L <= 1.  Leaves of
    both trees sit at level L - l0 with l0 = log2(leaf).
    """
    x: np.ndarray           # caller order
    xi: np.ndarray
    leaf: int
    lo: float
    W: float
    L: int
    l0: int
    h: int
    perm_x: np.ndarray      # sorted position -> caller index
    perm_xi: np.ndarray
    xs: np.ndarray          # sorted coordinates
    xis: np.ndarray
    xleaf: np.ndarray       # leaf index per sorted point
    xileaf: np.ndarray
    xoff: np.ndarray        # CSR offsets, nleaf + 1
    xioff: np.ndarray

    @property
    def nleaf(self):
        return 1 << (self.L - self.l0)

    def cx(self, level):
        """Centres of T_X boxes at `level`."""
        n = 1 << level
        return (np.arange(n) + 0.5) / n

    def wx(self, level):
        return 1.0 / (1 << level)

    def cxi(self, level):
        n = 1 << level
        return self.lo + (np.arange(n) + 0.5) * (self.W / n)

    def wxi(self, level):
        return self.W / (1 << level)


def build_tree(x, xi, leaf=16, lo=None, W=None):
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    n = len(xi)
    if W is None:
        W = float(n)
    if lo is None:
        lo = -float(n // 2)
    L = int(math.ceil(math.log2(W) - 1e-12))
    l0 = int(round(math.log2(leaf)))
    if (1 << l0) != leaf:
        raise ValueError("leaf must be a power of two")
    if L < 2 * l0:
        raise ValueError("need W >= leaf^2")
    h = L // 2
    nl = 1 << (L - l0)
    ix = np.clip(np.floor(x * nl).astype(np.int64), 0, nl - 1)
    ixi = np.clip(np.floor((xi - lo) * nl / W).astype(np.int64), 0, nl - 1)
    px = np.argsort(ix, kind="stable")
    pxi = np.argsort(ixi, kind="stable")
    xoff = np.concatenate([[0], np.cumsum(np.bincount(ix, minlength=nl))])
    xioff = np.concatenate([[0], np.cumsum(np.bincount(ixi, minlength=nl))])
    return Tree1D(x, xi, leaf, lo, W, L, l0, h, px, pxi, x[px], xi[pxi],
                  ix[px], ixi[pxi], xoff, xioff)


def leaf_slots(off):
    """Padded leaf table: idx[leaf, slot] into sorted points, -1 when empty."""
    cnt = np.diff(off)
    smax = max(int(cnt.max()), 1)
    idx = -np.ones((len(cnt), smax), dtype=np.int64)
    for s in range(smax):
        has = cnt > s
        idx[has, s] = off[:-1][has] + s
    return idx


# ----------------------------------------------------------------------------
# Problem description used by every oracle routine
# ----------------------------------------------------------------------------

@dataclass
class IBFProblem:
    kind: int
    params: tuple
    tree: Tree1D
    r: int
    z: np.ndarray
    Lc: np.ndarray          # child -> parent Lagrange matrices [2, r, r]
    amp: tuple | None = None   # amplitude (kind, params), None for a == 1

    def K(self, x, xi):
        return kernel(self.kind, self.params, x, xi)

    def Ka(self, x, xi):
        """The full kernel a(x, xi) exp(2 pi i Phi(x, xi)) (eqn:FIO)."""
        if self.amp is None:
            return self.K(x, xi)
        return amplitude(self.amp, x, xi) * self.K(x, xi)


def make_problem(kind, params, x, xi, r, leaf=16, lo=None, W=None, amp=None):
    tree = build_tree(x, xi, leaf, lo, W)
    z = cheb_nodes(r)
    return IBFProblem(kind, tuple(params), tree, r, z, child_to_parent(z), amp)


def _g_sorted(prob, g):
    g = np.asarray(g, dtype=np.complex128)
    if g.ndim == 1:
        g = g[:, None]
    return g[prob.tree.perm_xi]


def _unsort_u(prob, u_sorted):
    u = np.empty_like(u_sorted)
    u[prob.tree.perm_x] = u_sorted
    return u


# ----------------------------------------------------------------------------
# Algorithm 2.1 (butterfly algorithm), as a direct recursion on coefficients
# ----------------------------------------------------------------------------

def butterfly_algorithm(prob: IBFProblem, g):
    """u ~= K g by Algorithm 2.1 with the collapsed leaf levels.

    lam[a, b, t, n]: coefficients of pair (A = T_X box a at level l,
    B = T_Omega box b at level L - l), Chebyshev index t, right-hand side n.
    """
    T = prob.tree
    L, l0, h, r = T.L, T.l0, T.h, prob.r
    z, Lc = prob.z, prob.Lc
    gs = _g_sorted(prob, g)
    nrhs = gs.shape[1]

    # Initialisation (eqn:1): A over T_X level l0, B over Omega leaves.
    cA = T.cx(l0)
    lev_b = L - l0
    cB, wB = T.cxi(lev_b), T.wxi(lev_b)
    gB = cB[:, None] + wB * z[None, :]                      # [b, t]
    yb = (T.xis - cB[T.xileaf]) / wB                        # normalised xi
    Mxi = lagrange(z, yb)                                   # [j, t]
    E = prob.K(cA[:, None], T.xis[None, :])                 # [a, j]
    memb = sp.csr_matrix((np.ones(len(T.xis)), (T.xileaf, np.arange(len(T.xis)))),
                         shape=(T.nleaf, len(T.xis)))
    lam = np.empty((len(cA), T.nleaf, r, nrhs), dtype=np.complex128)
    for a in range(len(cA)):
        val = (E[a][:, None, None] * Mxi[:, :, None]) * gs[:, None, :]   # [j, t, n]
        s = memb @ val.reshape(len(T.xis), r * nrhs)
        lam[a] = np.asarray(s).reshape(T.nleaf, r, nrhs)
    lam *= np.conj(prob.K(cA[:, None, None], gB[None, :, :]))[..., None]

    # Recursion in xi (eqn:2) for l = l0+1 .. h.
    for l in range(l0 + 1, h + 1):
        na, nb = 1 << l, 1 << (L - l)
        cA = T.cx(l)
        cB, wB = T.cxi(L - l), T.wxi(L - l)
        cC, wC = T.cxi(L - l + 1), T.wxi(L - l + 1)
        gB = cB[:, None] + wB * z[None, :]                  # [b, t]
        gC = cC[:, None] + wC * z[None, :]                  # [child, s]
        new = np.zeros((na, nb, r, nrhs), dtype=np.complex128)
        for c in (0, 1):
            ch = 2 * np.arange(nb) + c
            # e^{2 pi i Phi(c_A, g^C_s)} lam^{PC}_s
            inner = prob.K(cA[:, None, None], gC[ch][None, :, :])[..., None] * \
                lam[np.arange(na) // 2][:, ch]
            new += np.einsum("ts,absn->abtn", Lc[c], inner)
        new *= np.conj(prob.K(cA[:, None, None], gB[None, :, :]))[..., None]
        lam = new

    # Switch at the middle level h: the only place where the amplitude enters
    # (the interpolation steps carry a(x, xi) exp(2 pi i R^{AB}) implicitly
    # through kernel values at grid points).
    gA = T.cx(h)[:, None] + T.wx(h) * z[None, :]
    gB = T.cxi(L - h)[:, None] + T.wxi(L - h) * z[None, :]
    Msw = prob.Ka(gA[:, None, :, None], gB[None, :, None, :])   # [a, b, t, s]
    lam = np.einsum("abts,absn->abtn", Msw, lam)

    # Recursion in x (eqn:3) for l = h+1 .. L-l0.
    for l in range(h + 1, L - l0 + 1):
        na, nb = 1 << l, 1 << (L - l)
        gA = T.cx(l)[:, None] + T.wx(l) * z[None, :]        # [a, t]
        gP = T.cx(l - 1)[:, None] + T.wx(l - 1) * z[None, :]
        cC = T.cxi(L - l + 1)
        new = np.zeros((na, nb, r, nrhs), dtype=np.complex128)
        par = np.arange(na) // 2
        alpha = np.arange(na) % 2
        for c in (0, 1):
            ch = 2 * np.arange(nb) + c
            # e^{-2 pi i Phi(g^P_s, c_C)} lam^{PC}_s
            inner = np.conj(prob.K(gP[par][:, None, :], cC[ch][None, :, None]))[..., None] * \
                lam[par][:, ch]                                        # [a, b, s, n]
            # M^P_s(g^A_t) = Lc[alpha][s, t]
            Mx = Lc[alpha]                                             # [a, s, t]
            interp = np.einsum("ast,absn->abtn", Mx, inner)
            new += prob.K(gA[:, None, :], cC[ch][None, :, None])[..., None] * interp
        lam = new

    # Termination (eqn:bf3): X leaves at level L-l0, B over T_Omega level l0.
    la = L - l0
    cA, wA = T.cx(la), T.wx(la)
    gA = cA[:, None] + wA * z[None, :]                      # [a, t]
    cB = T.cxi(l0)                                          # [b]
    ya = (T.xs - cA[T.xleaf]) / wA
    Mx = lagrange(z, ya)                                    # [i, t]
    D = np.conj(prob.K(gA[:, None, :], cB[None, :, None]))  # [a, b, t]
    coef = D[..., None] * lam                               # [a, b, t, n]
    Ei = prob.K(T.xs[:, None], cB[None, :])                 # [i, b]
    u_s = np.einsum("ib,it,ibtn->in", Ei, Mx, coef[T.xleaf])
    return _unsort_u(prob, u_s)


# ----------------------------------------------------------------------------
# Preliminary IBF: explicit factor blocks (Sec. 3)
# ----------------------------------------------------------------------------

@dataclass
class PrelimIBF:
    prob: IBFProblem
    Vs: np.ndarray          # [a, b, t, slot]  V^*_{AB} per (T_X box @l0, Omega leaf)
    xi_idx: np.ndarray      # [b, slot] sorted Omega index or -1
    H: dict                 # l -> [a, b, c, t, s] for output pair (a,b) @ l, l0 < l <= h
    M: np.ndarray           # [a, b, t, s] at level h
    G: dict                 # l -> [a, b, c, t, s] for output pair (a,b) @ l, h < l <= L-l0
    U: np.ndarray           # [a, b, slot, t] per (X leaf, T_Omega box @l0)
    x_idx: np.ndarray       # [a, slot] sorted X index or -1


def prelim_factors(prob: IBFProblem) -> PrelimIBF:
    """All blocks of the preliminary IBF from their explicit formulas.

    V^*  : eqn:PIBF1  e^{-2pi i Phi(c_A,g^B_t)} M^B_t(xi) e^{2pi i Phi(c_A,xi)}
    H^l  : eqn:PIBF2  e^{-2pi i Phi(c_A,g^B_t)} M^B_t(g^C_s) e^{2pi i Phi(c_A,g^C_s)}
    M^h  : eqn:switchlocM  K(g^A_t, g^B_s) = a(g^A_t, g^B_s) e^{2pi i Phi(g^A_t, g^B_s)}
           (with a general amplitude the interpolation of eqn:ab1 / eqn:ab2 is
           applied to a(x, xi) exp(2 pi i R^{AB}); a cancels from every other
           block because they only move between interpolation grids)
    G^l  : eqn:PIBF3  e^{2pi i Phi(g^A_t,c_C)} M^P_s(g^A_t) e^{-2pi i Phi(g^P_s,c_C)}
    U^L  : eqn:PIBFbf3  e^{2pi i Phi(x,c_B)} M^A_t(x) e^{-2pi i Phi(g^A_t,c_B)}
    """
    T, z, Lc, r = prob.tree, prob.z, prob.Lc, prob.r
    L, l0, h = T.L, T.l0, T.h

    # V^*: A at T_X level l0, B an Omega leaf.
    xi_idx = leaf_slots(T.xioff)
    lb = L - l0
    cA = T.cx(l0)
    cB, wB = T.cxi(lb), T.wxi(lb)
    gB = cB[:, None] + wB * z[None, :]
    ok = xi_idx >= 0
    xiv = np.where(ok, T.xis[np.maximum(xi_idx, 0)], cB[:, None])
    Mxi = lagrange(z, (xiv - cB[:, None]) / wB)                 # [b, slot, t]
    Mxi = Mxi * ok[..., None]
    Vs = (np.conj(prob.K(cA[:, None, None, None], gB[None, :, :, None])) *
          np.transpose(Mxi, (0, 2, 1))[None] *
          prob.K(cA[:, None, None, None], xiv[None, :, None, :]))  # [a, b, t, slot]

    H = {}
    for l in range(l0 + 1, h + 1):
        na, nb = 1 << l, 1 << (L - l)
        cA = T.cx(l)
        gB = T.cxi(L - l)[:, None] + T.wxi(L - l) * z[None, :]
        gC = T.cxi(L - l + 1)[:, None] + T.wxi(L - l + 1) * z[None, :]
        blk = np.empty((na, nb, 2, r, r), dtype=np.complex128)
        for c in (0, 1):
            ch = 2 * np.arange(nb) + c
            left = np.conj(prob.K(cA[:, None, None], gB[None, :, :]))     # [a, b, t]
            right = prob.K(cA[:, None, None], gC[ch][None, :, :])          # [a, b, s]
            blk[:, :, c] = left[..., :, None] * Lc[c][None, None] * right[..., None, :]
        H[l] = blk

    gA = T.cx(h)[:, None] + T.wx(h) * z[None, :]
    gB = T.cxi(L - h)[:, None] + T.wxi(L - h) * z[None, :]
    M = prob.Ka(gA[:, None, :, None], gB[None, :, None, :])

    G = {}
    for l in range(h + 1, L - l0 + 1):
        na, nb = 1 << l, 1 << (L - l)
        gA = T.cx(l)[:, None] + T.wx(l) * z[None, :]
        gP = T.cx(l - 1)[:, None] + T.wx(l - 1) * z[None, :]
        cC = T.cxi(L - l + 1)
        par = np.arange(na) // 2
        alpha = np.arange(na) % 2
        blk = np.empty((na, nb, 2, r, r), dtype=np.complex128)
        for c in (0, 1):
            ch = 2 * np.arange(nb) + c
            left = prob.K(gA[:, None, :], cC[ch][None, :, None])               # [a, b, t]
            right = np.conj(prob.K(gP[par][:, None, :], cC[ch][None, :, None]))  # [a, b, s]
            Mx = np.transpose(Lc[alpha], (0, 2, 1))                            # [a, t, s]
            blk[:, :, c] = left[..., :, None] * Mx[:, None] * right[..., None, :]
        G[l] = blk

    x_idx = leaf_slots(T.xoff)
    la = L - l0
    cA, wA = T.cx(la), T.wx(la)
    gA = cA[:, None] + wA * z[None, :]
    cB = T.cxi(l0)
    ok = x_idx >= 0
    xv = np.where(ok, T.xs[np.maximum(x_idx, 0)], cA[:, None])
    Mx = lagrange(z, (xv - cA[:, None]) / wA) * ok[..., None]   # [a, slot, t]
    U = (prob.K(xv[:, None, :, None], cB[None, :, None, None]) *
         Mx[:, None] *
         np.conj(prob.K(gA[:, None, None, :], cB[None, :, None, None])))   # [a, b, slot, t]
    return PrelimIBF(prob, Vs, xi_idx, H, M, G, U, x_idx)


def _leaf_gather(idx, v):
    """v[sorted] -> [leaf, slot, n] with zeros for empty slots."""
    ok = idx >= 0
    out = v[np.maximum(idx, 0)]
    out[~ok] = 0
    return out


def _stage(blk, lam):
    """new[a,b] = sum_c blk[a,b,c] @ lam[a//2, 2b+c]   (eqn:PIBFMatR1 pattern)."""
    na, nb = blk.shape[0], blk.shape[1]
    out = 0
    for c in (0, 1):
        src = lam[np.arange(na) // 2][:, 2 * np.arange(nb) + c]
        out = out + np.einsum("abts,absn->abtn", blk[:, :, c], src)
    return out


def _scatter_u(prob, x_idx, u_leaf):
    n = len(prob.tree.xs)
    u_s = np.zeros((n, u_leaf.shape[-1]), dtype=np.complex128)
    ok = x_idx >= 0
    u_s[x_idx[ok]] = u_leaf[ok]
    return _unsort_u(prob, u_s)


def apply_prelim(F: PrelimIBF, g):
    """u = U G^{L-l0-1..h} M (H^h..H^{l0+1})^* (V^0)^* g with the prelim blocks."""
    prob = F.prob
    gl = _leaf_gather(F.xi_idx, _g_sorted(prob, g))               # [b, slot, n]
    lam = np.einsum("abts,bsn->abtn", F.Vs, gl)
    T = prob.tree
    for l in range(T.l0 + 1, T.h + 1):
        lam = _stage(F.H[l], lam)
    lam = np.einsum("abts,absn->abtn", F.M, lam)
    for l in range(T.h + 1, T.L - T.l0 + 1):
        lam = _stage(F.G[l], lam)
    u_leaf = np.einsum("abit,abtn->ain", F.U, lam)
    return _scatter_u(prob, F.x_idx, u_leaf)


def prelim_sparse_factors(F: PrelimIBF):
    """The preliminary factors as explicit sparse matrices in the paper's order.

    First half (V^0, H^l): Lambda^l stacks pair (i, j) at index (j 2^l + i) r + t
    (j-major, Sec. 3 recursion).  The switch matrix M^{L/2} maps it to the
    i-major order (i 2^{L-l} + j) r + t used by G^l and U^L.  Returns the list
    [V0s, H^{l0+1}s, ..., M, G..., U] whose right-to-left product is K_IBF in
    sorted point order.
    """
    prob = F.prob
    T, r = prob.tree, prob.r
    L, l0, h = T.L, T.l0, T.h
    nx, nxi = len(T.xs), len(T.xis)

    def jmajor(l, i, j):
        return (j * (1 << l) + i) * r

    def imajor(l, i, j):
        return (i * (1 << (L - l)) + j) * r

    mats = []
    rows, cols, vals = [], [], []
    na, nb = 1 << l0, T.nleaf
    for i in range(na):
        for j in range(nb):
            for slot in range(F.xi_idx.shape[1]):
                col = F.xi_idx[j, slot]
                if col < 0:
                    continue
                for t in range(r):
                    rows.append(jmajor(l0, i, j) + t)
                    cols.append(col)
                    vals.append(F.Vs[i, j, t, slot])
    mats.append(sp.csr_matrix((vals, (rows, cols)), shape=(T.nleaf * na * r, nxi)))

    def stage_matrix(blk, l, out_idx, in_idx):
        na, nb = 1 << l, 1 << (L - l)
        rows, cols, vals = [], [], []
        for i in range(na):
            for j in range(nb):
                for c in (0, 1):
                    ro = out_idx(l, i, j)
                    ci = in_idx(l - 1, i // 2, 2 * j + c)
                    for t in range(r):
                        for s in range(r):
                            rows.append(ro + t)
                            cols.append(ci + s)
                            vals.append(blk[i, j, c, t, s])
        n = (1 << L) * r
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))

    for l in range(l0 + 1, h + 1):
        mats.append(stage_matrix(F.H[l], l, jmajor, jmajor))
    # switch: i-major out, j-major in, block (pair) diagonal in pair space
    rows, cols, vals = [], [], []
    for i in range(1 << h):
        for j in range(1 << (L - h)):
            for t in range(r):
                for s in range(r):
                    rows.append(imajor(h, i, j) + t)
                    cols.append(jmajor(h, i, j) + s)
                    vals.append(F.M[i, j, t, s])
    n = (1 << L) * r
    mats.append(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)))
    for l in range(h + 1, L - l0 + 1):
        mats.append(stage_matrix(F.G[l], l, imajor, imajor))
    rows, cols, vals = [], [], []
    la = L - l0
    for i in range(T.nleaf):
        for j in range(1 << l0):
            for slot in range(F.x_idx.shape[1]):
                row = F.x_idx[i, slot]
                if row < 0:
                    continue
                for t in range(r):
                    rows.append(row)
                    cols.append(imajor(la, i, j) + t)
                    vals.append(F.U[i, j, slot, t])
    mats.append(sp.csr_matrix((vals, (rows, cols)), shape=(nx, (1 << L) * r)))
    return mats


# ----------------------------------------------------------------------------
# Optimal IBF: sweeping structure-preserving compression (Sec. 4)
# ----------------------------------------------------------------------------

def truncated_svd(Z, tol):
    """Batched SVD Z = U S V^* with per-block rank k = #{s_i > tol s_1}.

    Returns U, S, Vh (full, descending) and k per block.
    """
    U, S, Vh = np.linalg.svd(Z, full_matrices=False)
    s1 = S[..., :1]
    k = np.sum(S > tol * s1, axis=-1)
    k = np.where(s1[..., 0] > 0, k, 0)
    return U, S, Vh, k


def cap_rank(S, k, cap):
    """Fixed-rank mode: per block keep min(k, cap) singular values, where k
    comes from the tolerance rule.  When the cap cuts through a cluster of
    equal singular values (sigma_k' >= (1 - 1e-10) sigma_{k'-1}, 0-based,
    i.e. the first dropped value equals the last kept one) the cut moves
    down until it does not: the kept subspace of a degenerate cluster is not
    unique, so splitting it would make the factorization ill-defined."""
    kk = np.minimum(k, cap)
    S = np.asarray(S)
    while True:
        cut = (kk < k) & (kk > 1)
        first = np.take_along_axis(S, np.clip(kk, 0, S.shape[-1] - 1)[..., None], -1)[..., 0]
        last = np.take_along_axis(S, np.clip(kk - 1, 0, S.shape[-1] - 1)[..., None], -1)[..., 0]
        move = cut & (first >= (1.0 - 1e-10) * last)
        if not move.any():
            return kk
        kk = np.where(move, kk - 1, kk)


def _keep(k, width):
    """Mask [..., width] keeping the first k entries."""
    return (np.arange(width) < k[..., None]).astype(np.float64)


@dataclass
class OptimalIBF:
    prob: IBFProblem
    Vbar: np.ndarray        # [a, b, k, slot]   (R^{l0})^* V^*
    xi_idx: np.ndarray
    F: dict                 # l -> [a, b, c, k_out, k_in], l0 < l <= h
    Mdot: np.ndarray | None  # [a, b, k, k] middle block (identity when None)
    Gbar: dict              # l -> [a, b, c, k_out, k_in], h < l <= L-l0
    Ubar: np.ndarray        # [a, b, slot, k]   U C^{L-l0}
    x_idx: np.ndarray
    ranks: dict             # level -> per-pair rank array [a, b]
    ranks_in: dict | None = None   # sweep-in ranks (level -> ([a,b] G side, [a,b] H side))


def sweep_out(F: PrelimIBF, tol: float, caps=None) -> OptimalIBF:
    """Sweep-out stage of Sec. 4.2: middle SVDs then recursions toward U and V.

    Blocks are kept at width r with exact zero padding beyond each pair's rank.
    `caps` (level -> rank), when given, bounds the rank of every block whose
    basis lives at that level (fixed-rank mode, cap_rank).
    """
    prob = F.prob
    T, r = prob.tree, prob.r
    L, l0, h = T.L, T.l0, T.h
    ranks = {}

    def trunc(Z, level):
        U, S, Vh, k = truncated_svd(Z, tol)
        if caps is not None and level in caps:
            k = cap_rank(S, k, int(caps[level]))
        return U, S, Vh, k

    # Middle level factorisation (eq:KeqUMV, eq:lowrankSVD): M~ = C (R)^*.
    Um, Sm, Vhm, km = trunc(F.M, h)
    keep = _keep(km, r)
    sq = np.sqrt(Sm) * keep
    C = Um * sq[..., None, :]                                        # [a,b,t,k]
    R = np.conj(np.swapaxes(Vhm, -1, -2)) * sq[..., None, :]          # [a,b,s,k]
    ranks[h] = km
    Cl = {h: C}
    Rl = {h: R}

    # Toward U (eqn:GC): W = [G_0 C_{PC0}, G_1 C_{PC1}] = C^{l+1} [Gbar_0, Gbar_1].
    Gbar = {}
    for l in range(h + 1, L - l0 + 1):
        na, nb = 1 << l, 1 << (L - l)
        Cprev = Cl[l - 1]
        par = np.arange(na) // 2
        parts = []
        for c in (0, 1):
            src = Cprev[par][:, 2 * np.arange(nb) + c]                   # [a,b,s,k]
            parts.append(F.G[l][:, :, c] @ src)
        W = np.concatenate(parts, axis=-1)                               # [a,b,r,2r]
        Uw, Sw, Vhw, kw = trunc(W, l)
        keep = _keep(kw, r)
        Cl[l] = Uw[..., :r] * (Sw[..., :r] * keep)[..., None, :]
        Vk = Vhw[..., :r, :] * keep[..., :, None]                        # [a,b,k,2r]
        Gbar[l] = np.stack([Vk[..., :r], Vk[..., r:]], axis=2)           # [a,b,c,k,r]
        ranks[l] = kw

    # Toward V (eqn:HR): per input pair (P,C) at l-1,
    # Z = [H_{A0B<-PC}^* R_{A0B}, H_{A1B<-PC}^* R_{A1B}] = R^{l-1} [Hbar_0, Hbar_1].
    Fh = {}
    for l in range(h, l0, -1):
        na, nb = 1 << l, 1 << (L - l)
        Rcur = Rl[l]
        Hb = F.H[l].reshape(na // 2, 2, nb, 2, r, r)       # [a', alpha, b, c, t, s]
        Rc = Rcur.reshape(na // 2, 2, nb, r, r)            # [a', alpha, b, t, k]
        parts = []
        for alpha in (0, 1):
            # H^*_{(2a'+alpha, b), c} R_{(2a'+alpha, b)} for c = 0,1 -> [a', b, c, s, k]
            Hs = np.conj(np.swapaxes(Hb[:, alpha], -1, -2))              # [a', b, c, s, t]
            parts.append(Hs @ Rc[:, alpha][:, :, None])
        Z = np.concatenate(parts, axis=-1)                               # [a', b, c, r, 2r]
        Z = Z.reshape(na // 2, 2 * nb, r, 2 * r)                         # input pair (a', 2b+c)
        Uz, Sz, Vhz, kz = trunc(Z, l - 1)
        keep = _keep(kz, r)
        Rl[l - 1] = Uz[..., :r] * (Sz[..., :r] * keep)[..., None, :]
        Vk = np.conj(np.swapaxes(Vhz[..., :r, :], -1, -2)) * keep[..., None, :]   # [a', j, 2r, k]
        Vk = Vk.reshape(na // 2, nb, 2, 2 * r, r)                         # [a', b, c, 2r, k]
        blk = np.empty((na, nb, 2, r, r), dtype=np.complex128)
        for alpha in (0, 1):
            blk[alpha::2] = Vk[:, :, :, alpha * r:(alpha + 1) * r, :]
        Fh[l] = blk
        ranks[l - 1] = kz

    Vbar = np.conj(np.swapaxes(Rl[l0], -1, -2)) @ F.Vs              # eqn:V0
    Ubar = F.U @ Cl[L - l0]                                          # U^L C^L
    return OptimalIBF(prob, Vbar, F.xi_idx, Fh, None, Gbar, Ubar, F.x_idx,
                      ranks)


def sweep_in(O: OptimalIBF, tol: float) -> OptimalIBF:
    """Sweep-in stage of Sec. 4.3, from the outer factors to the middle.

    U side: Ubar ~= Udot Cbar (Udot = U_k, Cbar = S_k V_k^*), then per input
    pair [Cbar_{A0B} Gbar_{A0B<-PC}; Cbar_{A1B} Gbar_{A1B<-PC}] ~= [Gdot_0; Gdot_1]
    Cbar_{PC}.  V side mirrored: Vbar^* ~= Rbar^* Vdot^* and per output pair
    [F_{AB<-PC0} Rbar^*_{PC0}, F_{AB<-PC1} Rbar^*_{PC1}] ~= Rbar^*_{AB} [Fdot_0, Fdot_1].
    Finally Mdot = Cbar^h Rbar^{h*} per middle pair.
    """
    prob = O.prob
    T, r = prob.tree, prob.r
    L, l0, h = T.L, T.l0, T.h
    la = L - l0
    ranks_g, ranks_h = {}, {}

    # U side.  Ubar[a,b] is [slot, k]; SVD per pair.
    Uu, Su, Vhu, ku = truncated_svd(O.Ubar, tol)        # Uu [a,b,slot,m], m=min(slot,r)
    m = Su.shape[-1]
    keep = _keep(ku, m)
    Udot = Uu * keep[..., None, :]
    Cbar = (Su * keep)[..., :, None] * Vhu                # [a,b,m,r]
    # pad the rank axis to width r
    if m < r:
        Udot = np.concatenate([Udot, np.zeros(Udot.shape[:-1] + (r - m,))], axis=-1)
        Cbar = np.concatenate([Cbar, np.zeros(Cbar.shape[:-2] + (r - m, r))], axis=-2)
    else:
        Udot, Cbar = Udot[..., :r], Cbar[..., :r, :]
    ranks_g[la] = ku
    Gdot = {}
    for l in range(la, h, -1):
        # stage (l-1 -> l); input pairs at l-1: (a', j = 2b + c)
        na, nb = 1 << l, 1 << (L - l)
        Gb = O.Gbar[l].reshape(na // 2, 2, nb, 2, r, r)     # [a', alpha, b, c, k_out, k_in]
        Cb = Cbar.reshape(na // 2, 2, nb, r, r)              # [a', alpha, b, m, k_out]
        parts = [Cb[:, alpha][:, :, None] @ Gb[:, alpha] for alpha in (0, 1)]   # [a', b, c, m, k_in]
        Y = np.concatenate(parts, axis=-2).reshape(na // 2, 2 * nb, 2 * r, r)
        Uy, Sy, Vhy, ky = truncated_svd(Y, tol)
        keep = _keep(ky, r)
        Cbar = (Sy[..., :r] * keep)[..., :, None] * Vhy[..., :r, :]          # [a', j, m, k_in]
        Uk = Uy[..., :, :r] * keep[..., None, :]                              # [a', j, 2r, m]
        Uk = Uk.reshape(na // 2, nb, 2, 2 * r, r)
        blk = np.empty((na, nb, 2, r, r), dtype=np.complex128)
        for alpha in (0, 1):
            blk[alpha::2] = Uk[:, :, :, alpha * r:(alpha + 1) * r, :]
        Gdot[l] = blk
        ranks_g[l - 1] = ky

    # V side.  Vbar[a,b] is [k, slot] = Rbar^* Vdot^* with Rbar^* = P S, Vdot^* = Q^*.
    Pv, Sv, Qhv, kv = truncated_svd(O.Vbar, tol)           # Pv [a,b,k,m]
    m = Sv.shape[-1]
    keep = _keep(kv, m)
    Rbs = Pv * (Sv * keep)[..., None, :]                   # Rbar^* [a,b,k,m]
    Vdot = Qhv * keep[..., :, None]                        # [a,b,m,slot]
    if m < r:
        Rbs = np.concatenate([Rbs, np.zeros(Rbs.shape[:-1] + (r - m,))], axis=-1)
        Vdot = np.concatenate([Vdot, np.zeros(Vdot.shape[:-2] + (r - m, Vdot.shape[-1]))], axis=-2)
    else:
        Rbs, Vdot = Rbs[..., :r], Vdot[..., :r, :]
    ranks_h[l0] = kv
    Fdot = {}
    for l in range(l0 + 1, h + 1):
        na, nb = 1 << l, 1 << (L - l)
        par = np.arange(na) // 2
        parts = []
        for c in (0, 1):
            src = Rbs[par][:, 2 * np.arange(nb) + c]                  # [a,b,k_in,m]
            parts.append(O.F[l][:, :, c] @ src)                       # [a,b,k_out,m]
        Y = np.concatenate(parts, axis=-1)                            # [a,b,r,2r]
        Uy, Sy, Vhy, ky = truncated_svd(Y, tol)
        keep = _keep(ky, r)
        Rbs = Uy[..., :r] * (Sy[..., :r] * keep)[..., None, :]
        Vk = Vhy[..., :r, :] * keep[..., :, None]
        Fdot[l] = np.stack([Vk[..., :r], Vk[..., r:]], axis=2)
        ranks_h[l] = ky

    Mdot = Cbar @ Rbs                                                 # [a,b,m_G,m_H]
    ranks = dict(O.ranks)
    return OptimalIBF(prob, Vdot, O.xi_idx, Fdot, Mdot, Gdot, Udot, O.x_idx,
                      ranks, {"G": ranks_g, "H": ranks_h})


def apply_optimal(O: OptimalIBF, g):
    """u = Ubar Gbar... [Mdot] F... Vbar^* g (Sec. 4, eqn:IBFout / eqn:IBFin)."""
    prob = O.prob
    T = prob.tree
    gl = _leaf_gather(O.xi_idx, _g_sorted(prob, g))
    mu = np.einsum("abks,bsn->abkn", O.Vbar, gl)
    for l in range(T.l0 + 1, T.h + 1):
        mu = _stage(O.F[l], mu)
    if O.Mdot is not None:
        mu = np.einsum("abts,absn->abtn", O.Mdot, mu)
    for l in range(T.h + 1, T.L - T.l0 + 1):
        mu = _stage(O.Gbar[l], mu)
    u_leaf = np.einsum("abik,abkn->ain", O.Ubar, mu)
    return _scatter_u(prob, O.x_idx, u_leaf)


def _stage_adjoint(blk, out):
    """Conjugate transpose of _stage: lam[a', 2b+c] = sum_d blk[2a'+d, b, c]^H out[2a'+d, b]."""
    na, nb, kin = blk.shape[0], blk.shape[1], blk.shape[4]
    lam = np.zeros((na // 2, 2 * nb, kin, out.shape[-1]), dtype=np.complex128)
    for c in (0, 1):
        contrib = np.einsum("abts,abtn->absn", blk[:, :, c].conj(), out)
        lam[:, c::2] = contrib[0::2] + contrib[1::2]
    return lam


def apply_optimal_adjoint(O: OptimalIBF, h):
    """v = (IBF)^* h: the factors of apply_optimal conjugate-transposed in
    reverse order (Ubar^*, Gbar^*, Mdot^*, F^*, Vbar); h has one entry per
    row point x, v one per column point xi (the type-I orientation of the
    non-uniform DFT of Sec. 6.1)."""
    prob = O.prob
    T = prob.tree
    h = np.asarray(h, dtype=np.complex128)
    if h.ndim == 1:
        h = h[:, None]
    hl = _leaf_gather(O.x_idx, h[T.perm_x])                     # [a, slot, n]
    mu = np.einsum("abik,ain->abkn", O.Ubar.conj(), hl)
    for l in range(T.L - T.l0, T.h, -1):
        mu = _stage_adjoint(O.Gbar[l], mu)
    if O.Mdot is not None:
        mu = np.einsum("abts,abtn->absn", O.Mdot.conj(), mu)
    for l in range(T.h, T.l0, -1):
        mu = _stage_adjoint(O.F[l], mu)
    v_leaf = np.einsum("abks,abkn->bsn", O.Vbar.conj(), mu)    # [b, slot, n]
    v_s = np.zeros((len(T.xis), v_leaf.shape[-1]), dtype=np.complex128)
    ok = O.xi_idx >= 0
    v_s[O.xi_idx[ok]] = v_leaf[ok]
    v = np.empty_like(v_s)
    v[T.perm_xi] = v_s
    return v


# ----------------------------------------------------------------------------
# Sizes, ranks and error metrics (Sec. 6)
# ----------------------------------------------------------------------------

def level_ranks(O: OptimalIBF):
    """Per-level maximum rank of the sweep-out bases, levels l0..L-l0."""
    return {l: int(np.max(k)) for l, k in sorted(O.ranks.items())}


def nnz_prelim(prob: IBFProblem):
    """Non-zeros of the preliminary IBF (memory numerator of eq:compratio)."""
    T, r = prob.tree, prob.r
    L, l0, h = T.L, T.l0, T.h
    npairs = 1 << L
    nv = len(T.xis) * (1 << l0) * r
    nu = len(T.xs) * (1 << l0) * r
    nstages = (h - l0) + (L - l0 - h)
    return nv + nu + nstages * npairs * 2 * r * r + npairs * r * r


def nnz_optimal(O: OptimalIBF):
    """Non-zeros of the compressed factors, each block at its own rank."""
    prob = O.prob
    T = prob.tree
    L, l0, h = T.L, T.l0, T.h
    rk = O.ranks
    xcnt = np.diff(T.xoff)
    xicnt = np.diff(T.xioff)
    tot = int(np.sum(rk[l0] * xicnt[None, :]))                 # Vbar: k x |B|
    tot += int(np.sum(rk[L - l0] * xcnt[:, None]))             # Ubar: |A| x k
    tot += int(np.sum(rk[h]))                                  # Mbar diagonal
    for l in list(range(l0 + 1, h + 1)) + list(range(h + 1, L - l0 + 1)):
        na, nb = 1 << l, 1 << (L - l)
        kin = rk[l - 1]
        kin_sum = kin[np.arange(na) // 2][:, 2 * np.arange(nb)] + \
            kin[np.arange(na) // 2][:, 2 * np.arange(nb) + 1]
        tot += int(np.sum(rk[l] * kin_sum))
    return tot


def nnz_optimal_in(O: OptimalIBF):
    """Non-zeros of the swept-in factors (eqn:IBFin), each block at its own rank."""
    T = O.prob.tree
    L, l0, h = T.L, T.l0, T.h
    rg, rh = O.ranks_in["G"], O.ranks_in["H"]
    xcnt = np.diff(T.xoff)
    xicnt = np.diff(T.xioff)
    tot = int(np.sum(rh[l0] * xicnt[None, :]))
    tot += int(np.sum(rg[L - l0] * xcnt[:, None]))
    tot += int(np.sum(rg[h] * rh[h]))
    for l in range(l0 + 1, L - l0 + 1):
        rk = rh if l <= h else rg
        na, nb = 1 << l, 1 << (L - l)
        kin = rk[l - 1]
        kin_sum = kin[np.arange(na) // 2][:, 2 * np.arange(nb)] + \
            kin[np.arange(na) // 2][:, 2 * np.arange(nb) + 1]
        tot += int(np.sum(rk[l] * kin_sum))
    return tot


def rel_error(u, u_ref):
    """eq:relativeerr over the given rows (Frobenius over all columns)."""
    u = np.asarray(u)
    u_ref = np.asarray(u_ref)
    return float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))


def rel_error_cols(u, u_ref):
    """eq:relativeerr per right-hand side (column); returns the largest."""
    u = np.asarray(u).reshape(len(u), -1)
    u_ref = np.asarray(u_ref).reshape(len(u_ref), -1)
    return float(np.max(np.linalg.norm(u - u_ref, axis=0) / np.linalg.norm(u_ref, axis=0)))


def build_optimal(kind, params, x, xi, r, tol, leaf=16, sweep_in_on=False,
                  lo=None, W=None, amp=None, caps=None):
    """Convenience: geometry, preliminary factors, sweep-out [, sweep-in]."""
    prob = make_problem(kind, params, x, xi, r, leaf, lo, W, amp)
    F = prelim_factors(prob)
    O = sweep_out(F, tol, caps)
    if sweep_in_on:
        O = sweep_in(O, tol)
    return prob, F, O
