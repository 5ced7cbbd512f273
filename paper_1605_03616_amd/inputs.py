"""Seeded synthetic inputs for the IBF workloads.

This module holds point sets, input vectors and workload descriptions only:
no step of the factorization or of its application lives here.  Both the
oracle-side tests and the HIP path receive the arrays produced here, so the
two implementations never share arithmetic.

Workload shapes follow the paper's numerical section: uniform grids
x_i = i/N, xi_j = j - N/2 for the 1-D FIO (Sec. 6.2, Table 3), i.i.d.
uniform random x in [0,1) for the non-uniform DFT (Sec. 6.1, Table 1), and
a uniform 2-D grid for the 2-D FIO (Sec. 6.3, Table 4).  Input vectors are
"randomly generated" in the paper; here they are complex standard normal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Phase-function identifiers shared by the C-ABI and every caller.
PHASE_DFT = 0        # Phi = s * x . xi                       (Sec. 6.1)
PHASE_FIO1D = 1      # Phi = x xi + c(x)|xi|, c = (p0 + p1 sin 2 pi x)/p2   (Sec. 6.2)
PHASE_FIO2D = 2      # Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2)           (Sec. 6.3)
PHASE_SEPARABLE = 3  # Phi = p0 x + p1 xi: R^{AB} == 0, exact factorization (Sec. 2.1)

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X2 = 2

DEFAULT_PARAMS = {
    PHASE_DFT: (1.0,),
    PHASE_FIO1D: (2.0, 1.0, 8.0),
    PHASE_FIO2D: (2.0, 1.0, 16.0),
    PHASE_SEPARABLE: (3.0, 0.3125),
}


def complex_normal(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """(n, nrhs) complex128 with i.i.d. CN(0,1) entries.

    The real block of shape (n, nrhs) is drawn first, then the imaginary
    block, each standard normal, and the sum is scaled by 1/sqrt(2).
    """
    re = rng.standard_normal((n, nrhs))
    im = rng.standard_normal((n, nrhs))
    return (re + 1j * im) / math.sqrt(2.0)


def uniform_x(n: int) -> np.ndarray:
    """x_i = i/n, i = 0..n-1 (the paper's uniform grid in [0,1))."""
    return np.arange(n, dtype=np.float64) / n


def uniform_xi(n: int) -> np.ndarray:
    """xi_j = j - n/2, j = 0..n-1 (integer frequencies in [-n/2, n/2))."""
    return np.arange(n, dtype=np.float64) - (n // 2)


@dataclass
class Problem1D:
    """A 1-D workload: points, phase, IBF knobs and right-hand sides."""
    name: str
    x: np.ndarray
    xi: np.ndarray
    phase: int
    params: tuple
    r: int
    tol: float
    leaf: int
    nrhs: int
    g: np.ndarray
    precision: int
    sweep_in: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xi.shape[0])


def fio1d_uniform(n: int, r: int, nrhs: int, seed: int, tol: float = 1e-6,
                  leaf: int = 16, precision: int = PREC_FP64,
                  name: str | None = None) -> Problem1D:
    """1-D FIO on uniform grids (paper Sec. 6.2): c(x) = (2 + sin 2 pi x)/8."""
    rng = np.random.default_rng(seed)
    g = complex_normal(n, nrhs, rng)
    return Problem1D(name or f"fio1d_n{n}_r{r}", uniform_x(n), uniform_xi(n),
                     PHASE_FIO1D, DEFAULT_PARAMS[PHASE_FIO1D], r, tol, leaf,
                     nrhs, g, precision)


def nudft_random(n: int, r: int, nrhs: int, seed: int, tol: float = 1e-6,
                 leaf: int = 16, precision: int = PREC_FP32,
                 sweep_in: int = 1, name: str | None = None) -> Problem1D:
    """Non-uniform DFT shape (paper Sec. 6.1): x i.i.d. U[0,1), xi_j = j - n/2.

    One generator seeded with `seed` draws x first (rng.random(n)) and then
    the right-hand sides.
    """
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    g = complex_normal(n, nrhs, rng)
    return Problem1D(name or f"nudft_n{n}_r{r}", x, uniform_xi(n), PHASE_DFT,
                     DEFAULT_PARAMS[PHASE_DFT], r, tol, leaf, nrhs, g,
                     precision, sweep_in)


def dft_uniform(n: int, r: int, nrhs: int, seed: int, tol: float = 1e-6,
                leaf: int = 16, precision: int = PREC_FP64) -> Problem1D:
    """Uniform DFT: x_i = i/n, xi_j = j - n/2, Phi = x xi."""
    rng = np.random.default_rng(seed)
    g = complex_normal(n, nrhs, rng)
    return Problem1D(f"dft_n{n}_r{r}", uniform_x(n), uniform_xi(n), PHASE_DFT,
                     DEFAULT_PARAMS[PHASE_DFT], r, tol, leaf, nrhs, g,
                     precision)


def separable_uniform(n: int, r: int, nrhs: int, seed: int, tol: float = 1e-6,
                      leaf: int = 16, precision: int = PREC_FP64) -> Problem1D:
    rng = np.random.default_rng(seed)
    g = complex_normal(n, nrhs, rng)
    return Problem1D(f"sep_n{n}_r{r}", uniform_x(n), uniform_xi(n),
                     PHASE_SEPARABLE, DEFAULT_PARAMS[PHASE_SEPARABLE], r, tol,
                     leaf, nrhs, g, precision)


# --- the five named workloads ------------------------------------------------

def workload_fio1d_1k() -> Problem1D:
    """Plain FP64 IBF, 1-D FIO N=1024, r=8, leaf 16, one RHS from seed 0."""
    return fio1d_uniform(1024, 8, 1, 0, tol=1e-6, precision=PREC_FP64,
                         name="fio1d_n1024_r8_fp64")


def workload_fio1d_64k(nrhs: int = 64) -> Problem1D:
    """1-D FIO N=65536, r=12, 64 RHS from seed 1, FP32 factors and apply."""
    return fio1d_uniform(65536, 12, nrhs, 1, tol=1e-6, precision=PREC_FP32,
                         name="fio1d_n65536_r12_fp32")


def workload_nudft_1m(n: int = 1 << 20, nrhs: int = 16,
                      precision: int = PREC_BF16X2) -> Problem1D:
    """Non-uniform DFT N=2^20 (x from seed 2), r=10, 16 RHS."""
    return nudft_random(n, 10, nrhs, 2, tol=1e-6, precision=precision,
                        sweep_in=1, name=f"nudft_n{n}_r10")


def batched_sizes(count: int = 256, seed: int = 3, lo: float = 10.0, hi: float = 16.0):
    """Uneven batch: N = round(2^U), U ~ U(lo,hi), bumped to even; nrhs in 1..8.

    Draw order: U = rng.uniform(lo, hi, count), then nrhs = rng.integers(1, 9, count).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(lo, hi, count)
    nrhs = rng.integers(1, 9, count)
    ns = np.round(2.0 ** u).astype(np.int64)
    ns = ns + (ns % 2)
    return ns, nrhs


def error_rows(n: int, count: int = 256, seed: int = 1234) -> np.ndarray:
    """Row sample S for the sampled relative error (paper eq. relativeerr)."""
    if n <= count:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=count, replace=False))


def workload_batched(count: int = 256, seed: int = 3, r: int = 12, lo: float = 10.0,
                     hi: float = 16.0, precision: int = PREC_FP32) -> list:
    """Uneven batch of independent 1-D FIO problems (uniform grids, phase as in
    workload_fio1d_1k): sizes and RHS counts from batched_sizes(count, seed, lo,
    hi); problem i draws its right-hand sides from default_rng(seed * 1000 + i)."""
    ns, nrhs = batched_sizes(count, seed, lo, hi)
    out = []
    for i, (n, k) in enumerate(zip(ns.tolist(), nrhs.tolist())):
        rng = np.random.default_rng(seed * 1000 + i)
        g = complex_normal(n, k, rng)
        out.append(Problem1D(f"batch{i}_fio1d_n{n}_r{r}", uniform_x(n), uniform_xi(n),
                             PHASE_FIO1D, DEFAULT_PARAMS[PHASE_FIO1D], r, 1e-6, 16, k, g,
                             precision))
    return out


def grid_x_2d(n: int) -> np.ndarray:
    """x = (i1, i2) / n on the n x n grid of [0,1)^2, row-major in (i1, i2)."""
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([i1.ravel() / n, i2.ravel() / n], axis=-1).astype(np.float64)


def grid_xi_2d(n: int) -> np.ndarray:
    """xi = (j1, j2) - n/2 on the integer grid [-n/2, n/2)^2, row-major."""
    j1, j2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([j1.ravel() - n // 2, j2.ravel() - n // 2], axis=-1).astype(np.float64)


def fio2d_grid(n: int, r: int, nrhs: int, seed: int, tol: float = 1e-4, leaf: int = 16,
               precision: int = PREC_FP32, name: str | None = None) -> Problem1D:
    """2-D FIO of Sec. 6.3 on the n x n grid (N = n^2 points), c1, c2 with /16,
    tensor order r x r, right-hand sides from default_rng(seed); Omega is the
    square of side n centred at the origin (the MIBF domain)."""
    rng = np.random.default_rng(seed)
    g = complex_normal(n * n, nrhs, rng)
    return Problem1D(name or f"fio2d_n{n}x{n}_r{r}", grid_x_2d(n), grid_xi_2d(n), PHASE_FIO2D,
                     DEFAULT_PARAMS[PHASE_FIO2D], r, tol, leaf, nrhs, g, precision,
                     extra={"omega_width": float(n)})


def workload_fio2d_256(nrhs: int = 8) -> Problem1D:
    """2-D FIO on the 256 x 256 grid, r = 5 x 5, tol 1e-4, 8 RHS from seed 3, FP32."""
    return fio2d_grid(256, 5, nrhs, 3, tol=1e-4, precision=PREC_FP32,
                      name="fio2d_n256x256_r5_fp32")
