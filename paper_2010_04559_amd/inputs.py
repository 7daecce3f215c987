"""Seeded synthetic problem definitions.

This module only describes problems: mesh sizes, angular-mesh recipes,
per-cell cross sections drawn from seeded generators, source, inflow and
detector boxes, solver options.  It holds none of the method's arithmetic
(no quadrature, no operators, no right-hand sides), so that both the HIP
library and the CPU oracle consume the same inputs without sharing code.

The paper's own experiments use a Gmsh cube that is not available; every
workload here is a structured Cartesian cube or square with cross sections
from the recipes below (the recipes are listed in the design notes).
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class AngularSpec:
    """Uniform refinement to ``base_level``; optionally ``extra_levels`` more
    inside a cone of ``cone_half_angle_deg`` around ``cone_axis`` with the
    two-irregularity closure; or (band_lmax > 0) the z-band rule of the
    paper's pencil-beam study (levels band_lmax .. band_lmax - 4).
    ``basis``: the angular basis of Section 2.2, "lin" (three functions per
    patch) or "const" (one)."""
    base_level: int = 1
    cone_axis: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    cone_half_angle_deg: float = 0.0
    extra_levels: int = 0
    closure: bool = True
    band_lmax: int = 0
    basis: str = "lin"

    @property
    def n_levels(self):
        return (self.band_lmax if self.band_lmax > 0 else self.base_level + self.extra_levels) + 1


@dataclass
class Inflow:
    """Boundary data on face (axis, side): kind 'iso' (isotropic value) or
    'beam' (unit current per area along ``direction``).  ``lo``/``hi`` bound
    the cell indices on the face (the face axis itself is ignored)."""
    kind: str = "iso"
    axis: int = 0
    side: int = 0
    lo: Tuple[int, int, int] = (0, 0, 0)
    hi: Tuple[int, int, int] = (10 ** 6, 10 ** 6, 10 ** 6)
    value: float = 1.0
    direction: Tuple[float, float, float] = (1.0, 0.0, 0.0)


@dataclass
class Problem:
    name: str
    dim: int
    n: Tuple[int, int, int]
    angular: AngularSpec
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    hg_g: float
    order: int                       # outer (full) Legendre order L
    mg_orders: List[int]             # per angular level T_0 .. T_L (coarsest first)
    q_cell: np.ndarray               # isotropic volume source per cell (per steradian)
    inflow: Optional[Inflow] = None
    detector: Optional[Tuple[Tuple[int, int, int], Tuple[int, int, int]]] = None
    restart: int = 10
    tol: float = 1e-8
    nu_pre: int = 1
    nu_post: int = 1
    nu_coarse: int = 10
    nu_post_coarse: int = 0          # post-smoothing below the finest level (0: nu_post)
    # Gauss-Seidel octant order on T_0 (octant id = [s_x<0] + 2[s_y<0] +
    # 4[s_z<0]).  The method leaves it open; the default is the reflected
    # Gray code, so consecutive octants (and the last and first) differ in
    # one sign and each octant's sweep starts at a corner next to the
    # previous one's start.
    octant_order: Tuple[int, ...] = (0, 1, 3, 2, 6, 7, 5, 4)
    length: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    fd_cells: Optional[np.ndarray] = None
    extras: dict = field(default_factory=dict)
    # Fokker-Planck-equivalent moments of order fp_N instead of HG (the
    # paper's Section 5 workloads): sigma_{s,n} / sigma_{s,0} = 1 - n (n+1) /
    # (N (N+1)) for n <= N, zero beyond
    fp_N: Optional[int] = None

    @property
    def cells(self):
        return int(np.prod(self.n[:self.dim]))

    def moments(self, order=None):
        """Normalised Legendre coefficients f_n (sigma_{s,n} = sigma_s f_n),
        n <= order: HG f_n = g^n (plain truncation), or the
        Fokker-Planck-equivalent ratios when fp_N is set."""
        L = self.order if order is None else order
        if self.fp_N is not None:
            N = self.fp_N
            return np.array([1.0 - k * (k + 1) / (N * (N + 1)) if k <= N else 0.0 for k in range(L + 1)])
        return np.array([self.hg_g ** k for k in range(L + 1)], dtype=np.float64)

    def with_sigma(self, sigma_t, sigma_s):
        return replace(self, sigma_t=np.asarray(sigma_t, float), sigma_s=np.asarray(sigma_s, float))


def lognormal_sigma(ncells, median, log_sd, seed):
    """sigma_t,j = median * exp(log_sd * z_j), z = standard normals from
    ``numpy.random.default_rng(seed)`` in cell order j = ix + nx (iy + ny iz)."""
    z = np.random.default_rng(seed).standard_normal(ncells)
    return median * np.exp(log_sd * z)


def checkerboard_mask(n, block):
    """1 where the block parity (bx + by + bz) mod 2 is even, else 0."""
    nx, ny, nz = n
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    par = (ix // block + iy // block + iz // block) % 2
    return (par == 0).ravel().astype(np.float64)


def box_mask(n, dim, lo, hi):
    nx, ny, nz = (tuple(n) + (1, 1))[:3]
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = [ix.ravel(), iy.ravel(), iz.ravel()]
    ok = np.ones(nx * ny * nz, dtype=bool)
    for a in range(dim):
        ok &= (c[a] >= lo[a]) & (c[a] <= hi[a])
    return ok.astype(np.float64)


def central_box(n):
    """Cells [n/2-2, n/2+1] on each axis (a 4-cell-wide central box)."""
    return tuple(k // 2 - 2 for k in n), tuple(k // 2 + 1 for k in n)


def fd_cells(ncells, seed, count=20):
    return np.random.default_rng(seed + 1).choice(ncells, count, replace=False)


# ------------------------------------------------------------------ configs

def config1():
    """2-D unit square, 16x16 cells, angular level 1 (32 patches), HG g=0.9
    at L=8, sigma_t=10, c=0.99, isotropic unit inflow on x=0, GMRES(20)."""
    n = (16, 16, 1)
    C = 256
    st = np.full(C, 10.0)
    return Problem("cfg1-2d-16x16-ang1-L8", 2, n, AngularSpec(1), st, 0.99 * st, 0.9, 8,
                   [8, 8], np.zeros(C), Inflow("iso", 0, 0, value=1.0), restart=20)


def config2(n=32):
    """3-D unit cube, 32^3 cells, angular level 2 (128 patches), HG g=0.95 at
    L=16, lognormal sigma_t (median 5, log-sd 1.0, seed 0), c=0.98, unit
    source in the central 4^3 box, vacuum, GMRES(10)."""
    nn = (n, n, n)
    C = n ** 3
    st = lognormal_sigma(C, 5.0, 1.0, 0)
    lo, hi = central_box(nn)
    return Problem(f"cfg2-3d-{n}^3-ang2-L16", 3, nn, AngularSpec(2), st, 0.98 * st, 0.95, 16,
                   [16, 16, 16], box_mask(nn, 3, lo, hi), None)


# V-cycle of the 48^3 precision problem's timed solves (pre-smoothing
# sweeps, post-smoothing sweeps on the finest level, coarsest-level
# Gauss-Seidel sweeps, post-smoothing sweeps on the levels between), chosen
# by measuring time to 1e-8 over cycle shapes: V(1,1) with 10 coarse sweeps
# takes 10 flexible-GMRES iterations, this cycle 4 at 60% of the time.
# config3() itself keeps V(1,1) and 10 (its oracle reference).
CFG3_CYCLE = (1, 6, 5, 1)


def config3(n=48):
    """3-D cube, 48^3 cells, angular level 3 (512 patches), HG g=0.98 at
    L=32, coarse MG levels at L=8, checkerboard of 8^3 blocks
    (sigma_t 1 / 20, c 0.999 / 0.9), central unit source, vacuum."""
    nn = (n, n, n)
    m = checkerboard_mask(nn, 8)
    st = np.where(m > 0, 1.0, 20.0)
    c = np.where(m > 0, 0.999, 0.9)
    lo, hi = central_box(nn)
    return Problem(f"cfg3-3d-{n}^3-ang3-L32", 3, nn, AngularSpec(3), st, c * st, 0.98, 32,
                   [8, 8, 8, 32], box_mask(nn, 3, lo, hi), None)


def config4(n=32):
    """3-D cube, 32^3, angular level 2, HG g=0.95 at L=16, lognormal sigma_t
    (median 5, log-sd 0.5, seed 1), c=0.95, unit beam along +x on a 4x4
    patch of x=0, detector box of 4^3 cells at the far side."""
    nn = (n, n, n)
    C = n ** 3
    st = lognormal_sigma(C, 5.0, 0.5, 1)
    lo = (0, n // 2 - 2, n // 2 - 2)
    hi = (0, n // 2 + 1, n // 2 + 1)
    det = ((n - 4, n // 2 - 2, n // 2 - 2), (n - 1, n // 2 + 1, n // 2 + 1))
    return Problem(f"cfg4-3d-{n}^3-ang2-L16-beam", 3, nn, AngularSpec(2), st, 0.95 * st, 0.95, 16,
                   [16, 16, 16], np.zeros(C), Inflow("beam", 0, 0, lo, hi, 1.0, (1.0, 0.0, 0.0)),
                   detector=det, fd_cells=fd_cells(C, 1))


def config5(n=32):
    """3-D cube, 32^3, angular level 2 plus 3 levels in a 15-degree cone
    around +x (two-irregular), HG g=0.99 at L=64, MG orders 16 then 4,
    lognormal sigma_t (median 10, log-sd 0.7, seed 2), c=0.99, beam as in
    the differentiation config, detector at the far side."""
    nn = (n, n, n)
    C = n ** 3
    st = lognormal_sigma(C, 10.0, 0.7, 2)
    lo = (0, n // 2 - 2, n // 2 - 2)
    hi = (0, n // 2 + 1, n // 2 + 1)
    det = ((n - 4, n // 2 - 2, n // 2 - 2), (n - 1, n // 2 + 1, n // 2 + 1))
    return Problem(f"cfg5-3d-{n}^3-cone-L64", 3, nn, AngularSpec(2, (1.0, 0.0, 0.0), 15.0, 3, True),
                   st, 0.99 * st, 0.99, 64, [4, 4, 4, 16, 16, 16], np.zeros(C),
                   Inflow("beam", 0, 0, lo, hi, 1.0, (1.0, 0.0, 0.0)), detector=det,
                   fd_cells=fd_cells(C, 2))


def small_problem(dim=2, n=4, level=1, g=0.8, order=4, c=0.9, seed=0, inflow=True, source=True,
                  mg_orders=None, restart=10, angular=None):
    """Small random heterogeneous problem for parity tests (n: cells per
    axis, or a tuple of per-axis counts; angular: an AngularSpec replacing
    the uniform mesh of ``level`` refinements, whose level count then sets
    the length of mg_orders)."""
    if isinstance(n, (tuple, list)):
        nn = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        n = "x".join(str(v) for v in n)
    else:
        nn = (n, n, n if dim == 3 else 1)
    C = int(np.prod(nn[:dim]))
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 4.0, C)
    ss = c * st * rng.uniform(0.8, 1.0, C)
    q = rng.uniform(0.0, 1.0, C) if source else np.zeros(C)
    spec = angular if angular is not None else AngularSpec(level)
    nlev = spec.n_levels
    mg = mg_orders if mg_orders is not None else [order] * nlev
    tag = (f"ang{level}" if angular is None else f"band{spec.band_lmax}" if spec.band_lmax
           else f"cone{spec.base_level}+{spec.extra_levels}" if spec.extra_levels else f"ang{spec.base_level}")
    if spec.basis != "lin":
        tag += "-" + spec.basis
    return Problem(f"small-{dim}d-{n}-{tag}-L{order}-s{seed}", dim, nn, spec,
                   st, ss, g, order, mg, q, Inflow("iso", 0, 0, value=1.0) if inflow else None,
                   restart=restart)


# ------------------------------------------------------ the paper's workloads

def paper_box(N, level=3, nr=None, n=30, nu_pre=1, nu_post=1, beam=False, band_lmax=0, restart=20,
              nr_levels="all", nu_coarse=10, basis="lin"):
    """The cube of the paper's Section 5 experiments: 5 x 5 x 5 cm, n^3
    hexahedra (30^3 in the paper), vacuum boundaries, Fokker-Planck-
    equivalent scatter moments of order N with transport cross section 1
    (alpha = 1: sigma_{s,0} = N (N + 1) / 2), no absorption (sigma_t =
    sigma_{s,0}, a reading: the paper gives only the transport cross
    section).  Volume-source study (Sections 5.1-5.4): a uniform isotropic
    unit source in the whole cube, uniform angular level ``level``.  Pencil
    beam (Section 5.5, ``beam``): no volume source, a unit beam along +z on
    the z = 0 face over 2 < x, y < 3 cm, angular mesh by the z-band rule with
    ``band_lmax``.  Multigrid scatter orders: ``nr`` (default N) on every
    preconditioner level (``nr_levels="all"``, Sections 5.3-5.5) or on the
    coarsest level only with N elsewhere (``"coarsest"``, the Section 5.1
    study); the problem operator keeps order N.  ``nu_coarse`` Gauss-Seidel
    sweeps on the coarsest level (10 in Sections 5.3-5.5).  ``basis``: the
    angular basis, "lin" or "const" (both studied in Section 5)."""
    nn = (n, n, n)
    C = n ** 3
    sig = 0.5 * N * (N + 1)
    st = np.full(C, sig)
    spec = AngularSpec(level, basis=basis) if not band_lmax else AngularSpec(0, band_lmax=band_lmax, basis=basis)
    nlev = spec.n_levels
    nr = N if nr is None else nr
    if nr_levels == "all":
        mg = [nr] * nlev
    elif nr_levels == "coarsest":
        mg = [nr] + [N] * (nlev - 1)
    else:
        raise ValueError("nr_levels is 'all' or 'coarsest'")
    name = "paper-box-%d^3-N%d-%s-nr%d%s-V%d%d-gs%d-%s" % (
        n, N, ("band%d" % band_lmax) if band_lmax else ("lev%d" % level), nr, "c" if nr_levels == "coarsest" else "",
        nu_pre, nu_post, nu_coarse, basis)
    inflow = None
    q = np.ones(C)
    if beam:
        # cells whose centres lie in 2 < x, y < 3 cm (exactly the band for n = 30)
        h = 5.0 / n
        cen = (np.arange(n) + 0.5) * h
        inside = np.nonzero((cen > 2.0) & (cen < 3.0))[0]
        lo_c, hi_c = int(inside[0]), int(inside[-1])
        inflow = Inflow("beam", 2, 0, (lo_c, lo_c, 0), (hi_c, hi_c, 0), 1.0, (0.0, 0.0, 1.0))
        q = np.zeros(C)
        name += "-zbeam"
    return Problem(name, 3, nn, spec, st, st.copy(), 0.0, N, mg, q, inflow, restart=restart, nu_pre=nu_pre,
                   nu_post=nu_post, nu_coarse=nu_coarse, length=(5.0, 5.0, 5.0), fp_N=N)
