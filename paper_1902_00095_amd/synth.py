"""Seeded synthetic workloads for the coupled pressure-temperature solve.

This module only draws inputs: grids, permeability/porosity/conductivity
fields, Newton states and well lists.  It holds none of the discretisation,
preconditioner or Krylov arithmetic, so the GPU library and the CPU oracle
can both consume the very same arrays.

Physical model (Section 2.1 of the paper): single-phase flow with an
exponential density law and backward-Euler time stepping.  The fluid laws
and sizes follow the five benchmark workloads:

  * W1  32x32 2-D, homogeneous k = 1e-13 m^2, porosity 0.2, perturbed state;
  * W2  64x64x32 layered log-normal permeability, corner wells at 450 K;
  * W3  128x128x64, same layered field (4 decades through the clip);
  * W4  96^3 channelised field (sinusoidal 1e-11 streaks in 1e-15 matrix),
        hot injection at 550 K;
  * W5  256x256x64 layered field with streaks overlaid.

Random numbers come from numpy's PCG64 with a fixed draw order, so a
(workload, seed) pair always yields bit-identical arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass(frozen=True)
class Props:
    """Fluid/rock constants, SI units.

    rho = rho0*exp(c_p (p-p0) + c_T (T-T0));  mu = mu0*exp(mu_B (1/T - 1/T0)),
    or, with api > 0, the Bennison heavy-oil correlation of API gravity `api`
    (Section 2.1, eq. bennison).  cv, c_r: specific heats of fluid and rock
    (values of the paper's parameter table); rho_r: rock density (not given
    by the paper); g: gravitational acceleration along -z (0 disables gravity).
    """
    rho0: float = 1000.0
    p0: float = 1.0e7
    T0: float = 350.0
    c_p: float = 4.5e-10
    c_T: float = -3.0e-4
    mu0: float = 1.0e-3
    mu_B: float = 1500.0
    cv: float = 2093.4
    rho_r: float = 2500.0
    c_r: float = 920.0
    g: float = 0.0
    api: float = 0.0

    def as_tuple(self):
        return (self.rho0, self.p0, self.T0, self.c_p, self.c_T, self.mu0,
                self.mu_B, self.cv, self.rho_r, self.c_r, self.g, self.api)


@dataclasses.dataclass(frozen=True)
class Well:
    cell: int
    kind: int          # 0 injector, 1 producer, 2 heater, 3 / 4 Peaceman injector / producer
    rate: float        # m^3/s, >= 0 (heater: the heat-transfer coefficient U in W/K;
                       # Peaceman wells: the maximum rate)
    T_inj: float       # K (injectors; heater: its temperature)
    p_bh: float = 0.0  # Pa, bottom-hole pressure (Peaceman wells)
    wi: float = 0.0    # m^3, well index 2 pi h K_e / ln(r_e / r_w) (Peaceman wells)


def peaceman_wi(Kx: float, Ky: float, h: float = 5.0, r_w: float = 0.1,
                Dx: float = 5.0, Dy: float = 5.0) -> float:
    """Well index of the Peaceman model for K = diag(Kx, Ky, .) (Section 2.1):
    2 pi h K_e / ln(r_e / r_w) with K_e = sqrt(Kx Ky) and the equivalent radius
    r_e of the paper's formula; the paper fixes Dx = Dy = 5 m, h = 5 m and
    r_w = 0.1 m so that the model does not change under mesh refinement."""
    a, b = (Ky / Kx) ** 0.5, (Kx / Ky) ** 0.5
    r_e = 0.14 * (a * Dx * Dx + b * Dy * Dy) ** 0.5 / (0.5 * ((Ky / Kx) ** 0.25 + (Kx / Ky) ** 0.25))
    return 2.0 * np.pi * h * (Kx * Ky) ** 0.5 / np.log(r_e / r_w)


@dataclasses.dataclass
class Problem:
    """One linearised coupled solve: the Jacobian is taken at x_k."""
    name: str
    grid: Grid
    props: Props
    K: np.ndarray          # (n,) permeability, m^2, or (3, n): diag(K_x, K_y, K_z)
    phi: np.ndarray        # (n,) porosity
    kappa: np.ndarray      # (n,) thermal conductivity, W/m/K
    wells: list
    dt: float
    x_prev: np.ndarray     # (2n,) interleaved [p0, T0, p1, T1, ...]
    x_k: np.ndarray        # (2n,) interleaved Newton iterate
    seed: int


DAY = 86400.0
WELL_RATE = 1.0e-5


def _porosity_from_logk(logk: np.ndarray) -> np.ndarray:
    return np.clip(0.2 + 0.05 * (logk + 13.0), 0.1, 0.3)


def layered_field(rng: np.random.Generator, grid: Grid):
    """Layer-wise correlated log-normal permeability.

    Each z-layer draws a mean m_l ~ N(-13, 1); every cell adds U(-0.2, 0.2)
    jitter and log10 k is clipped to [-15, -11] (four decades).
    """
    m = rng.normal(-13.0, 1.0, size=grid.nz)
    jit = rng.uniform(-0.2, 0.2, size=(grid.nz, grid.ny, grid.nx))
    logk = np.clip(m[:, None, None] + jit, -15.0, -11.0)
    return logk.reshape(-1)


def add_streaks(rng: np.random.Generator, grid: Grid, logk: np.ndarray,
                nstreak: int, logk_streak: float = -11.0) -> np.ndarray:
    """Overlay sinusoidal high-permeability channels.

    Streak s has centre line y = y0 + A sin(2 pi x / L + psi) in the x-y
    plane at height z0, with y0 ~ U(0, ny), A ~ U(4, 16), L ~ U(32, 96),
    psi ~ U(0, 2 pi), z0 ~ U(0, nz), half-widths hy, hz in {1, 2} cells.
    A cell centre within the half-widths of a centre line joins the streak.
    """
    logk = logk.reshape(grid.nz, grid.ny, grid.nx).copy()
    xc = np.arange(grid.nx) + 0.5
    yc = np.arange(grid.ny) + 0.5
    zc = np.arange(grid.nz) + 0.5
    for _ in range(nstreak):
        y0 = rng.uniform(0.0, grid.ny)
        amp = rng.uniform(4.0, 16.0)
        lam = rng.uniform(32.0, 96.0)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        z0 = rng.uniform(0.0, grid.nz)
        hy = int(rng.integers(1, 3))
        hz = int(rng.integers(1, 3))
        ycl = y0 + amp * np.sin(2.0 * math.pi * xc / lam + psi)       # (nx,)
        iny = np.abs(yc[:, None] - ycl[None, :]) < hy                 # (ny, nx)
        inz = np.abs(zc - z0) < hz                                    # (nz,)
        mask = inz[:, None, None] & iny[None, :, :]
        logk[mask] = logk_streak
    return logk.reshape(-1)


def perturbed_state(rng: np.random.Generator, n: int, props: Props,
                    sigma_p: float = 1.0e5, sigma_T: float = 5.0):
    """x_prev uniform (p0, T0); x_k = x_prev + (N(0, sigma_p), N(0, sigma_T))."""
    x_prev = np.empty(2 * n)
    x_prev[0::2] = props.p0
    x_prev[1::2] = props.T0
    dp = rng.normal(0.0, sigma_p, size=n)
    dT = rng.normal(0.0, sigma_T, size=n)
    x_k = x_prev.copy()
    x_k[0::2] += dp
    x_k[1::2] += dT
    return x_prev, x_k


def corner_wells(grid: Grid, T_inj: float, rate: float = WELL_RATE):
    return [Well(0, 0, rate, T_inj), Well(grid.n - 1, 1, rate, T_inj)]


def _paper_perm(n: int, anisotropic: bool) -> np.ndarray:
    """Homogeneous 3e-13 m^2; anisotropic: diag(3e-11, 3e-13, 3e-13) (Section 4,
    Cases IV and V)."""
    if not anisotropic:
        return np.full(n, 3.0e-13)
    K = np.full((3, n), 3.0e-13)
    K[0] = 3.0e-11
    return K


def make_problem(name: str, seed: int | None = None, props: Props | None = None,
                 kappa: float | None = None, grid: Grid | None = None) -> Problem:
    """Build one of the named workloads (W1..W5) or a scaled variant.

    ``grid`` overrides the size of the named workload (same recipe on a
    different grid), used for small parity cases.
    """
    props = props or Props()
    if name == "W1":
        seed = 1 if seed is None else seed
        grid = grid or Grid(32, 32, 1, 20.0 / 32, 20.0 / 32, 1.0)
        rng = np.random.default_rng(np.random.PCG64(seed))
        n = grid.n
        K = np.full(n, 1.0e-13)
        phi = np.full(n, 0.2)
        kap = np.full(n, 2.0 if kappa is None else kappa)
        x_prev, x_k = perturbed_state(rng, n, props)
        return Problem(name, grid, props, K, phi, kap, [], DAY, x_prev, x_k, seed)
    if name in ("W2", "W3"):
        seed = (2 if name == "W2" else 3) if seed is None else seed
        dims = (64, 64, 32) if name == "W2" else (128, 128, 64)
        grid = grid or Grid(*dims, 1.0, 1.0, 1.0)
        rng = np.random.default_rng(np.random.PCG64(seed))
        logk = layered_field(rng, grid)
        K = 10.0 ** logk
        phi = _porosity_from_logk(logk)
        kap = np.full(grid.n, 2.0 if kappa is None else kappa)
        x_prev, x_k = perturbed_state(rng, grid.n, props)
        return Problem(name, grid, props, K, phi, kap, corner_wells(grid, 450.0),
                       DAY, x_prev, x_k, seed)
    if name == "W4":
        seed = 4001 if seed is None else seed
        grid = grid or Grid(96, 96, 96, 1.0, 1.0, 1.0)
        rng = np.random.default_rng(np.random.PCG64(seed))
        logk = np.full(grid.n, -15.0)
        nstreak = max(1, int(round(24 * grid.n / 96 ** 3)))
        logk = add_streaks(rng, grid, logk, nstreak)
        K = 10.0 ** logk
        phi = np.where(logk > -13.0, 0.3, 0.1)
        kap = np.full(grid.n, 2.0 if kappa is None else kappa)
        x_prev, x_k = perturbed_state(rng, grid.n, props)
        return Problem(name, grid, props, K, phi, kap, corner_wells(grid, 550.0),
                       DAY, x_prev, x_k, seed)
    if name == "W5":
        seed = 5 if seed is None else seed
        grid = grid or Grid(256, 256, 64, 1.0, 1.0, 1.0)
        rng = np.random.default_rng(np.random.PCG64(seed))
        logk = layered_field(rng, grid)
        nstreak = max(1, int(round(24 * grid.n / 96 ** 3)))
        logk = add_streaks(rng, grid, logk, nstreak)
        K = 10.0 ** logk
        phi = _porosity_from_logk(logk)
        kap = np.full(grid.n, 20.0 if kappa is None else kappa)
        x_prev = np.empty(2 * grid.n)
        x_prev[0::2] = props.p0
        x_prev[1::2] = props.T0
        return Problem(name, grid, props, K, phi, kap, corner_wells(grid, 450.0),
                       DAY, x_prev, x_prev.copy(), seed)
    if name == "R2":
        # mesh-refinement recipe: N x N cells of a 20 m x 20 m x 1 m slab,
        # homogeneous, uniform start, an injector (450 K) and a producer at
        # opposite corners; the flow the wells drive stays smooth as the mesh
        # is refined
        seed = 0 if seed is None else seed
        grid = grid or Grid(80, 80, 1, 20.0 / 80, 20.0 / 80, 1.0)
        n = grid.n
        K = np.full(n, 1.0e-13)
        phi = np.full(n, 0.2)
        kap = np.full(n, 2.0 if kappa is None else kappa)
        x_prev = np.empty(2 * n)
        x_prev[0::2] = props.p0
        x_prev[1::2] = props.T0
        return Problem(name, grid, props, K, phi, kap, corner_wells(grid, 450.0, rate=1.0e-6),
                       DAY, x_prev, x_prev.copy(), seed)
    if name in ("CaseI", "CaseIV"):
        # the problem-size study's heater cases (Section 4): as Case II with six
        # heaters (coefficient 5.44409e-6 W/K, 422.039 K) instead of wells; the
        # paper does not place them: x = 5, 10, 15 m at y = 5 and 15 m.  Case IV
        # raises the permeability along x to 3e-11 m^2
        seed = 0 if seed is None else seed
        N = 80
        grid = grid or Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
        n = grid.n
        K = _paper_perm(n, name == "CaseIV")
        phi = np.full(n, 0.2)
        kap = np.full(n, 2.0 if kappa is None else kappa)

        def cell(x, y):
            return min(grid.nx - 1, int(x / grid.dx)) + grid.nx * min(grid.ny - 1, int(y / grid.dy))
        heaters = [Well(cell(x, y), 2, 5.44409e-6, 422.039) for y in (5.0, 15.0) for x in (5.0, 10.0, 15.0)]
        x_prev = np.empty(2 * n)
        x_prev[0::2] = props.p0
        x_prev[1::2] = 288.706
        return Problem(name, grid, props, K, phi, kap, heaters, 10.0 * DAY, x_prev, x_prev.copy(), seed)
    if name in ("CaseII", "CaseIII", "CaseV"):
        # the problem-size study's well cases (Section 4): N x N cells of a
        # 20 m x 20 m x 1 m square, k = 3e-13 m^2, porosity 0.2, uniform start
        # at 288.706 K (Case III: 320 K), 3 injectors (422.039 K) and 3
        # producers at constant rates 5e-8 m^3/s (Cases III and V: 1e-6),
        # 10-day steps (Case V: 12 hours, with K_x raised to 3e-11 m^2); the
        # paper does not place the wells: injectors at x = 2.5 m and producers
        # at x = 17.5 m, both at y = 2.5, 10 and 17.5 m
        seed = 0 if seed is None else seed
        N = 80
        grid = grid or Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
        n = grid.n
        K = _paper_perm(n, name == "CaseV")
        phi = np.full(n, 0.2)
        kap = np.full(n, 2.0 if kappa is None else kappa)
        T_init = 320.0 if name == "CaseIII" else 288.706
        rate = 5.0e-8 if name == "CaseII" else 1.0e-6
        dt = 0.5 * DAY if name == "CaseV" else 10.0 * DAY

        def cell(x, y):
            ix = min(grid.nx - 1, int(x / grid.dx))
            iy = min(grid.ny - 1, int(y / grid.dy))
            return ix + grid.nx * iy
        wells = [Well(cell(2.5, y), 0, rate, 422.039) for y in (2.5, 10.0, 17.5)]
        wells += [Well(cell(17.5, y), 1, rate, 422.039) for y in (2.5, 10.0, 17.5)]
        x_prev = np.empty(2 * n)
        x_prev[0::2] = props.p0
        x_prev[1::2] = T_init
        return Problem(name, grid, props, K, phi, kap, wells, dt, x_prev, x_prev.copy(), seed)
    raise ValueError(f"unknown workload {name!r}")


def random_rhs(seed: int, m: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.standard_normal(m)


def poisson_csr(dims, dirichlet: bool = True):
    """Constant-coefficient 5-point (2-D) or 7-point (3-D) Laplacian, CSR.

    Unit grid spacing; Dirichlet rows keep the full diagonal 2*d so the
    operator is the standard SPD finite-difference Laplacian.  Columns are
    sorted ascending.  Used as an AMG test operator.
    """
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    if nd == 2:
        dims = (dims[0], dims[1], 1)
    nx, ny, nz = dims
    n = nx * ny * nz
    rowptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    diag = 2.0 * nd
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                i = ix + nx * (iy + ny * iz)
                row = []
                if iz > 0:
                    row.append((i - nx * ny, -1.0))
                if iy > 0:
                    row.append((i - nx, -1.0))
                if ix > 0:
                    row.append((i - 1, -1.0))
                nb = sum(1 for _ in row)
                row.append((i, 0.0))
                if ix < nx - 1:
                    row.append((i + 1, -1.0))
                if iy < ny - 1:
                    row.append((i + nx, -1.0))
                if iz < nz - 1:
                    row.append((i + nx * ny, -1.0))
                nnb = len(row) - 1
                d = diag if dirichlet else float(nnb)
                row[nb] = (i, d)
                for c, v in row:
                    cols.append(c)
                    vals.append(v)
                rowptr[i + 1] = len(cols)
    return (n, rowptr, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64))
