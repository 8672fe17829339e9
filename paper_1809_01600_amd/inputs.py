"""Seeded synthetic inputs shared by the HIP path's tests, the oracle's tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws porous geometries and
boundary data and carries the physical parameters of each workload.  The lattice conversion,
the connectivity clean-up of the pore space and everything after it are done separately by the
HIP library and by the oracle.

Workloads (the paper's anode problem, Section 4.1, with synthetic stand-ins for its measured
anode, whose geometry and data are not available):

* ``stefan_tube``  - open 128 x 8 channel, no solid, ternary H2-H2O-Ar, T = 1073 K, p = 1 atm,
  X_in = (0.6, 0.3, 0.1), j = 0.5 A/cm^2 (the quasi-1D Stefan tube).
* ``porous_2d``    - 1024 x 1024 slice of overlapping disks (radius U[4, 12]) at void fraction
  0.40, X_in ~ Dirichlet(6, 3, 1), j = 1.0 A/cm^2.
* ``porous_3d``    - 256^3 block of overlapping spheres (radius U[3, 8]) at void fraction
  U[0.35, 0.50].
* ``batch_2d``     - 64 square slices with sides in [256, 1024], void fraction U[0.3, 0.5],
  disk radius U[3, 12], j ~ U[0, 2] A/cm^2.

All random draws use numpy's PCG64 generator, seeded explicitly.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

# Binary Maxwell-Stefan diffusivities of the ternary H2 (1) - H2O (2) - Ar (3) mixture used by the
# synthetic workloads [m^2/s] (physical inputs, like the paper's Table 2 operating point).
D12_DEFAULT = 7.6e-4
D13_DEFAULT = 6.8e-4
D23_DEFAULT = 2.5e-4


@dataclasses.dataclass
class Case:
    """One problem instance: physical inputs plus the solid mask (uint8, 1 = solid).

    Arrays are indexed ``solid[z, y, x]`` (x fastest, x = diffusion direction, inlet at x = 0,
    reactive outlet at x = nx - 1).  ``nz == 1`` for the two-dimensional lattice.
    """

    name: str
    lattice: str                      # "D2Q9" or "D3Q19"
    nx: int
    ny: int
    nz: int
    T: float = 1073.0                 # K
    p: float = 101325.0               # Pa
    D12: float = D12_DEFAULT          # m^2/s
    D13: float = D13_DEFAULT
    D23: float = D23_DEFAULT
    dx: float = 1.0e-6                # m
    tau_ref: float = 100.0
    X_in: Tuple[float, float, float] = (0.6, 0.3, 0.1)
    j_A_cm2: float = 1.0              # current density, A/cm^2
    nu: Tuple[int, int, int] = (-1, 1, 0)
    n_electrons: int = 2
    solid: Optional[np.ndarray] = None
    seed: Optional[int] = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def j_A_m2(self) -> float:
        return self.j_A_cm2 * 1.0e4

    def mask(self) -> np.ndarray:
        if self.solid is None:
            return np.zeros(self.shape, dtype=np.uint8)
        return np.ascontiguousarray(self.solid, dtype=np.uint8)

    def D_matrix(self) -> np.ndarray:
        D = np.zeros((3, 3))
        D[0, 1] = D[1, 0] = self.D12
        D[0, 2] = D[2, 0] = self.D13
        D[1, 2] = D[2, 1] = self.D23
        return D


# ----------------------------------------------------------------------------------------------
# geometry generators
# ----------------------------------------------------------------------------------------------

def disks_2d(nx: int, ny: int, porosity: float, r_lo: float, r_hi: float,
             rng: np.random.Generator) -> np.ndarray:
    """Overlapping disks with uniform centres, periodic in y, clipped in x.

    Cell (x, y) is solid when (x + 1/2 - cx)^2 + wrap_y(y + 1/2 - cy)^2 <= r^2.  Disks are added
    until the void fraction first drops to ``porosity`` or below.  Returns uint8 [1, ny, nx].
    """
    solid = np.zeros((ny, nx), dtype=np.uint8)
    n_total = nx * ny
    n_solid = 0
    target = (1.0 - porosity) * n_total
    while n_solid < target:
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        r = rng.uniform(r_lo, r_hi)
        x0 = max(int(np.floor(cx - r - 1)), 0)
        x1 = min(int(np.ceil(cx + r + 1)), nx)
        ys = np.arange(int(np.floor(cy - r - 1)), int(np.ceil(cy + r + 1)))
        xs = np.arange(x0, x1)
        if xs.size == 0:
            continue
        dy = ys + 0.5 - cy
        yw = np.mod(ys, ny)
        dx = xs + 0.5 - cx
        hit = (dy[:, None] ** 2 + dx[None, :] ** 2) <= r * r
        # a disk wider than the domain in y could wrap onto itself; radii here are far smaller
        sub = solid[yw[:, None], xs[None, :]]
        newly = hit & (sub == 0)
        n_solid += int(newly.sum())
        sub[hit] = 1
        solid[yw[:, None], xs[None, :]] = sub
    return solid[None, :, :]


def spheres_3d(nx: int, ny: int, nz: int, porosity: float, r_lo: float, r_hi: float,
               rng: np.random.Generator) -> np.ndarray:
    """Overlapping spheres with uniform centres, periodic in y and z, clipped in x.

    Returns uint8 [nz, ny, nx]; spheres are added until the void fraction is <= ``porosity``.
    """
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    n_total = nx * ny * nz
    n_solid = 0
    target = (1.0 - porosity) * n_total
    while n_solid < target:
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        cz = rng.uniform(0.0, nz)
        r = rng.uniform(r_lo, r_hi)
        xs = np.arange(max(int(np.floor(cx - r - 1)), 0), min(int(np.ceil(cx + r + 1)), nx))
        if xs.size == 0:
            continue
        ys = np.arange(int(np.floor(cy - r - 1)), int(np.ceil(cy + r + 1)))
        zs = np.arange(int(np.floor(cz - r - 1)), int(np.ceil(cz + r + 1)))
        d2 = ((zs + 0.5 - cz)[:, None, None] ** 2 + (ys + 0.5 - cy)[None, :, None] ** 2
              + (xs + 0.5 - cx)[None, None, :] ** 2)
        hit = d2 <= r * r
        iz = np.mod(zs, nz)[:, None, None]
        iy = np.mod(ys, ny)[None, :, None]
        ix = xs[None, None, :]
        sub = solid[iz, iy, ix]
        n_solid += int((hit & (sub == 0)).sum())
        sub[hit] = 1
        solid[iz, iy, ix] = sub
    return solid


# ----------------------------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------------------------

def stefan_tube(nx: int = 128, ny: int = 8, j_A_cm2: float = 0.5, dx: Optional[float] = None,
                tau_ref: float = 50.0, X_in=(0.6, 0.3, 0.1), lattice: str = "D2Q9",
                nz: int = 1) -> Case:
    """Open quasi-1D channel (no solid).  Default: 2 mm over 128 nodes, j = 0.5 A/cm^2."""
    if dx is None:
        dx = 2.0e-3 / 128
    if lattice == "D2Q9":
        nz = 1
    return Case(name="stefan_tube", lattice=lattice, nx=nx, ny=ny, nz=nz, T=1073.0,
                p=101325.0, dx=dx, tau_ref=tau_ref, X_in=tuple(X_in), j_A_cm2=j_A_cm2)


def porous_2d(n: int = 1024, seed: int = 2, porosity: float = 0.40, j_A_cm2: float = 1.0,
              r_lo: float = 4.0, r_hi: float = 12.0, ny: Optional[int] = None,
              tau_ref: float = 100.0) -> Case:
    """Porous anode slice of overlapping disks; X_in drawn from Dirichlet(6, 3, 1) afterwards."""
    ny = n if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = disks_2d(n, ny, porosity, r_lo, r_hi, rng)
    X_in = tuple(float(v) for v in rng.dirichlet((6.0, 3.0, 1.0)))
    return Case(name="porous_2d", lattice="D2Q9", nx=n, ny=ny, nz=1, dx=1.0e-6,
                tau_ref=tau_ref, X_in=X_in, j_A_cm2=j_A_cm2, solid=solid, seed=seed)


def porous_3d(n: int = 256, seed: int = 3, j_A_cm2: float = 1.0, r_lo: float = 3.0,
              r_hi: float = 8.0, porosity: Optional[float] = None,
              tau_ref: float = 100.0) -> Case:
    """Porous anode block of overlapping spheres; void fraction ~ U[0.35, 0.50] from the seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if porosity is None:
        porosity = float(rng.uniform(0.35, 0.50))
    solid = spheres_3d(n, n, n, porosity, r_lo, r_hi, rng)
    return Case(name="porous_3d", lattice="D3Q19", nx=n, ny=n, nz=n, dx=1.0e-6,
                tau_ref=tau_ref, X_in=(0.6, 0.3, 0.1), j_A_cm2=j_A_cm2, solid=solid, seed=seed)


def batch_2d(count: int = 64, base_seed: int = 4000, side_lo: int = 256, side_hi: int = 1024,
             j_hi: float = 2.0, tau_ref: float = 100.0, accept=None):
    """Ragged batch of square porous slices for one polarization curve (one X_in).  Instance k
    draws from seed base_seed + k; if accept(solid) is given and rejects the geometry (say, no
    pore path from inlet to outlet), it draws again from seed base_seed + k + 1000 a, a = 1, 2..."""
    cases = []
    for k in range(count):
        for attempt in range(100):
            seed = base_seed + k + 1000 * attempt
            rng = np.random.Generator(np.random.PCG64(seed))
            side = int(rng.integers(side_lo, side_hi + 1))
            por = float(rng.uniform(0.3, 0.5))
            j = float(rng.uniform(0.0, j_hi))
            solid = disks_2d(side, side, por, 3.0, 12.0, rng)
            if accept is None or accept(solid):
                break
        else:
            raise RuntimeError("no accepted geometry for instance %d" % k)
        cases.append(Case(name=f"batch_{k}", lattice="D2Q9", nx=side, ny=side, nz=1,
                          dx=1.0e-6, tau_ref=tau_ref, X_in=(0.6, 0.3, 0.1), j_A_cm2=j,
                          solid=solid, seed=seed))
    return cases


def random_small(nx: int, ny: int, nz: int, lattice: str, seed: int, solid_frac: float = 0.25,
                 j_A_cm2: float = 1.0, dx: float = 1.0e-6, tau_ref: float = 3.0,
                 X_in=(0.6, 0.3, 0.1)) -> Case:
    """Tiny grid with independent random solid voxels (for brute-force and parity cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = (rng.random((nz, ny, nx)) < solid_frac).astype(np.uint8)
    return Case(name="random_small", lattice=lattice, nx=nx, ny=ny, nz=nz, dx=dx,
                tau_ref=tau_ref, X_in=tuple(X_in), j_A_cm2=j_A_cm2, solid=solid, seed=seed)


def random_field(shape, seed: int, lo: float = 0.05, hi: float = 0.9) -> np.ndarray:
    """A random ternary composition field [3, nz, ny, nx] (rows sum to one), for warm starts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(lo, hi, size=(3,) + tuple(shape))
    return a / a.sum(axis=0, keepdims=True)
