"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module defines *inputs* only: the parameters of the model systems
(mesh sizes, box, potential and field generators, pseudo-atoms, block sizes),
the scalar fields V_eff(r) and B_xc(r) as plain functions of position, and the
counter-based random numbers used for starting vectors.  It contains none of
the finite-element or eigensolver arithmetic: quadrature points, basis
functions, cell matrices and projectors are computed independently by each
consumer from the point sets they own.

The paper's systems (twisted WTe2 bilayers, MnSi supercells with ONCV
pseudopotentials, Sec. V) are not available; these seeded systems stand in for
them with the same structure: periodic orthorhombic boxes, degree-p spectral
elements, a smooth effective potential, a noncollinear exchange field of
constant magnitude, and atom-centred spin-orbit projectors (Sec. II.B,
eqn:nlOP).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014).  Counter-based use: the i-th output (i >= 0) of the
# sequential generator seeded with `seed` is mix(seed + (i + 1) * GAMMA).
# --------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number `counters` (uint64 array) of SplitMix64 seeded with `seed`."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, counters: np.ndarray) -> np.ndarray:
    """U[-1, 1) doubles from the top 53 bits of SplitMix64 outputs."""
    z = splitmix64(seed, counters)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def random_block(seed: int, n_rows: int, n_cols: int, row0: int = 0,
                 col0: int = 0, n_total_cols: Optional[int] = None) -> np.ndarray:
    """Complex block X[r, n] = u(2 j) + i u(2 j + 1), j = r * n_total_cols + n.

    Returns rows [row0, row0 + n_rows) and columns [col0, col0 + n_cols) of the
    seeded [rows][n_total_cols] complex128 multivector.
    """
    ntc = n_cols if n_total_cols is None else n_total_cols
    r = np.arange(row0, row0 + n_rows, dtype=np.uint64)[:, None]
    n = np.arange(col0, col0 + n_cols, dtype=np.uint64)[None, :]
    j = r * np.uint64(ntc) + n
    re = uniform_pm1(seed, np.uint64(2) * j)
    im = uniform_pm1(seed, np.uint64(2) * j + np.uint64(1))
    return re + 1j * im


def random_rows(seed: int, rows, n_cols: int, n_total_cols: Optional[int] = None,
                col0: int = 0) -> np.ndarray:
    """Arbitrary rows of the same seeded multivector as random_block."""
    ntc = n_cols if n_total_cols is None else n_total_cols
    r = np.asarray(rows, dtype=np.uint64)[:, None]
    n = np.arange(col0, col0 + n_cols, dtype=np.uint64)[None, :]
    j = r * np.uint64(ntc) + n
    return uniform_pm1(seed, np.uint64(2) * j) + 1j * uniform_pm1(seed, np.uint64(2) * j + np.uint64(1))


# --------------------------------------------------------------------------
# System description
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Atom:
    pos: Tuple[float, float, float]
    lmax: int               # projectors for l = 0..lmax, 2l+1 real harmonics each
    sigma: float            # Gaussian width of the radial part (bohr)
    rcut: float             # projector support radius (bohr)
    d0: Tuple[float, ...]   # scalar nonlocal strength per l (Ha)
    dso: float              # spin-orbit strength (Ha), couples via L.S


@dataclasses.dataclass
class System:
    name: str
    n_cells: Tuple[int, int, int]
    box: Tuple[float, float, float]
    p: int
    quad: str                      # "gl" (Gauss-Legendre, n_q points) or "gll"
    n_q: int
    kpts: np.ndarray               # [n_k][3] Cartesian (1/bohr)
    # V_eff = sum_g A_g exp(-|r - c_g|^2 / (2 w^2)) over periodic images
    v_centres: np.ndarray
    v_amps: np.ndarray
    v_width: float
    v_const: float
    # B_xc = b_mag * v / |v|,  v = b_bias + sum_g d_g exp(-|r - c'_g|^2 / (2 wb^2))
    b_mag: float
    b_bias: np.ndarray
    b_centres: np.ndarray
    b_dirs: np.ndarray
    b_width: float
    atoms: List[Atom]
    n_vec: int
    block: int
    degree: int
    passes: int
    seed: int

    @property
    def nodes_per_dir(self):
        return tuple(n * self.p for n in self.n_cells)

    @property
    def n_nodes(self):
        a, b, c = self.nodes_per_dir
        return a * b * c

    @property
    def n_dof(self):
        return 2 * self.n_nodes

    @property
    def n_cell_total(self):
        a, b, c = self.n_cells
        return a * b * c


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_system(name: str = "tiny", *, n_cells=(3, 3, 3), box=(8.0, 8.0, 8.0),
                p: int = 4, quad: str = "gl", n_q: Optional[int] = None,
                kpts: Optional[Sequence[Sequence[float]]] = None,
                n_gauss: int = 6, v_width: float = 1.0, v_const: float = 0.0,
                b_mag: float = 0.1, b_gauss: int = 3, b_width: float = 2.0,
                b_bias=(0.0, 0.0, 0.5),
                n_atoms: int = 2, atom_lattice: Optional[int] = None,
                lmax: int = 1, sigma: float = 0.7, rcut_sigmas: float = 8.0,
                d0=(1.0, 0.5, 0.25), dso: float = 0.05,
                n_vec: int = 32, block: Optional[int] = None, degree: int = 10,
                passes: int = 3, seed: int = 0) -> System:
    """Seeded system; parameter draws in a fixed order from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(box, dtype=np.float64)
    v_centres = rng.uniform(0.0, 1.0, size=(n_gauss, 3)) * L
    v_amps = rng.uniform(-2.0, 0.0, size=n_gauss)
    b_centres = rng.uniform(0.0, 1.0, size=(b_gauss, 3)) * L
    b_dirs = _unit_vectors(rng, b_gauss)
    atoms: List[Atom] = []
    if atom_lattice:
        g = atom_lattice
        jit = rng.uniform(-0.5, 0.5, size=(g ** 3, 3))
        idx = 0
        for iz in range(g):
            for iy in range(g):
                for ix in range(g):
                    base = (np.array([ix, iy, iz]) + 0.5) / g * L
                    pos = np.mod(base + jit[idx], L)
                    idx += 1
                    atoms.append(Atom(tuple(pos), lmax, sigma, rcut_sigmas * sigma,
                                      tuple(d0[: lmax + 1]), dso))
    else:
        pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
        for a in range(n_atoms):
            atoms.append(Atom(tuple(pos[a]), lmax, sigma, rcut_sigmas * sigma,
                              tuple(d0[: lmax + 1]), dso))
    if kpts is None:
        kpts = [(0.0, 0.0, 0.0)]
    if n_q is None:
        n_q = p + 1
    if quad == "gll":
        n_q = p + 1
    return System(name=name, n_cells=tuple(int(x) for x in n_cells),
                  box=tuple(float(x) for x in box), p=int(p), quad=quad, n_q=int(n_q),
                  kpts=np.asarray(kpts, dtype=np.float64).reshape(-1, 3),
                  v_centres=v_centres, v_amps=v_amps, v_width=float(v_width),
                  v_const=float(v_const), b_mag=float(b_mag),
                  b_bias=np.asarray(b_bias, dtype=np.float64), b_centres=b_centres,
                  b_dirs=b_dirs, b_width=float(b_width), atoms=atoms,
                  n_vec=int(n_vec), block=int(block or n_vec), degree=int(degree),
                  passes=int(passes), seed=int(seed))


def monkhorst_pack(q: int, box) -> np.ndarray:
    """q x q x q Monkhorst-Pack grid, k_d = (2r - q - 1)/(2q) * 2 pi / L_d."""
    L = np.asarray(box, dtype=np.float64)
    f = [(2 * r - q - 1) / (2.0 * q) for r in range(1, q + 1)]
    out = []
    for fz in f:
        for fy in f:
            for fx in f:
                out.append(2.0 * np.pi * np.array([fx, fy, fz]) / L)
    return np.array(out)


# Named workloads -----------------------------------------------------------
def config(name: str) -> System:
    """The named workloads.

    tiny    : 3^3 cells, p=4, L=8, Gamma, 6 Gaussians, 2 atoms (l<=1), N=32, m=10, 3 passes
    scale   : 20^3 cells, p=6, L=24, Gamma, 200 Gaussians, 64 atoms (l<=2), N=512 (4x128), m=24, 4 passes
    reduced : 6^3 cells, p=6, h=1.2 with the same generator densities as `scale`, N=128, m=24
    kgrid   : 12^3 cells, p=5, L=14.4, 2x2x2 Monkhorst-Pack, 27 atoms (l<=1), N=384, m=16
    uneven1..uneven5 : Gamma systems of 6^3, 8^3, 10^3, 12^3, 14^3 cells, p=5, h=1.2, Gaussians
              at 6/512 per bohr^3, ceil(E/32) atoms (l<=1), N=64, 128, 192, 256, 320, m=16,
              seeds 1..5 (the uneven members of the batched workload)
    adjoint : 10^3 cells, p=5, L=12, Gamma, 8 atoms (l<=1), N=256, m=16
    """
    if name == "tiny":
        return make_system("tiny")
    if name == "scale":
        return make_system("scale", n_cells=(20, 20, 20), box=(24.0, 24.0, 24.0), p=6,
                           n_gauss=200, n_atoms=64, atom_lattice=4, lmax=2,
                           rcut_sigmas=6.0, n_vec=512, block=128, degree=24, passes=4)
    if name == "reduced":
        return make_system("reduced", n_cells=(6, 6, 6), box=(7.2, 7.2, 7.2), p=6,
                           n_gauss=max(1, round(200 * 7.2 ** 3 / 24.0 ** 3)),
                           n_atoms=2, lmax=2, rcut_sigmas=6.0, n_vec=128, block=128,
                           degree=24, passes=4)
    if name == "kgrid":
        L = 14.4
        return make_system("kgrid", n_cells=(12, 12, 12), box=(L, L, L), p=5,
                           kpts=monkhorst_pack(2, (L, L, L)),
                           n_gauss=round(6 / 512 * L ** 3), n_atoms=27, atom_lattice=3,
                           lmax=1, rcut_sigmas=6.0, n_vec=384, block=128, degree=16,
                           passes=3, seed=1)
    if name.startswith("uneven") and name[6:].isdigit() and 1 <= int(name[6:]) <= 5:
        i = int(name[6:])
        nc = 4 + 2 * i
        L = 1.2 * nc
        return make_system(name, n_cells=(nc, nc, nc), box=(L, L, L), p=5,
                           n_gauss=max(1, round(6 / 512 * L ** 3)), n_atoms=-(-nc ** 3 // 32),
                           lmax=1, rcut_sigmas=6.0, n_vec=64 * i, block=64 * i, degree=16,
                           passes=3, seed=i)
    if name == "adjoint":
        return make_system("adjoint", n_cells=(10, 10, 10), box=(12.0, 12.0, 12.0), p=5,
                           n_gauss=round(6 / 512 * 12.0 ** 3), n_atoms=8, lmax=1,
                           rcut_sigmas=6.0, n_vec=256, block=128, degree=16, passes=1)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Fields as functions of position (periodic images summed explicitly)
# --------------------------------------------------------------------------
def _gauss_sum(points: np.ndarray, centres: np.ndarray, weights: np.ndarray,
               width: float, box) -> np.ndarray:
    """sum_g weights[g] * sum_L exp(-|r - c_g - L|^2 / (2 width^2)).

    weights is [G] (scalar result) or [G][3] (vector result).  Images are summed
    out to 9 widths, beyond which a term is below 1e-17 of its amplitude.
    """
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    L = np.asarray(box, dtype=np.float64)
    cut = 9.0 * width
    vec = weights.ndim == 2
    out = np.zeros((pts.shape[0], 3) if vec else pts.shape[0])
    # |minimum-image displacement| <= L/2, so shifts with |n| L < cut + L/2 suffice
    nimg = [int(math.floor((cut + L[d] / 2) / L[d])) for d in range(3)]
    chunk = 1 << 16
    for s in range(0, pts.shape[0], chunk):
        P = pts[s:s + chunk]
        acc = np.zeros((P.shape[0], 3) if vec else P.shape[0])
        for g in range(centres.shape[0]):
            d0 = P - centres[g]
            d0 = d0 - L * np.round(d0 / L)        # minimum image
            for ix in range(-nimg[0], nimg[0] + 1):
                for iy in range(-nimg[1], nimg[1] + 1):
                    for iz in range(-nimg[2], nimg[2] + 1):
                        d = d0 - np.array([ix, iy, iz]) * L
                        r2 = np.einsum("ij,ij->i", d, d)
                        m = r2 < cut * cut
                        if not np.any(m):
                            continue
                        e = np.zeros(P.shape[0])
                        e[m] = np.exp(-r2[m] / (2.0 * width * width))
                        if vec:
                            acc += e[:, None] * weights[g][None, :]
                        else:
                            acc += e * weights[g]
        out[s:s + chunk] = acc
    return out


def veff(system: System, points: np.ndarray) -> np.ndarray:
    """V_eff at the given points [P][3] -> [P]."""
    return system.v_const + _gauss_sum(points, system.v_centres, system.v_amps,
                                       system.v_width, system.box)


def bxc(system: System, points: np.ndarray) -> np.ndarray:
    """B_xc at the given points [P][3] -> [P][3] (magnitude b_mag everywhere)."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if system.b_mag == 0.0:
        return np.zeros((pts.shape[0], 3))
    v = system.b_bias[None, :] + _gauss_sum(pts, system.b_centres, system.b_dirs,
                                             system.b_width, system.box)
    return system.b_mag * v / np.linalg.norm(v, axis=1, keepdims=True)


def start_block(system: System, n_rows: int, n_cols: Optional[int] = None,
                col0: int = 0) -> np.ndarray:
    """X0: the seeded [2M][n_vec] starting block (columns col0..col0+n_cols)."""
    n_cols = system.n_vec if n_cols is None else n_cols
    return random_block(system.seed, n_rows, n_cols, col0=col0,
                        n_total_cols=system.n_vec)


def lanczos_start(system: System, n_rows: int) -> np.ndarray:
    """Seeded Lanczos starting vector (its own stream: seed + 1)."""
    return random_block(system.seed + 1, n_rows, 1)[:, 0]
