"""Seeded synthetic inputs for the NEP molecular-dynamics path.

This module is shared by the HIP path, the tests and the oracle's callers. It
builds atoms, boxes, velocities and random model parameters from
``numpy.random.default_rng`` seeds and holds none of the NEP arithmetic
(no cutoff, basis, descriptor, network or force code).

Workloads stand in for the paper's copper runs (Section VI.A: FCC Cu, 1 fs
step, Maxwell-Boltzmann velocities at 300 K). The trained copper potential is
not available, so every model here is a random-weight NEP with the paper's
hyperparameters (Section VI.A: n_max 4, basis size 8, three-body l_max 4,
four-body l_max 2, 30 hidden neurons) and the cutoffs of the synthetic
workloads (radial 6 A, angular 5 A).
"""
from __future__ import annotations

import dataclasses
import json
from typing import Optional, Tuple

import numpy as np

# Unit system: angstrom, femtosecond, eV, amu, kelvin.
# 1 amu * A^2 / fs^2 expressed in eV.
AMU_A2_FS2_IN_EV = 103.642697
BOLTZMANN_EV_PER_K = 8.617333262e-5

CU_LATTICE_A = 3.615
CU_MASS_AMU = 63.546

FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]],
    dtype=np.float64,
)


@dataclasses.dataclass
class Atoms:
    """An orthorhombic periodic system in original atom order."""

    x: np.ndarray          # [N][3] float64, wrapped into [0, L)
    types: np.ndarray      # [N] int32
    box: np.ndarray        # [3] float64 side lengths
    masses: np.ndarray     # [n_types] float64 (amu)
    v: Optional[np.ndarray] = None  # [N][3] float64 (A/fs)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Map coordinates into [0, L) per axis."""
    y = np.mod(x, box)
    # np.mod can return L itself for tiny negative inputs; fold those back.
    y = np.where(y >= box, y - box, y)
    return np.ascontiguousarray(y)


def fcc_lattice(n_cells: int, a: float = CU_LATTICE_A) -> tuple[np.ndarray, np.ndarray]:
    """Perfect FCC sites; id = 4*((ix*n + iy)*n + iz) + b."""
    idx = np.arange(n_cells, dtype=np.float64)
    ix, iy, iz = np.meshgrid(idx, idx, idx, indexing="ij")
    cells = np.stack([ix, iy, iz], axis=-1).reshape(-1, 1, 3)
    pos = (cells + FCC_BASIS[None, :, :]) * a
    box = np.full(3, n_cells * a, dtype=np.float64)
    return np.ascontiguousarray(pos.reshape(-1, 3)), box


def fcc_box(n_cells: int, sigma: float, seed: Optional[int], a: float = CU_LATTICE_A,
            mass: float = CU_MASS_AMU) -> Atoms:
    """Single-species FCC box with Gaussian displacements (std ``sigma`` per component)."""
    x, box = fcc_lattice(n_cells, a)
    if sigma > 0.0:
        rng = np.random.default_rng(seed)
        x = x + rng.normal(0.0, sigma, size=x.shape)
    return Atoms(x=wrap(x, box), types=np.zeros(x.shape[0], np.int32), box=box,
                 masses=np.array([mass], np.float64))


def alloy_box(n_cells: int, type_seed: int, n_vacancies: int, vacancy_seed: int,
              sigma: float, disp_seed: int, a: float = CU_LATTICE_A,
              masses=(CU_MASS_AMU, CU_MASS_AMU)) -> Atoms:
    """Two-species 50/50 random FCC alloy with random vacancies.

    Types come from a seeded permutation (first half type 0, second half type 1),
    vacancies remove ``n_vacancies`` seeded random sites, and surviving sites keep
    their ascending site order as atom ids.
    """
    x, box = fcc_lattice(n_cells, a)
    n_sites = x.shape[0]
    perm = np.random.default_rng(type_seed).permutation(n_sites)
    types = np.zeros(n_sites, np.int32)
    types[perm[n_sites // 2:]] = 1
    removed = np.random.default_rng(vacancy_seed).choice(n_sites, size=n_vacancies, replace=False)
    keep = np.ones(n_sites, bool)
    keep[removed] = False
    x = x[keep]
    types = types[keep]
    if sigma > 0.0:
        x = x + np.random.default_rng(disp_seed).normal(0.0, sigma, size=x.shape)
    return Atoms(x=wrap(x, box), types=np.ascontiguousarray(types), box=box,
                 masses=np.asarray(masses, np.float64))


def maxwell_boltzmann(atoms: Atoms, temperature: float, seed: int) -> np.ndarray:
    """Velocities ~ N(0, kT/(m*xi)) per component, zero total momentum, rescaled to exactly T.

    Uses 3N-3 degrees of freedom for the temperature.
    """
    n = atoms.n
    m = atoms.masses[atoms.types]
    rng = np.random.default_rng(seed)
    std = np.sqrt(BOLTZMANN_EV_PER_K * temperature / (m * AMU_A2_FS2_IN_EV))
    v = rng.normal(0.0, 1.0, size=(n, 3)) * std[:, None]
    p = (m[:, None] * v).sum(axis=0)
    v = v - p / m.sum()
    ke = 0.5 * AMU_A2_FS2_IN_EV * float((m[:, None] * v * v).sum())
    dof = 3 * n - 3
    t_now = 2.0 * ke / (dof * BOLTZMANN_EV_PER_K)
    if t_now > 0.0:
        v = v * np.sqrt(temperature / t_now)
    return np.ascontiguousarray(v)


# --------------------------------------------------------------------------------------
# Model hyperparameters and packed parameter vector.
#
# Packed FP64 layout (the same contract the C-ABI documents):
#   cR    [T][T][n_max_R+1][basis_R+1]   radial expansion coefficients, (center, neighbor)
#   cA    [T][T][n_max_A+1][basis_A+1]   angular expansion coefficients
#   sigma [D]                            descriptor scaler
#   W0    [H][D]                         hidden weights, row = hidden unit
#   b0    [H]
#   w1    [H]
#   b1    [1]
# with D = (n_max_R+1) + (n_max_A+1)*l_max_3b + (n_max_A+1 if l_max_4b == 2 else 0).
# --------------------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class HParams:
    n_types: int = 1
    rc_radial: float = 6.0
    rc_angular: float = 5.0
    n_max_radial: int = 4
    n_max_angular: int = 4
    basis_radial: int = 8
    basis_angular: int = 8
    l_max_3b: int = 4
    l_max_4b: int = 2
    n_hidden: int = 30
    # ZBL repulsion (Section VI.A): outer switching radius (0 = none), inner radius
    # (None = half the outer one) and the atomic number of each species
    zbl_outer: float = 0.0
    zbl_inner_radius: Optional[float] = None
    zbl_z: Tuple[float, ...] = (29.0, 29.0)

    @property
    def zbl_inner(self) -> float:
        return 0.5 * self.zbl_outer if self.zbl_inner_radius is None else self.zbl_inner_radius

    @property
    def n_desc(self) -> int:
        nr = self.n_max_radial + 1
        na = self.n_max_angular + 1
        return nr + na * self.l_max_3b + (na if self.l_max_4b == 2 else 0)

    def int_array(self) -> np.ndarray:
        return np.array([self.n_types, self.n_max_radial, self.n_max_angular,
                         self.basis_radial, self.basis_angular, self.l_max_3b,
                         self.l_max_4b, self.n_hidden], dtype=np.int32)

    def real_array(self) -> np.ndarray:
        z = list(self.zbl_z) + [0.0] * (2 - len(self.zbl_z))
        return np.array([self.rc_radial, self.rc_angular, self.zbl_inner, self.zbl_outer, z[0], z[1]],
                        dtype=np.float64)

    def sizes(self) -> dict:
        t = self.n_types
        nr, na = self.n_max_radial + 1, self.n_max_angular + 1
        kr, ka = self.basis_radial + 1, self.basis_angular + 1
        d, h = self.n_desc, self.n_hidden
        return {"cR": t * t * nr * kr, "cA": t * t * na * ka, "sigma": d,
                "W0": h * d, "b0": h, "w1": h, "b1": 1}

    def n_params(self) -> int:
        return int(sum(self.sizes().values()))

    def offsets(self) -> dict:
        off, out = 0, {}
        for k, v in self.sizes().items():
            out[k] = (off, off + v)
            off += v
        return out


def save_model(path: str, hp: HParams, params: np.ndarray) -> None:
    """Write a model as .npz: the hyperparameters as JSON text and the packed FP64
    parameters (no pickled objects, so np.load's default allow_pickle=False reads it)."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    if params.size != hp.n_params():
        raise ValueError(f"{params.size} parameters for a model of {hp.n_params()}")
    np.savez(path, hparams=np.array(json.dumps(dataclasses.asdict(hp))), params=params)


def load_model(path: str) -> tuple[HParams, np.ndarray]:
    with np.load(path) as d:
        fields = json.loads(str(d["hparams"]))
        fields["zbl_z"] = tuple(fields["zbl_z"])
        hp = HParams(**fields)
        params = np.array(d["params"], dtype=np.float64)
    if params.size != hp.n_params():
        raise ValueError(f"{path}: {params.size} parameters for a model of {hp.n_params()}")
    return hp, params


FULL_HPARAMS = HParams()
SURROGATE_HPARAMS = HParams(l_max_3b=2, l_max_4b=0, n_hidden=8)
# The same surrogate with 5 / 4 A cutoffs: fewer pairs, so a cheaper inner step.
SURROGATE_SHORT_HPARAMS = HParams(rc_radial=5.0, rc_angular=4.0, l_max_3b=2, l_max_4b=0, n_hidden=8)
# 4 / 3 A: two radial neighbour shells and one angular shell of FCC Cu (a = 3.615 A).
SURROGATE_SHORTER_HPARAMS = HParams(rc_radial=4.0, rc_angular=3.0, l_max_3b=2, l_max_4b=0, n_hidden=8)

# Descriptor scaler of the synthetic models, one constant per descriptor block
# (radial, angular l = 1..4, four-body). The constants were chosen once so that
# scaled descriptors are of order one for thermally disordered FCC boxes at the
# cutoffs above; they are part of the model definition, not derived at run time.
SIGMA_RADIAL = 0.3
SIGMA_ANGULAR = (2.0, 2.0, 2.0, 2.0)
SIGMA_FOURBODY = 10.0


def default_sigma(hp: HParams) -> np.ndarray:
    nr, na = hp.n_max_radial + 1, hp.n_max_angular + 1
    parts = [np.full(nr, SIGMA_RADIAL)]
    for l in range(1, hp.l_max_3b + 1):
        parts.append(np.full(na, SIGMA_ANGULAR[l - 1]))
    if hp.l_max_4b == 2:
        parts.append(np.full(na, SIGMA_FOURBODY))
    return np.concatenate(parts).astype(np.float64)


def random_model(hp: HParams, seed: int, std: float = 0.1,
                 sigma: Optional[np.ndarray] = None) -> np.ndarray:
    """Packed parameters: cR, cA, W0, b0, w1, b1 drawn N(0, std) in that order from one stream."""
    rng = np.random.default_rng(seed)
    s = hp.sizes()
    cR = rng.normal(0.0, std, s["cR"])
    cA = rng.normal(0.0, std, s["cA"])
    W0 = rng.normal(0.0, std, s["W0"])
    b0 = rng.normal(0.0, std, s["b0"])
    w1 = rng.normal(0.0, std, s["w1"])
    b1 = rng.normal(0.0, std, s["b1"])
    sig = default_sigma(hp) if sigma is None else np.asarray(sigma, np.float64)
    return np.ascontiguousarray(np.concatenate([cR, cA, sig, W0, b0, w1, b1]))


def unpack(hp: HParams, params: np.ndarray) -> dict:
    """Views of the packed vector by block name (no arithmetic)."""
    return {k: params[a:b] for k, (a, b) in hp.offsets().items()}


def surrogate_from_teacher(teacher_hp: HParams, teacher: np.ndarray, sur_hp: HParams,
                           seed: int, std: float = 0.1) -> np.ndarray:
    """Surrogate initial parameters: expansion coefficients copied from the teacher, network drawn.

    The surrogate keeps the teacher's channel counts and basis sizes, so its coefficient
    blocks have the teacher's shape and values (with shorter cutoffs they expand the
    basis over the shorter range); its scaler keeps the teacher's radial and l <= l_max
    entries; the network is drawn N(0, std) from ``seed``.
    """
    assert (sur_hp.n_types, sur_hp.n_max_radial, sur_hp.n_max_angular, sur_hp.basis_radial,
            sur_hp.basis_angular) == (teacher_hp.n_types, teacher_hp.n_max_radial,
                                      teacher_hp.n_max_angular, teacher_hp.basis_radial,
                                      teacher_hp.basis_angular)
    tb = unpack(teacher_hp, teacher)
    rng = np.random.default_rng(seed)
    s = sur_hp.sizes()
    nr = sur_hp.n_max_radial + 1
    na = sur_hp.n_max_angular + 1
    sig = tb["sigma"][: nr + na * sur_hp.l_max_3b].copy()
    W0 = rng.normal(0.0, std, s["W0"])
    b0 = rng.normal(0.0, std, s["b0"])
    w1 = rng.normal(0.0, std, s["w1"])
    b1 = rng.normal(0.0, std, s["b1"])
    return np.ascontiguousarray(np.concatenate([tb["cR"], tb["cA"], sig, W0, b0, w1, b1]))


# --------------------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------------------

def workload_small(seed_disp: int = 11, seed_vel: int = 12) -> Atoms:
    """10^3 FCC cells (4,000 atoms), sigma 0.05 A, 300 K."""
    at = fcc_box(10, 0.05, seed_disp)
    at.v = maxwell_boltzmann(at, 300.0, seed_vel)
    return at


def workload_4m(n_cells: int = 100) -> Atoms:
    """100^3 FCC cells (4,000,000 atoms), sigma 0.08 A, 600 K."""
    at = fcc_box(n_cells, 0.08, 21)
    at.v = maxwell_boltzmann(at, 600.0, 22)
    return at


def workload_alloy(n_cells: int = 60, vacancy_fraction: float = 0.05) -> Atoms:
    """60^3-cell two-species alloy (864,000 sites) with 5% vacancies, sigma 0.05 A, 300 K."""
    n_sites = 4 * n_cells ** 3
    at = alloy_box(n_cells, 31, int(round(vacancy_fraction * n_sites)), 32, 0.05, 33)
    at.v = maxwell_boltzmann(at, 300.0, 34)
    return at


def workload_disordered_frames(n_cells: int = 20, n_frames: int = 16, first_seed: int = 40,
                               sigma: float = 0.17, temperature: float = 1200.0) -> list[Atoms]:
    """Thermally disordered FCC frames (1200 K: sigma 0.17 A displacements, MB velocities)."""
    out = []
    for f in range(n_frames):
        at = fcc_box(n_cells, sigma, first_seed + f)
        at.v = maxwell_boltzmann(at, temperature, 1000 + first_seed + f)
        out.append(at)
    return out


def workload_32m(n_cells: int = 200) -> Atoms:
    """200^3 FCC cells (32,000,000 atoms), sigma 0.08 A, 600 K."""
    at = fcc_box(n_cells, 0.08, 51)
    at.v = maxwell_boltzmann(at, 600.0, 52)
    return at


def sample_ids(n: int, k: int, seed: int) -> np.ndarray:
    """``k`` distinct atom ids in ascending order."""
    k = min(k, n)
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False)).astype(np.int64)
