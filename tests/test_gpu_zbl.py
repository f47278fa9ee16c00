"""ZBL repulsion on the GPU (through the C-ABI) against the FP64 oracle.

Compressed FCC boxes put many pairs inside the ZBL radius (nearest neighbours at
2.1 A against an outer radius of 2.0 or 2.4 A). Bars: those of the plain model
(energies within 1e-6 eV per atom, forces within 1e-4 eV/A, virial within 1e-6 eV
per atom) plus a relative term of 5e-7 (about eight FP32 roundings) of the largest
per-atom energy, force or virial component: with the inner radius at 2.05 A an
atom's ZBL energy reaches ~30 eV, where one FP32 rounding is already 2e-6 eV.
"""
import numpy as np
import pytest

import oracle
from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, min_image_diff, say

pytestmark = pytest.mark.gpu


def _compressed(at, scale=0.82):
    return I.Atoms(x=at.x * scale, types=at.types, box=at.box * scale, masses=at.masses, v=at.v)


REL = 5e-7


def _check(s, m, at):
    E, W, F, U = s.compute(per_atom=True)
    Eo, Wo, Uo, Fo = oracle.evaluate(m, at.x, at.types, at.box)
    du, de = np.abs(U - Uo).max(), abs(E - Eo) / at.n
    df, dw = np.abs(F - Fo).max(), np.abs(W - Wo).max() / at.n
    e_tol = 1e-6 + REL * np.abs(Uo).max()
    f_tol = 1e-4 + REL * np.abs(Fo).max()
    w_tol = 1e-6 + REL * np.abs(Wo).max() / at.n
    say(f"  N={at.n}: max|dU|={du:.2e} |dE|/N={de:.2e} max|dF|={df:.2e} max|dW|/N={dw:.2e} "
        f"(bars {e_tol:.1e}, {f_tol:.1e}, {w_tol:.1e}; max|U| {np.abs(Uo).max():.1f} eV)")
    assert du < e_tol and de < e_tol and df < f_tol and dw < w_tol, (du, de, df, dw)


@pytest.mark.parametrize("outer,inner", [(2.0, None), (2.4, 2.05)])
def test_zbl_energy_forces_virial(outer, inner):
    hp = I.HParams(zbl_outer=outer, zbl_inner_radius=inner)
    params = I.random_model(hp, 0)
    m = oracle.Model.from_hparams(hp, params)
    at = _compressed(I.fcc_box(6, 0.12, 17))
    close, _ = oracle.neighbors(at.x, at.box, outer)
    say(f"case: ZBL outer {outer} inner {hp.zbl_inner}, compressed FCC 6^3, {close.sum() // 2} close pairs")
    assert close.sum() > 100
    s = make_system(at, hp, params, cap_radial=320, cap_angular=200)
    _check(s, m, at)
    # the same positions without ZBL: the difference is the ZBL energy alone
    hp0 = I.HParams()
    s0 = make_system(at, hp0, params, cap_radial=320, cap_angular=200)
    E0 = s0.compute()[0]
    E = s.compute()[0]
    Eo0 = oracle.evaluate(oracle.Model.from_hparams(hp0, params), at.x, at.types, at.box)[0]
    Eo = oracle.evaluate(m, at.x, at.types, at.box)[0]
    say(f"  ZBL energy: gpu {E - E0:.6e} oracle {Eo - Eo0:.6e} eV")
    assert abs((E - E0) - (Eo - Eo0)) < (1e-6 + REL * abs(Eo - Eo0) / at.n) * at.n and abs(Eo - Eo0) > 1.0


def test_zbl_two_species():
    hp = I.HParams(n_types=2, zbl_outer=2.0, zbl_z=(29.0, 79.0))
    params = I.random_model(hp, 8)
    m = oracle.Model.from_hparams(hp, params)
    at = _compressed(I.alloy_box(6, 1, 30, 2, 0.12, 3))
    say(f"case: ZBL Cu-Au, compressed alloy, N={at.n}")
    s = make_system(at, hp, params, cap_radial=320, cap_angular=200)
    _check(s, m, at)


def test_zbl_velocity_verlet():
    """Ten steps of NVE with close contacts: positions and velocities follow the oracle."""
    hp = I.HParams(zbl_outer=2.0)
    params = I.random_model(hp, 0)
    at = _compressed(I.fcc_box(6, 0.12, 17))
    at.v = I.maxwell_boltzmann(at, 600.0, 5)
    say("case: ZBL NVE, 10 steps of 1 fs")
    s = make_system(at, hp, params, cap_radial=320, cap_angular=200)
    s.step(10, dt=1.0, rebuild_every=10, skin=1.0)
    x, v, _ = s.get_state()
    xo, vo, _ = oracle.velocity_verlet(oracle.Model.from_hparams(hp, params), at.x, at.v, at.types, at.masses,
                                       at.box, 1.0, 10)
    dx, dv = np.abs(min_image_diff(x, xo, at.box)).max(), np.abs(v - vo).max()
    say(f"  max|dx|={dx:.2e} max|dv|={dv:.2e}")
    assert dx < 1e-6 and dv < 1e-6
