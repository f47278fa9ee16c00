"""Checkpoint / resume and run-to-run agreement on the GPU.

Resuming rebuilds the lists at the checkpoint, so entries come in another order and
FP32 forces are summed in another order: trajectories agree to rounding (a force
difference of ~1e-7 eV/A moves atoms by ~1e-11 A in 5 fs), not bit for bit. The
angular reaction forces are added with LDS atomics, whose order can change between
runs; two evaluations of the same state must agree within 1e-6 eV/A.
"""
import numpy as np
import pytest

from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, min_image_diff, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    hp = I.FULL_HPARAMS
    return hp, I.random_model(hp, 0)


@pytest.mark.parametrize("nvt", [False, True])
def test_resume_from_checkpoint(model, nvt):
    hp, params = model
    at = I.workload_small()
    at.v = I.maxwell_boltzmann(at, 600.0, 14)
    say(f"case: 10 steps against 5 + checkpoint + 5, {'NVT' if nvt else 'NVE'}")
    a = make_system(at, hp, params)
    if nvt:
        a.set_thermostat(300.0, tau=20.0, chain=3)
    a.step(10)
    xa, va, _ = a.get_state()
    b = make_system(at, hp, params)
    if nvt:
        b.set_thermostat(300.0, tau=20.0, chain=3)
    b.step(5)
    x5, v5, step5 = b.get_state()
    assert step5 == 5
    c = make_system(I.Atoms(x=x5, types=at.types, box=at.box, masses=at.masses, v=v5), hp, params)
    if nvt:
        eta, ve, _ = b.get_thermostat()
        c.set_thermostat(300.0, tau=20.0, chain=3)
        c.set_thermostat_state(eta, ve)
    c.step(5)
    xc, vc, _ = c.get_state()
    dx, dv = np.abs(min_image_diff(xc, xa, at.box)).max(), np.abs(vc - va).max()
    say(f"  max|dx|={dx:.2e} max|dv|={dv:.2e}")
    assert dx < 1e-8 and dv < 1e-9
    if nvt:
        ea, vea, _ = a.get_thermostat()
        ec, vec, _ = c.get_thermostat()
        assert np.abs(ec - ea).max() < 1e-9 * np.abs(ea).max() and np.abs(vec - vea).max() < 1e-9 * np.abs(vea).max()


def test_repeated_evaluations_agree(model):
    hp, params = model
    at = I.workload_small()
    say("case: the same state evaluated twice")
    s = make_system(at, hp, params)
    E1, W1, F1, U1 = s.compute(per_atom=True)
    E2, W2, F2, U2 = s.compute(per_atom=True)
    say(f"  max|dF|={np.abs(F1 - F2).max():.2e} |dE|={abs(E1 - E2):.2e}")
    assert np.array_equal(U1, U2) and E1 == E2        # no atomics in the energies
    assert np.abs(F1 - F2).max() < 1e-6 and np.abs(W1 - W2).max() < 1e-6 * at.n
