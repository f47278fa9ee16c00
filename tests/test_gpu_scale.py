"""Parity at the full 4,000,000-atom size, in the launch configuration the benchmark times.

The oracle evaluates per-atom energies of every atom (total energy per atom) and
forces of 2,000 sampled atoms one by one; properties that hold at any size
(momentum conservation, NVE energy conservation) cover the integrated run.
"""
import numpy as np
import pytest

import oracle
from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    hp = I.FULL_HPARAMS
    params = I.random_model(hp, 0)
    say("case: building the 100^3-cell FCC box (4,000,000 atoms)")
    at = I.workload_4m()
    s = make_system(at, hp, params)
    return hp, params, at, s


def test_sampled_atoms_and_total_energy_4m(big):
    hp, params, at, s = big
    m = oracle.Model.from_hparams(hp, params)
    say("case: 4M atoms fp32 evaluation vs oracle (2000 sampled atoms + all per-atom energies)")
    E, W, F, U = s.compute(per_atom=True)
    sel = I.sample_ids(at.n, 2000, 23)
    Us, Fs = oracle.evaluate_sampled(m, at.x, at.types, at.box, sel)
    du = np.abs(U[sel] - Us).max()
    df = np.abs(F[sel] - Fs).max()
    Uall, _, _ = oracle.energies(m, at.x, at.types, at.box)
    de = abs(E - Uall.sum()) / at.n
    say(f"  sampled max|dU|={du:.2e} max|dF|={df:.2e}; |dE|/N={de:.2e}")
    assert du < 1e-6 and df < 1e-4 and de < 1e-6
    assert np.abs(U - Uall).max() < 1e-6


def test_nve_run_4m_conserves_momentum_and_energy(big):
    hp, params, at, s = big
    say("case: 4M atoms, 20 NVE steps, rebuild every 10")
    th = s.step(20, dt=1.0, rebuild_every=10, skin=1.0, thermo_every=10)
    x, v, step = s.get_state()
    mass = at.masses[at.types]
    p = (mass[:, None] * v).sum(0)
    etot = th[:, 1] + th[:, 2]
    say(f"  |P|={np.abs(p).max():.2e} amu A/fs, E_tot rows={etot}")
    assert np.abs(p).max() < 1e-6 * at.n
    assert abs(etot[-1] - etot[0]) / at.n < 1e-5
    assert np.isfinite(x).all()


def test_alloy_820k_fp32_and_bf16_errors_against_fp64():
    """Two-species 60^3-cell alloy with 5% vacancies (820,800 atoms): FP32 and BF16 forms
    against the FP64 oracle over every atom; the errors are printed (stated) and bounded."""
    hp = I.HParams(n_types=2)
    params = I.random_model(hp, 0)
    m = oracle.Model.from_hparams(hp, params)
    at = I.workload_alloy()
    say(f"case: alloy 60^3 cells, 5% vacancies, N={at.n}")
    s = make_system(at, hp, params)
    Eo, Wo, Uo, Fo = oracle.evaluate(m, at.x, at.types, at.box)
    _, _, Ub, Fb = oracle.evaluate(m, at.x, at.types, at.box, bf16=True)
    off, _ = s.export_neighbors(1)
    cnt = np.diff(off)
    say(f"  angular list (skin) counts p50={np.percentile(cnt, 50):.0f} p90={np.percentile(cnt, 90):.0f} "
        f"max={cnt.max()}; rms|F|={np.sqrt(np.mean(Fo ** 2)):.3e} eV/A")
    res = {}
    for prec in ("fp32", "bf16"):
        E, W, F, U = s.compute(precision=prec, per_atom=True)
        dU = np.abs(U - Uo)
        dF = np.abs(F - Fo)
        res[prec] = (dU.max(), dU.mean(), abs(E - Eo) / at.n, dF.max(), np.sqrt(np.mean((F - Fo) ** 2)),
                     np.abs(W - Wo).max() / at.n)
        say(f"  {prec} vs FP64: max|dU|={res[prec][0]:.2e} mean|dU|={res[prec][1]:.2e} |dE|/N={res[prec][2]:.2e} "
            f"max|dF|={res[prec][3]:.2e} rms dF={res[prec][4]:.2e} max|dW|/N={res[prec][5]:.2e}")
        if prec == "bf16":
            say(f"  bf16 vs oracle bf16 model: max|dU|={np.abs(U - Ub).max():.2e} "
                f"mean|dU|={np.abs(U - Ub).mean():.2e} max|dF|={np.abs(F - Fb).max():.2e}")
    assert res["fp32"][0] < 1e-6 and res["fp32"][2] < 1e-6 and res["fp32"][3] < 1e-4
    assert res["bf16"][0] < 5e-2 and res["bf16"][3] < 5e-2
