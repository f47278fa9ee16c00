"""Parity at the 32,000,000-atom size of the production forms (200^3 FCC cells, 600 K).

The oracle evaluates 10,000 sampled atoms one by one for the plain FP32 form, the
BF16 network form (against the oracle's own bfloat16 model) and the 5 / 4 A
surrogate; an MTS run of four r-RESPA blocks then keeps momentum, stays finite and
its final full-model forces match the oracle on the same sampled atoms.
"""
import numpy as np
import pytest

import oracle
from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, say

pytestmark = pytest.mark.gpu


def test_32m_forms_sampled_parity():
    hp = I.FULL_HPARAMS
    params = I.random_model(hp, 0)
    shp = I.SURROGATE_SHORT_HPARAMS
    sur = I.surrogate_from_teacher(hp, params, shp, 1)
    say("case: building the 200^3-cell FCC box (32,000,000 atoms)")
    at = I.workload_32m()
    s = make_system(at, hp, params, shp, sur, cap_radial=160, cap_angular=96)
    m = oracle.Model.from_hparams(hp, params)
    ms = oracle.Model.from_hparams(shp, sur)
    sel = I.sample_ids(at.n, 10000, 53)
    say("case: 32M atoms, fp32 / bf16 / surrogate against the oracle on 10,000 sampled atoms")
    E, W, F, U = s.compute(per_atom=True)
    Us, Fs = oracle.evaluate_sampled(m, at.x, at.types, at.box, sel)
    du, df = np.abs(U[sel] - Us).max(), np.abs(F[sel] - Fs).max()
    say(f"  fp32: max|dU|={du:.2e} max|dF|={df:.2e}")
    assert du < 1e-6 and df < 1e-4
    _, _, Fb, Ub = s.compute(precision="bf16", per_atom=True)
    Ubs, Fbs = oracle.evaluate_sampled(m, at.x, at.types, at.box, sel, bf16=True)
    say(f"  bf16 vs oracle bf16 model: mean|dU|={np.abs(Ub[sel] - Ubs).mean():.2e} "
        f"max|dU|={np.abs(Ub[sel] - Ubs).max():.2e} max|dF|={np.abs(Fb[sel] - Fbs).max():.2e}")
    assert np.abs(Ub[sel] - Ubs).mean() < 2e-6 and np.abs(Ub[sel] - Ubs).max() < 5e-4
    assert np.abs(Fb[sel] - Fbs).max() < 5e-3
    _, _, Fsur, Usur = s.compute(slot=1, per_atom=True)
    Uss, Fss = oracle.evaluate_sampled(ms, at.x, at.types, at.box, sel)
    dus, dfs = np.abs(Usur[sel] - Uss).max(), np.abs(Fsur[sel] - Fss).max()
    say(f"  surrogate 5/4 A: max|dU|={dus:.2e} max|dF|={dfs:.2e}")
    assert dus < 1e-6 and dfs < 1e-4
    say("case: 32M atoms, 4 MTS blocks (k = 4), fallback off")
    s.step(16, mts_k=4, fallback_rms=1e9, fallback_max=1e9)
    x, v, step = s.get_state()
    mass = at.masses[at.types]
    p = (mass[:, None] * v).sum(0)
    assert step == 16 and np.isfinite(x).all() and np.abs(p).max() < 1e-6 * at.n
    _, _, F2, U2 = s.compute(per_atom=True)
    U2s, F2s = oracle.evaluate_sampled(m, x, at.types, at.box, sel)
    du2, df2 = np.abs(U2[sel] - U2s).max(), np.abs(F2[sel] - F2s).max()
    say(f"  after MTS: |P|={np.abs(p).max():.2e}; full model max|dU|={du2:.2e} max|dF|={df2:.2e}")
    assert du2 < 1e-6 and df2 < 1e-4
