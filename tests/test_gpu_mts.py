"""Multiple time stepping with the surrogate, its fallback, and surrogate training on the GPU."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, min_image_diff, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def models():
    hp = I.FULL_HPARAMS
    teacher = I.random_model(hp, 0)
    shp = I.SURROGATE_HPARAMS
    sur = I.surrogate_from_teacher(hp, teacher, shp, 1)
    return hp, teacher, shp, sur


@pytest.mark.parametrize("cutoffs", ["teacher", "short", "shorter"])
def test_mts_blocks_match_oracle_rrespa(models, cutoffs):
    """'shorter' (4 / 3 A) brings the two models' bin edges to 17, so the list keeps 16."""
    hp, teacher, shp, sur = models
    if cutoffs != "teacher":
        shp = I.SURROGATE_SHORT_HPARAMS if cutoffs == "short" else I.SURROGATE_SHORTER_HPARAMS
        sur = I.surrogate_from_teacher(hp, teacher, shp, 1)
    at = I.workload_small()
    say(f"case: MTS k=4, 3 blocks, 4000 atoms, untrained surrogate ({cutoffs} cutoffs), no fallback")
    s = make_system(at, hp, teacher, shp, sur)
    th = s.step(12, dt=1.0, rebuild_every=10, skin=1.0, mts_k=4, fallback_rms=1e9, fallback_max=1e9,
                thermo_every=4)
    x, v, step = s.get_state()
    xo, vo, err = oracle.mts(oracle.Model.from_hparams(hp, teacher), oracle.Model.from_hparams(shp, sur),
                             at.x, at.v, at.types, at.masses, at.box, 1.0, 4, 3)
    dx = np.abs(min_image_diff(x, xo, at.box)).max()
    say(f"  max|dx|={dx:.2e}; block errors gpu={th[:, 5:7].tolist()} oracle={err.tolist()}")
    assert step == 12 and dx < 1e-6 and np.abs(v - vo).max() < 1e-7
    assert np.allclose(th[:, 5], err[:, 0], rtol=1e-4) and np.allclose(th[:, 6], err[:, 1], rtol=1e-4)
    assert s.stats()["mts_blocks"] == 3 and s.stats()["fallback_blocks"] == 0


def test_mts_with_identical_models_is_velocity_verlet(models):
    hp, teacher, _, _ = models
    at = I.workload_small()
    say("case: MTS with surrogate = full model")
    s = make_system(at, hp, teacher, hp, teacher)
    s.step(8, mts_k=4, fallback_rms=1e9, fallback_max=1e9)
    x, v, _ = s.get_state()
    xo, vo, _ = oracle.velocity_verlet(oracle.Model.from_hparams(hp, teacher), at.x, at.v, at.types, at.masses,
                                       at.box, 1.0, 8)
    assert np.abs(min_image_diff(x, xo, at.box)).max() < 1e-6 and np.abs(v - vo).max() < 1e-7


def test_mts_fallback_engages(models):
    hp, teacher, shp, sur = models
    zero = sur.copy()
    zero[shp.offsets()["W0"][0]:] = 0.0   # network output constant: surrogate forces vanish
    at = I.workload_small()
    say("case: MTS fallback with a zero-force surrogate")
    s = make_system(at, hp, teacher, shp, zero)
    th = s.step(12, mts_k=4, fallback_rms=1e-3, fallback_max=1e9, thermo_every=4)
    st = s.stats()
    assert st["mts_blocks"] == 1 and st["fallback_blocks"] == 2 and th[0, 7] == 1
    x, v, _ = s.get_state()
    mf = oracle.Model.from_hparams(hp, teacher)
    x1, v1, _ = oracle.mts(mf, oracle.Model.from_hparams(shp, zero), at.x, at.v, at.types, at.masses, at.box,
                           1.0, 4, 1)
    xo, vo, _ = oracle.velocity_verlet(mf, x1, v1, at.types, at.masses, at.box, 1.0, 8)
    assert np.abs(min_image_diff(x, xo, at.box)).max() < 1e-6


def test_relative_judge_follows_the_full_force_scale(models):
    """With a zero-force surrogate the block's rms error equals the rms full-model force
    exactly, so a relative threshold just below 1 falls back at the first block and one
    just above 1 never does."""
    hp, teacher, shp, sur = models
    zero = sur.copy()
    zero[shp.offsets()["W0"][0]:] = 0.0
    at = I.workload_small()
    for frac, mts, fb in ((0.999, 1, 2), (1.001, 3, 0)):
        say(f"case: relative judge {frac} x rms(F_full), zero-force surrogate")
        s = make_system(at, hp, teacher, shp, zero)
        th = s.step(12, mts_k=4, fallback_rms=frac, fallback_max=1e9, thermo_every=4, relative_judge=True)
        st = s.stats()
        assert st["mts_blocks"] == mts and st["fallback_blocks"] == fb, (frac, st)
        assert th[0, 7] == (1 if fb else 0)


def test_surrogate_training_and_gain(models):
    """Trained surrogate against the untrained one: lower force error against the full model,
    and an MTS run whose judge accepts the trained surrogate but falls back for the untrained."""
    from paper_2604_24816_amd import surrogate as SG
    hp, teacher, shp, sur0 = models
    say("case: frames from full-NEP MD (40 trajectories x 10 frames, 4000 atoms) and GPU training")
    fr = SG.generate_frames(hp, teacher, n_traj=40, cells=10, steps=100, every=10)
    res = SG.train_surrogate(fr, shp, sur0, epochs=6, batch=8, lr=1e-2, log=say)
    say(f"  val force RMSE {res.val_force_rmse_init:.4e} -> {res.val_force_rmse:.4e} eV/A; "
        f"energy MAE {res.val_energy_mae_init:.3e} -> {res.val_energy_mae:.3e} eV/atom; {res.seconds:.1f} s")
    assert res.history[-1] < res.history[0]
    assert res.val_force_rmse < 0.8 * res.val_force_rmse_init
    # judge thresholds from the full model's force scale (0.75 x rms force)
    at = I.fcc_box(10, 0.083 * np.sqrt(2.0), 977)
    at.v = I.maxwell_boltzmann(at, 600.0, 978)
    runs = {}
    for name, p in (("untrained", sur0), ("trained", res.params)):
        s = make_system(at, hp, teacher, shp, p)
        tau_rms, tau_max, rms = SG.judge_thresholds(s)
        th = s.step(40, mts_k=4, fallback_rms=tau_rms, fallback_max=tau_max, thermo_every=4)
        runs[name] = (s.stats(), float(np.mean(th[:, 5])))
        say(f"  {name}: mean block rms error {runs[name][1]:.4e} eV/A, stats {runs[name][0]}")
    assert runs["trained"][1] < runs["untrained"][1]
    assert runs["trained"][0]["fallback_blocks"] < runs["untrained"][0]["fallback_blocks"]


def test_coefficient_training_beats_network_only(models):
    """Training the expansion coefficients as well as the network lowers the 5 / 4 A
    surrogate's held-out force error against the full model, at equal epochs."""
    from paper_2604_24816_amd import surrogate as SG
    hp, teacher, _, _ = models
    shp = I.SURROGATE_SHORT_HPARAMS
    sur0 = I.surrogate_from_teacher(hp, teacher, shp, 1)
    say("case: 5/4 A surrogate, network-only against coefficient training (40 x 10 frames, 6 epochs)")
    fr = SG.generate_frames(hp, teacher, n_traj=40, cells=10, steps=100, every=10)
    nn = SG.train_surrogate(fr, shp, sur0, epochs=6, batch=8, lr=1e-2)
    co = SG.train_surrogate(fr, shp, sur0, epochs=6, batch=8, lr=1e-2, train_coeffs=True)
    say(f"  held-out force RMSE: start {nn.val_force_rmse_init:.4e}, network only {nn.val_force_rmse:.4e}, "
        f"with coefficients {co.val_force_rmse:.4e} eV/A")
    assert co.val_force_rmse < 0.85 * nn.val_force_rmse
    o = shp.offsets()
    a, b = o["sigma"]
    assert np.array_equal(co.params[a:b], sur0[a:b])              # the scaler stays fixed
    assert np.abs(co.params[:a] - sur0[:a]).max() > 1e-3          # the coefficients moved


def test_shorter_surrogate_is_accepted_once_trained(models):
    """The 4/3 A surrogate of the MTS form (the two nearest radial shells, the nearest
    angular one), coefficients and network trained on the GPU, in r-RESPA with k = 4 on a
    600 K 10^3-cell box under the relative judge (block rms error <= 0.75 x the block's rms
    full-model force, max <= 10 x): accepted in all 6 blocks, while the untrained one
    fails the first block and falls back to the full model for the rest."""
    from paper_2604_24816_amd import surrogate as SG
    hp, teacher, _, _ = models
    shp = I.SURROGATE_SHORTER_HPARAMS
    sur0 = I.surrogate_from_teacher(hp, teacher, shp, 1)
    say("case: 4/3 A surrogate, coefficients + network trained (100 x 10 frames, 30 epochs), relative judge")
    fr = SG.generate_frames(hp, teacher, n_traj=100, cells=10, steps=100, every=10)
    res = SG.train_surrogate(fr, shp, sur0, epochs=30, batch=8, lr=1e-2, lr_end=1e-4, train_coeffs=True)
    say(f"  held-out force RMSE {res.val_force_rmse_init:.4e} -> {res.val_force_rmse:.4e} eV/A ({res.seconds:.1f} s)")
    at = I.fcc_box(10, 0.08, 61)
    at.v = I.maxwell_boltzmann(at, 600.0, 62)
    runs = {}
    for name, p in (("untrained", sur0), ("trained", res.params)):
        s = make_system(at, hp, teacher, shp, p)
        th = s.step(24, mts_k=4, fallback_rms=0.75, fallback_max=10.0, thermo_every=4, relative_judge=True)
        runs[name] = (s.stats(), th)
        say(f"  {name}: stats {runs[name][0]}, block rms errors {np.round(th[:, 5], 5).tolist()}, "
            f"fallback flags {th[:, 7].astype(int).tolist()}")
    st, th = runs["trained"]
    assert st["mts_blocks"] == 6 and st["fallback_blocks"] == 0
    st0, th0 = runs["untrained"]
    assert st0["mts_blocks"] == 1 and st0["fallback_blocks"] == 5 and th0[0, 7] == 1
    assert th[:, 5].mean() < 0.5 * th0[:, 5].mean()
