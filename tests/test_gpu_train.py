"""Weight gradients, the autograd Function and Adam on the GPU, against the FP64 oracle.

The oracle's weight gradients are pinned to central finite differences in the CPU
suite; here the GPU's FP32 kernels (FP64 reduction over atoms) must match them.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_24816_amd import inputs as I
from tests.gpu_helpers import make_system, say

pytestmark = pytest.mark.gpu


def _nn(hp, params):
    from paper_2604_24816_amd import nep
    return torch.tensor(nep.network_params(hp, params), dtype=torch.float32, device="cuda")


def _noisy(hp, params, seed, std=0.01):
    """Network block of ``params`` plus N(0, std) noise (the descriptor block is kept)."""
    p = params.copy()
    a, b = hp.offsets()["W0"][0], hp.n_params()
    p[a:b] += np.random.default_rng(seed).normal(0.0, std, b - a)
    return p


def _compare(g_gpu, g_ref, label, rel=1e-4, floor=1e-5):
    """Entry by entry: |g - ref| <= rel |ref| + floor max|ref|. The floor is for entries
    that cancel to almost nothing over the atoms, where the FP32 per-atom terms leave an
    absolute error of the block's scale rather than a relative one."""
    scale = np.abs(g_ref).max()
    err = np.abs(g_gpu - g_ref)
    bound = rel * np.abs(g_ref) + floor * scale
    big = np.abs(g_ref) >= 0.01 * scale
    rel_big = float((err[big] / np.abs(g_ref[big])).max())
    k = int(np.argmax(err / bound))
    say(f"  {label}: {g_ref.size} entries, max|grad|={scale:.3e}, max rel err over entries above 1% of it "
        f"{rel_big:.2e}, worst entry {k}: {g_gpu[k]:.6e} vs {g_ref[k]:.6e} ({err[k] / bound[k]:.2f} of its bound)")
    assert (err <= bound).all(), (label, k, g_gpu[k], g_ref[k])


@pytest.mark.parametrize("kind", ["full", "two_species", "surrogate"])
def test_weight_gradient_matches_oracle(kind):
    if kind == "surrogate":
        thp = I.FULL_HPARAMS
        hp = I.SURROGATE_HPARAMS
        params = I.surrogate_from_teacher(thp, I.random_model(thp, 0), hp, 3)
    elif kind == "two_species":
        hp = I.HParams(n_types=2)
        params = I.random_model(hp, 8)
    else:
        hp = I.FULL_HPARAMS
        params = I.random_model(hp, 6)
    at = I.alloy_box(6, 1, 30, 2, 0.17, 3) if kind == "two_species" else I.fcc_box(6, 0.17, 40)
    say(f"case: weight gradient, {kind}, N={at.n}")
    s = make_system(at, hp, params) if kind != "surrogate" else None
    if kind == "surrogate":
        # the surrogate goes in slot 0 of its own system here
        s = make_system(at, hp, params)
    theta = _nn(hp, params)
    rng = np.random.default_rng(5)
    gF = rng.normal(size=(at.n, 3))
    gE = 0.7
    E, F = s.train_forward(0, theta)
    g = s.train_backward(0, theta, gE, torch.tensor(gF, dtype=torch.float32, device="cuda")).cpu().numpy()
    m = oracle.Model.from_hparams(hp, params)
    ref = oracle.weight_grad(m, at.x, at.types, at.box, gE, gF)
    _compare(g, ref, "energy+force loss")
    g0 = s.train_backward(0, theta, gE, None).cpu().numpy()
    ref0 = oracle.weight_grad(m, at.x, at.types, at.box, gE, None)
    _compare(g0, ref0, "energy only")
    # accumulate mode adds
    acc = torch.tensor(g0, device="cuda")
    s.train_backward(0, theta, gE, None, out=acc)
    assert np.allclose(acc.cpu().numpy(), 2 * g0, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kind", ["full", "two_species", "surrogate"])
def test_param_gradient_matches_oracle(kind):
    """Gradient with respect to every parameter (expansion coefficients per species pair,
    scaler, network) against the oracle's, block by block; the forward with the packed
    vector equals the network-only forward."""
    if kind == "surrogate":
        thp = I.FULL_HPARAMS
        hp = I.SURROGATE_HPARAMS
        params = I.surrogate_from_teacher(thp, I.random_model(thp, 0), hp, 3)
    elif kind == "two_species":
        hp = I.HParams(n_types=2)
        params = I.random_model(hp, 8)
    else:
        hp = I.FULL_HPARAMS
        params = I.random_model(hp, 6)
    at = I.alloy_box(6, 1, 30, 2, 0.17, 3) if kind == "two_species" else I.fcc_box(6, 0.17, 40)
    say(f"case: gradient of every parameter, {kind}, N={at.n}")
    s = make_system(at, hp, params)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    E1, F1 = s.train_forward_params(0, pt)
    E0, F0 = s.train_forward(0, _nn(hp, params))
    # same FP32 values; the forces may differ in rounding where LDS atomics reorder sums
    assert abs(E1 - E0) <= 1e-9 * abs(E0) and float((F1 - F0).abs().max()) < 1e-5
    rng = np.random.default_rng(5)
    gF = rng.normal(size=(at.n, 3))
    gE = 0.7
    m = oracle.Model.from_hparams(hp, params)
    o = hp.offsets()
    for with_f in (True, False):
        gFt = torch.tensor(gF, dtype=torch.float32, device="cuda") if with_f else None
        g = s.train_backward_params(0, pt, gE, gFt).cpu().numpy()
        ref = oracle.param_grad(m, at.x, at.types, at.box, gE, gF if with_f else None)
        for name in ("cR", "cA", "sigma"):
            a, b = o[name]
            _compare(g[a:b], ref[a:b], f"{name} ({'energy+force' if with_f else 'energy'})")
        a = o["W0"][0]
        _compare(g[a:], ref[a:], f"network ({'energy+force' if with_f else 'energy'})")
    acc = torch.tensor(g, device="cuda")
    s.train_backward_params(0, pt, gE, None, out=acc)
    assert np.allclose(acc.cpu().numpy(), 2 * g, rtol=1e-6, atol=1e-6)


def test_autograd_function_energy_force_loss_16_frames():
    """Loss of energy + force MSE over 16 thermally disordered 32,000-atom frames."""
    from paper_2604_24816_amd import autograd as AG
    hp = I.FULL_HPARAMS
    teacher = I.random_model(hp, 0)
    student = _noisy(hp, teacher, 56)
    mt = oracle.Model.from_hparams(hp, teacher)
    ms = oracle.Model.from_hparams(hp, student)
    frames = I.workload_disordered_frames(20, 16)
    say(f"case: autograd loss over {len(frames)} frames of {frames[0].n} atoms")
    theta = _nn(hp, student).requires_grad_(True)
    systems, labels, ref = [], [], None
    for f, at in enumerate(frames):
        Et, _, _, Ft = oracle.evaluate(mt, at.x, at.types, at.box)
        labels.append((Et, torch.tensor(Ft, device="cuda")))
        s = make_system(at, hp, student, build=True)
        systems.append((s, None))
        # oracle gradient of this frame's term
        Es, _, _, Fs = oracle.evaluate(ms, at.x, at.types, at.box)
        n = at.n
        gE = 2.0 * (Es - Et) / n / n / len(frames)
        gF = 2.0 * (Fs - Ft) / (3 * n) / len(frames)
        g = oracle.weight_grad(ms, at.x, at.types, at.box, gE, gF)
        ref = g if ref is None else ref + g
    loss = AG.energy_force_loss(systems, theta, labels)
    loss.backward()
    g_gpu = theta.grad.detach().cpu().numpy()
    say(f"  loss={float(loss):.6e}")
    # the loss residuals F_student - F_teacher come from FP32 forces on the GPU and FP64 on the
    # oracle, and they are 1e-3 of the forces themselves (the student is the teacher plus noise)
    _compare(g_gpu, ref, "16-frame loss", rel=1e-3, floor=1e-4)


def test_position_gradient_is_minus_force():
    from paper_2604_24816_amd import autograd as AG
    hp = I.FULL_HPARAMS
    params = I.random_model(hp, 0)
    at = I.fcc_box(5, 0.1, 12)
    say("case: dE/dx through the autograd Function")
    s = make_system(at, hp, params)
    x = torch.tensor(at.x, device="cuda", requires_grad=True)
    theta = _nn(hp, params)
    E, F = AG.energy_forces(s, theta, x)
    E.backward()
    m = oracle.Model.from_hparams(hp, params)
    _, _, _, Fo = oracle.evaluate(m, at.x, at.types, at.box)
    assert np.abs(-x.grad.cpu().numpy() - Fo).max() < 1e-4
    assert abs(float(E.detach()) - oracle.evaluate(m, at.x, at.types, at.box)[0]) / at.n < 1e-6


def test_adam_update_matches_oracle():
    hp = I.FULL_HPARAMS
    at = I.fcc_box(4, 0.05, 1)
    s = make_system(at, hp, I.random_model(hp, 0))
    rng = np.random.default_rng(3)
    n = 961
    th, g = rng.normal(size=n), rng.normal(size=n)
    m1, m2 = rng.normal(size=n) * 0.1, rng.uniform(0, 0.1, n)
    tt = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in (th, g, m1, m2)]
    ref = [a.astype(np.float32).astype(np.float64) for a in (th, g, m1, m2)]
    for t in (1, 2, 3):
        s.adam(tt[0], tt[1], tt[2], tt[3], t, lr=1e-3)
        oracle.adam(ref[0], ref[1], ref[2], ref[3], t, lr=1e-3)
    assert np.allclose(tt[0].cpu().numpy(), ref[0], rtol=1e-6, atol=1e-6)
    assert np.allclose(tt[2].cpu().numpy(), ref[2], rtol=1e-5, atol=1e-7)
