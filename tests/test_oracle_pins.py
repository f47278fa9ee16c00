"""Pins of the FP64 oracle against facts fixed outside it (no GPU needed).

Each test checks the oracle against a closed form, a textbook identity, a
library routine, a brute-force evaluation, an invariance or a value printed in
the paper, so that a dropped term, a wrong sign, a wrong index or a transposed
operand in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

import oracle
from paper_2604_24816_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _single_block_model(hp, block, seed=5):
    """Random model whose hidden weights see only one descriptor block."""
    p = I.random_model(hp, seed)
    b = I.unpack(hp, p)
    nr, na = hp.n_max_radial + 1, hp.n_max_angular + 1
    W0 = b["W0"].reshape(hp.n_hidden, hp.n_desc)
    keep = np.zeros(hp.n_desc, bool)
    if block == "radial":
        keep[:nr] = True
    elif block == "fourbody":
        keep[nr + na * hp.l_max_3b:] = True
    else:  # angular l
        l = int(block)
        keep[nr + (l - 1) * na: nr + l * na] = True
    W0[:, ~keep] = 0.0
    return oracle.Model.from_hparams(hp, p)


# ----------------------------------------------------------------------------- neighbours

@pytest.mark.parametrize("box,n,seed", [((14.5, 14.5, 14.5), 300, 1), ((14.2, 21.7, 30.1), 600, 2),
                                        ((28.0, 14.0, 15.0), 500, 3)])
@pytest.mark.parametrize("cut", [6.0, 7.0])
def test_cell_list_equals_brute_force(box, n, seed, cut):
    rng = np.random.default_rng(seed)
    box = np.array(box)
    x = rng.uniform(0, 1, size=(n, 3)) * box
    cb, ib = oracle.neighbors(x, box, cut, brute=True, cap=400)
    cc, ic = oracle.neighbors(x, box, cut, brute=False, cap=400)
    assert np.array_equal(cb, cc)
    assert np.array_equal(ib, ic)
    # symmetric lists and strict inequality against an independent numpy distance
    i, j = 7, ib[7, 0]
    d = x[j] - x[i]
    d -= box * np.round(d / box)
    assert np.dot(d, d) < cut * cut
    assert i in ib[j, : cb[j]]


def test_fcc_shell_counts_match_paper_and_closed_form():
    g = json.load(open(os.path.join(GOLDEN, "fcc_shells.json")))
    x, box = I.fcc_lattice(6)
    for cut_s, want in g["closed_form"]["counts"].items():
        c, _ = oracle.neighbors(x, box, float(cut_s), cap=200)
        assert np.all(c == want), (cut_s, np.unique(c))
    c, _ = oracle.neighbors(x, box, g["paper_pin"]["cutoff"], cap=200)
    assert np.percentile(c, 90) == g["paper_pin"]["count"]


def test_box_too_small_rejected():
    x = np.zeros((2, 3))
    x[1] = 1.0
    with pytest.raises(RuntimeError, match="box too small"):
        oracle.neighbors(x, np.array([11.0, 20.0, 20.0]), 6.0)


# ----------------------------------------------------------------------------- bases

@pytest.mark.parametrize("rc", [5.0, 6.0])
def test_radial_basis_closed_forms(rc):
    K = 9
    f0, _ = oracle.radial_basis(0.0, rc, K)
    assert np.allclose(f0, 1.0, atol=1e-15)           # x = 1, T_k(1) = 1, f_c(0) = 1
    fe, dfe = oracle.radial_basis(rc * (1 - 1e-12), rc, K)
    assert np.max(np.abs(fe)) < 1e-20 and np.max(np.abs(dfe)) < 1e-9   # smooth at r_c
    fo, dfo = oracle.radial_basis(rc, rc, K)
    assert np.all(fo == 0) and np.all(dfo == 0)
    for r in np.linspace(0.3, rc - 0.3, 7):
        f, df = oracle.radial_basis(r, rc, K)
        fc = 0.5 * (1 + np.cos(np.pi * r / rc))
        x = 2 * (r / rc - 1) ** 2 - 1
        theta = np.arccos(x)
        Tk = 2 * f / fc - 1
        assert np.allclose(Tk, np.cos(np.arange(K) * theta), atol=1e-12)  # T_k(cos t) = cos kt
        h = 1e-6
        fp, _ = oracle.radial_basis(r + h, rc, K)
        fm, _ = oracle.radial_basis(r - h, rc, K)
        assert np.allclose(df, (fp - fm) / (2 * h), atol=1e-8)


def test_legendre_against_scipy():
    for c in [-1.0, -0.3, 0.0, 0.41, 1.0]:
        P, dP = oracle.legendre(c, 6)
        assert np.allclose(P, [eval_legendre(l, c) for l in range(7)], atol=1e-14)
        # P_l'(1) = l(l+1)/2 closed form, and central differences elsewhere
        if c == 1.0:
            assert np.allclose(dP, [l * (l + 1) / 2 for l in range(7)], atol=1e-12)
        elif abs(c) < 1:
            h = 1e-6
            Pp = np.array([eval_legendre(l, c + h) for l in range(7)])
            Pm = np.array([eval_legendre(l, c - h) for l in range(7)])
            assert np.allclose(dP, (Pp - Pm) / (2 * h), atol=1e-7)


def test_spherical_harmonics_orthonormal_by_quadrature():
    nt, nph = 12, 24
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phis = 2 * np.pi * np.arange(nph) / nph
    for l in range(1, 5):
        for lp in range(1, 5):
            G = np.zeros((2 * l + 1, 2 * lp + 1))
            for ct, w in zip(xg, wg):
                st = np.sqrt(1 - ct * ct)
                for ph in phis:
                    u = np.array([st * np.cos(ph), st * np.sin(ph), ct])
                    G += w * (2 * np.pi / nph) * np.outer(oracle.sph_harm(l, u), oracle.sph_harm(lp, u))
            want = np.eye(2 * l + 1) if l == lp else np.zeros_like(G)
            assert np.allclose(G, want, atol=1e-12), (l, lp)


def test_spherical_harmonics_addition_theorem_and_scipy():
    rng = np.random.default_rng(0)
    U = _rand_unit(rng, 6)
    for l in range(1, 5):
        for a in range(3):
            for b in range(3, 6):
                lhs = np.dot(oracle.sph_harm(l, U[a]), oracle.sph_harm(l, U[b]))
                rhs = (2 * l + 1) / (4 * np.pi) * eval_legendre(l, np.dot(U[a], U[b]))
                assert abs(lhs - rhs) < 1e-13
        # |Y| per m against scipy's complex harmonics: Y_{l,+-m} = sqrt(2) |Y_l^m| cos/sin
        u = U[0]
        theta = np.arccos(u[2])
        phi = np.arctan2(u[1], u[0])
        Y = oracle.sph_harm(l, u)
        for m in range(1, l + 1):
            c = sph_harm_y(l, m, theta, phi)
            amp = np.sqrt(2) * abs(c)
            assert abs(np.hypot(Y[l + m], Y[l - m]) - amp) < 1e-13
        assert abs(abs(Y[l]) - abs(sph_harm_y(l, 0, theta, phi))) < 1e-13


# ----------------------------------------------------------------------------- descriptors

def test_descriptor_paths_agree(full_model):
    at = I.workload_small()
    cen = np.arange(0, at.n, 97)
    q0 = oracle.descriptors(full_model, at.x, at.types, at.box, centers=cen, path=0)
    q1 = oracle.descriptors(full_model, at.x, at.types, at.box, centers=cen, path=1)
    assert np.allclose(q0, q1, rtol=1e-12, atol=1e-15)


def _cluster(points, L=40.0):
    """Atoms around the box centre (atom 0 is the center)."""
    x = np.asarray(points, float) + L / 2
    return x, np.zeros(len(points), np.int32), np.full(3, L)


def _g(hp, params, r, which):
    b = I.unpack(hp, params)
    if which == "R":
        K, n, rc, c = hp.basis_radial + 1, hp.n_max_radial + 1, hp.rc_radial, b["cR"]
    else:
        K, n, rc, c = hp.basis_angular + 1, hp.n_max_angular + 1, hp.rc_angular, b["cA"]
    f, _ = oracle.radial_basis(r, rc, K)
    return c.reshape(n, K) @ f


def test_dimer_and_trimer_closed_forms(full_hp):
    hp = full_hp
    p = I.random_model(hp, 3)
    m = oracle.Model.from_hparams(hp, p)
    nr, na = hp.n_max_radial + 1, hp.n_max_angular + 1
    # dimer: q_n = g_n, q_nl = g_n^2 (P_l(1) = 1), q4_n = (2/9) g_n^3 (tr(M^3) = 2/9)
    r = 2.7
    x, t, box = _cluster([[0, 0, 0], [r * 0.6, r * 0.8, 0]])
    q = oracle.descriptors(m, x, t, box, centers=[0])[0]
    gR, gA = _g(hp, p, r, "R"), _g(hp, p, r, "A")
    assert np.allclose(q[:nr], gR, atol=1e-14)
    for l in range(1, 5):
        assert np.allclose(q[nr + (l - 1) * na: nr + l * na], gA ** 2, atol=1e-14)
    assert np.allclose(q[nr + 4 * na:], 2.0 / 9.0 * gA ** 3, atol=1e-14)
    # trimer at angle theta: q_nl = g1^2 + g2^2 + 2 g1 g2 P_l(cos theta)
    r1, r2, th = 2.5, 3.4, 1.1
    x, t, box = _cluster([[0, 0, 0], [r1, 0, 0], [r2 * np.cos(th), r2 * np.sin(th), 0]])
    q = oracle.descriptors(m, x, t, box, centers=[0])[0]
    g1, g2 = _g(hp, p, r1, "A"), _g(hp, p, r2, "A")
    assert np.allclose(q[:nr], _g(hp, p, r1, "R") + _g(hp, p, r2, "R"), atol=1e-14)
    for l in range(1, 5):
        want = g1 ** 2 + g2 ** 2 + 2 * g1 * g2 * eval_legendre(l, np.cos(th))
        assert np.allclose(q[nr + (l - 1) * na: nr + l * na], want, atol=1e-13)


def test_four_body_triple_sum_identity(full_hp):
    """tr(S^3) equals sum_jkl g_j g_k g_l [c_jk c_kl c_lj - (c_jk^2 + c_kl^2 + c_lj^2)/3 + 2/9]."""
    hp = full_hp
    p = I.random_model(hp, 4)
    m = oracle.Model.from_hparams(hp, p)
    rng = np.random.default_rng(9)
    dirs = _rand_unit(rng, 5)
    rs = rng.uniform(2.2, 4.8, 5)
    pts = [[0, 0, 0]] + list(dirs * rs[:, None])
    x, t, box = _cluster(pts)
    q = oracle.descriptors(m, x, t, box, centers=[0])[0]
    nr, na = hp.n_max_radial + 1, hp.n_max_angular + 1
    G = np.array([_g(hp, p, r, "A") for r in rs])  # [j][n]
    C = dirs @ dirs.T
    want = np.zeros(na)
    for j in range(5):
        for k in range(5):
            for l in range(5):
                br = C[j, k] * C[k, l] * C[l, j] - (C[j, k] ** 2 + C[k, l] ** 2 + C[l, j] ** 2) / 3 + 2 / 9
                want += G[j] * G[k] * G[l] * br
    assert np.allclose(q[nr + 4 * na:], want, rtol=1e-11, atol=1e-15)


def test_isolated_atom_network_and_weight_orientation():
    """q = 0 gives U = sum w1 tanh(-b0) - b1; a one-entry W0 pins row = hidden, column = descriptor."""
    hp = I.HParams(n_max_radial=0, n_max_angular=0, basis_radial=1, basis_angular=1, l_max_3b=1,
                   l_max_4b=0, n_hidden=2)
    assert hp.n_desc == 2
    p = I.random_model(hp, 1)
    b = I.unpack(hp, p)
    x, t, box = _cluster([[0, 0, 0]])
    m = oracle.Model.from_hparams(hp, p)
    U, Fp, q = oracle.energies(m, x, t, box)
    assert np.all(q == 0)
    assert np.isclose(U[0], np.sum(b["w1"] * np.tanh(-b["b0"])) - b["b1"][0], atol=1e-15)
    # worked example: W0 = [[0, 1], [0, 0]], w1 = [1, 0], b0 = b1 = 0, sigma = (1, 1):
    # hidden unit 0 sees only descriptor 1 (the angular one), so U = tanh(q_1).
    b["W0"][:] = [0.0, 1.0, 0.0, 0.0]
    b["w1"][:] = [1.0, 0.0]
    b["b0"][:] = 0.0
    b["b1"][:] = 0.0
    b["sigma"][:] = 1.0
    b["cR"][:] = [0.0, 1.0]
    b["cA"][:] = [1.0, 0.0]
    m = oracle.Model.from_hparams(hp, p)
    x, t, box = _cluster([[0, 0, 0], [2.0, 1.0, 0.5]])
    r = np.sqrt(2.0 ** 2 + 1 + 0.25)
    U, Fp, q = oracle.energies(m, x, t, box, centers=[0])
    fR, _ = oracle.radial_basis(r, hp.rc_radial, 2)
    fA, _ = oracle.radial_basis(r, hp.rc_angular, 2)
    assert np.isclose(q[0, 0], fR[1]) and np.isclose(q[0, 1], fA[0] ** 2)
    assert np.isclose(U[0], np.tanh(fA[0] ** 2), atol=1e-15)
    assert np.allclose(Fp[0], [0.0, 1.0 - np.tanh(fA[0] ** 2) ** 2], atol=1e-15)


def test_network_gradient_fd(full_model, full_hp):
    """Fp = dU/dq against central differences through a tiny displacement of descriptors."""
    at = I.workload_small()
    cen = [5, 17]
    U, Fp, q = oracle.energies(full_model, at.x, at.types, at.box, centers=cen)
    b = I.unpack(full_hp, full_model.params)
    W0 = b["W0"].reshape(full_hp.n_hidden, full_hp.n_desc)

    def u_of(qv):
        return np.sum(b["w1"] * np.tanh(W0 @ (qv * b["sigma"]) - b["b0"])) - b["b1"][0]
    for c in range(2):
        assert np.isclose(u_of(q[c]), U[c], atol=1e-14)
        for v in range(full_hp.n_desc):
            h = 1e-6 / max(b["sigma"][v], 1.0)
            e = np.zeros(full_hp.n_desc)
            e[v] = h
            fd = (u_of(q[c] + e) - u_of(q[c] - e)) / (2 * h)
            assert abs(fd - Fp[c, v]) < 1e-6 * max(1.0, abs(Fp[c, v]))


# ----------------------------------------------------------------------------- forces, virial

@pytest.mark.parametrize("block", ["radial", "1", "2", "3", "4", "fourbody", "all"])
def test_forces_equal_minus_energy_gradient(full_hp, block):
    hp = full_hp
    m = _single_block_model(hp, block) if block != "all" else oracle.Model.from_hparams(hp, I.random_model(hp, 5))
    at = I.fcc_box(4, 0.15, 7)
    E, W, U, F = oracle.evaluate(m, at.x, at.types, at.box)
    rng = np.random.default_rng(1)
    h = 1e-5
    scale = np.abs(F).max()
    assert scale > 1e-4
    for _ in range(6):
        k, c = int(rng.integers(at.n)), int(rng.integers(3))
        xp = at.x.copy()
        xp[k, c] += h
        xm = at.x.copy()
        xm[k, c] -= h
        Up = oracle.evaluate(m, xp, at.types, at.box)[2]
        Um = oracle.evaluate(m, xm, at.types, at.box)[2]
        fd = -np.sum(Up - Um) / (2 * h)
        assert abs(fd - F[k, c]) < 1e-7 * max(1.0, scale), (block, k, c, fd, F[k, c])


# ----------------------------------------------------------------------------- ZBL repulsion

KE_COULOMB = 14.3996454784   # e^2 / (4 pi eps0) in eV A (CODATA)


def _zbl_models(z=(29.0, 29.0), n_types=1, outer=2.0):
    hp0 = I.HParams(n_types=n_types)
    hpz = I.HParams(n_types=n_types, zbl_outer=outer, zbl_z=z)
    p = I.random_model(hp0, 0)
    return hp0, hpz, oracle.Model.from_hparams(hp0, p), oracle.Model.from_hparams(hpz, p)


def _dimer_dE(m0, mz, r, types=(0, 0)):
    x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    t = np.array(types, np.int32)
    box = np.array([30.0, 30.0, 30.0])
    return oracle.evaluate(mz, x, t, box)[0] - oracle.evaluate(m0, x, t, box)[0]


def test_zbl_dimer_limits_and_switch():
    """The ZBL term of a dimer (energy with it minus without): as r -> 0 it tends to the
    bare Coulomb repulsion k_e Z_i Z_j / r (the screening weights sum to one); below the
    inner radius r E / (k_e Z_i Z_j) is the screening function, inside (0, 1) and
    decreasing; it is zero from the outer radius on, and value and slope are continuous
    at both radii (inner radius = half the outer one)."""
    _, _, m0, mz = _zbl_models()
    zz = KE_COULOMB * 29.0 * 29.0
    for r in (1e-6, 1e-7):
        assert abs(_dimer_dE(m0, mz, r) * r / zz - 1.0) < 20.0 * r
    scr = [_dimer_dE(m0, mz, r) * r / zz for r in (0.2, 0.5, 0.9)]
    assert 1.0 > scr[0] > scr[1] > scr[2] > 0.0
    assert _dimer_dE(m0, mz, 2.0) == 0.0 and _dimer_dE(m0, mz, 2.7) == 0.0
    h = 1e-6
    for r0 in (1.0, 2.0):
        lo, hi = _dimer_dE(m0, mz, r0 - h), _dimer_dE(m0, mz, r0 + h)
        slo = (_dimer_dE(m0, mz, r0 - h) - _dimer_dE(m0, mz, r0 - 2 * h)) / h
        shi = (_dimer_dE(m0, mz, r0 + 2 * h) - _dimer_dE(m0, mz, r0 + h)) / h
        # no jump: the change across r0 is what the one-sided slopes give over 2h
        assert abs((hi - lo) - h * (slo + shi)) < 1e-3 * h * max(1.0, abs(slo)), (r0, lo, hi)
        assert abs(slo - shi) < 1e-3 * max(1.0, abs(slo)), (r0, slo, shi)
    assert abs(_dimer_dE(m0, mz, 2.0 - 1e-4)) < 1e-6


def test_zbl_two_species_symmetry():
    """Cu-Au pairs: the limit k_e Z_Cu Z_Au / r, and the pair term does not depend on
    which atom is the center."""
    _, _, m0, mz = _zbl_models(z=(29.0, 79.0), n_types=2)
    zz = KE_COULOMB * 29.0 * 79.0
    assert abs(_dimer_dE(m0, mz, 1e-7, (0, 1)) * 1e-7 / zz - 1.0) < 1e-5
    for r in (0.4, 1.3):
        assert abs(_dimer_dE(m0, mz, r, (0, 1)) - _dimer_dE(m0, mz, r, (1, 0))) < 1e-9 * abs(
            _dimer_dE(m0, mz, r, (0, 1)))


def test_zbl_forces_and_virial_fd():
    """With close pairs (FCC compressed to a nearest-neighbour distance of 2.05 A, many
    pairs inside 2 A), forces are minus the energy gradient, they sum to zero, and the
    virial is minus the strain derivative of the energy."""
    _, _, _, mz = _zbl_models()
    at = I.fcc_box(5, 0.1, 31)
    x, box = at.x * 0.8, at.box * 0.8
    cnt, _ = oracle.neighbors(x, box, 2.0)
    assert cnt.sum() > 200
    E, W, U, F = oracle.evaluate(mz, x, at.types, box)
    assert np.abs(F.sum(0)).max() < 1e-9 * np.abs(F).max()
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(8):
        k, c = int(rng.integers(at.n)), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[k, c] += h
        xm[k, c] -= h
        fd = -(oracle.evaluate(mz, xp, at.types, box)[0] - oracle.evaluate(mz, xm, at.types, box)[0]) / (2 * h)
        assert abs(fd - F[k, c]) < 1e-6 * max(1.0, np.abs(F).max()), (k, c, fd, F[k, c])
    for a in range(3):
        e = 1e-7
        sc = np.ones(3)
        sc[a] = 1 + e
        Ep = oracle.evaluate(mz, x * sc, at.types, box * sc)[0]
        sc[a] = 1 - e
        Em = oracle.evaluate(mz, x * sc, at.types, box * sc)[0]
        assert abs(-(Ep - Em) / (2 * e) - W[a, a]) < 1e-6 * np.abs(W).max()


def test_net_force_zero_and_invariances(full_model):
    at = I.fcc_box(4, 0.2, 8)
    E, W, U, F = oracle.evaluate(full_model, at.x, at.types, at.box)
    assert np.allclose(F.sum(0), 0, atol=1e-12)
    assert np.allclose(W, W.T, atol=1e-10 * np.abs(W).max())
    # translation (with wrap)
    E2, _, U2, F2 = oracle.evaluate(full_model, I.wrap(at.x + [1.3, -0.7, 2.9], at.box), at.types, at.box)
    assert np.allclose(U2, U, atol=1e-12) and np.allclose(F2, F, atol=1e-12)
    # permutation of atom ids
    perm = np.random.default_rng(3).permutation(at.n)
    E3, _, U3, F3 = oracle.evaluate(full_model, at.x[perm], at.types[perm], at.box)
    assert np.allclose(U3, U[perm], atol=1e-12) and np.allclose(F3, F[perm], atol=1e-12)
    assert abs(E3 - E) < 1e-10


def test_rotation_invariance_of_isolated_cluster(full_model):
    rng = np.random.default_rng(12)
    pts = rng.normal(0, 2.2, size=(24, 3))
    L = 60.0
    E, _, U, F = oracle.evaluate(full_model, pts + L / 2, np.zeros(24, np.int32), np.full(3, L))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    E2, _, U2, F2 = oracle.evaluate(full_model, pts @ Q.T + L / 2, np.zeros(24, np.int32), np.full(3, L))
    assert np.allclose(U2, U, atol=1e-12)
    assert np.allclose(F2, F @ Q.T, atol=1e-12)


def test_perfect_fcc_symmetry(full_model):
    x, box = I.fcc_lattice(4)
    E, W, U, F = oracle.evaluate(full_model, x, np.zeros(len(x), np.int32), box)
    assert np.allclose(U, U[0], atol=1e-12)
    assert np.abs(F).max() < 1e-12
    assert np.allclose(np.diag(W), W[0, 0], rtol=1e-12)
    assert np.abs(W - np.diag(np.diag(W))).max() < 1e-10


def test_virial_equals_minus_strain_derivative(full_model):
    # isotropic / diagonal strain of a periodic box
    at = I.fcc_box(4, 0.15, 13)
    E, W, U, F = oracle.evaluate(full_model, at.x, at.types, at.box)
    h = 1e-6
    for a in range(3):
        s = np.ones(3)
        s[a] += h
        Ep = oracle.evaluate(full_model, at.x * s, at.types, at.box * s)[0]
        s[a] -= 2 * h
        Em = oracle.evaluate(full_model, at.x * s, at.types, at.box * s)[0]
        assert abs(-(Ep - Em) / (2 * h) - W[a, a]) < 1e-6 * abs(W[a, a]) + 1e-8
    # shear components on an isolated cluster (no periodic images inside the cutoff)
    rng = np.random.default_rng(5)
    pts = rng.normal(0, 2.0, size=(20, 3))
    L = 60.0
    t = np.zeros(20, np.int32)
    E, W, U, F = oracle.evaluate(full_model, pts + L / 2, t, np.full(3, L))
    for a, b in [(0, 1), (1, 2), (2, 0)]:
        eps = np.zeros((3, 3))
        eps[a, b] = h
        Ep = oracle.evaluate(full_model, pts @ (np.eye(3) + eps).T + L / 2, t, np.full(3, L))[0]
        Em = oracle.evaluate(full_model, pts @ (np.eye(3) - eps).T + L / 2, t, np.full(3, L))[0]
        assert abs(-(Ep - Em) / (2 * h) - W[a, b]) < 1e-6 * np.abs(W).max()


def test_sampled_forces_match_full(full_model):
    at = I.fcc_box(5, 0.1, 14)
    E, W, U, F = oracle.evaluate(full_model, at.x, at.types, at.box)
    sel = I.sample_ids(at.n, 25, 1)
    Us, Fs = oracle.evaluate_sampled(full_model, at.x, at.types, at.box, sel)
    assert np.allclose(Us, U[sel], atol=1e-13) and np.allclose(Fs, F[sel], atol=1e-12)


def test_two_species_pair_coefficients_ordered(full_hp):
    """Coefficients are indexed (center type, neighbour type): swapping types changes the dimer."""
    hp = I.HParams(n_types=2)
    p = I.random_model(hp, 21)
    m = oracle.Model.from_hparams(hp, p)
    b = I.unpack(hp, p)
    nr, kr = hp.n_max_radial + 1, hp.basis_radial + 1
    r = 3.1
    x, _, box = _cluster([[0, 0, 0], [r, 0, 0]])
    q = oracle.descriptors(m, x, np.array([0, 1], np.int32), box, centers=[0, 1])
    f, _ = oracle.radial_basis(r, hp.rc_radial, kr)
    cR = b["cR"].reshape(2, 2, nr, kr)
    assert np.allclose(q[0, :nr], cR[0, 1] @ f, atol=1e-14)
    assert np.allclose(q[1, :nr], cR[1, 0] @ f, atol=1e-14)


# ----------------------------------------------------------------------------- integration

def test_velocity_verlet_energy_conservation_scales_dt2(full_model):
    at = I.fcc_box(4, 0.05, 15)
    v = I.maxwell_boltzmann(at, 300.0, 16)
    fl = []
    for dt, n in [(2.0, 10), (1.0, 20)]:
        _, _, th = oracle.velocity_verlet(full_model, at.x, v, at.types, at.masses, at.box, dt, n)
        etot = th[:, 0] + th[:, 1]
        fl.append(np.max(np.abs(etot - etot[0])))
    ratio = fl[0] / fl[1]
    assert 2.5 < ratio < 6.0, (fl, ratio)


def test_velocity_verlet_time_reversible(full_model):
    at = I.fcc_box(4, 0.05, 17)
    v = I.maxwell_boltzmann(at, 300.0, 18)
    x1, v1, _ = oracle.velocity_verlet(full_model, at.x, v, at.types, at.masses, at.box, 1.0, 8)
    x2, v2, _ = oracle.velocity_verlet(full_model, x1, -v1, at.types, at.masses, at.box, 1.0, 8)
    d = x2 - at.x
    d -= at.box * np.round(d / at.box)
    assert np.abs(d).max() < 1e-9 and np.allclose(-v2, v, atol=1e-11)


def test_mts_reduces_to_velocity_verlet(full_hp):
    hp = full_hp
    m = oracle.Model.from_hparams(hp, I.random_model(hp, 0))
    sur_hp = I.SURROGATE_HPARAMS
    s = oracle.Model.from_hparams(sur_hp, I.surrogate_from_teacher(hp, m.params, sur_hp, 1))
    at = I.fcc_box(4, 0.05, 19)
    v = I.maxwell_boltzmann(at, 300.0, 20)
    xv, vv, _ = oracle.velocity_verlet(m, at.x, v, at.types, at.masses, at.box, 1.0, 8)
    # surrogate identical to the full model: bit-for-bit velocity Verlet
    xm, vm, err = oracle.mts(m, m, at.x, v, at.types, at.masses, at.box, 1.0, 4, 2)
    assert np.array_equal(xm, xv) and np.array_equal(vm, vv) and np.all(err == 0)
    # k = 1: velocity Verlet with the full force up to rounding, whatever the surrogate
    xk, vk, err = oracle.mts(m, s, at.x, v, at.types, at.masses, at.box, 1.0, 1, 8)
    assert np.allclose(xk, xv, atol=1e-12) and np.allclose(vk, vv, atol=1e-13)
    assert np.all(err[:, 0] > 0)


def test_mts_time_reversible(full_hp):
    """r-RESPA is a symmetric splitting: three blocks forward, reverse the velocities,
    three blocks more return to the start (untrained surrogate, so the slow correction
    is large)."""
    hp = full_hp
    m = oracle.Model.from_hparams(hp, I.random_model(hp, 0))
    sur_hp = I.SURROGATE_HPARAMS
    s = oracle.Model.from_hparams(sur_hp, I.surrogate_from_teacher(hp, m.params, sur_hp, 1))
    at = I.fcc_box(4, 0.1, 21)
    v = I.maxwell_boltzmann(at, 600.0, 22)
    x1, v1, _ = oracle.mts(m, s, at.x, v, at.types, at.masses, at.box, 1.0, 4, 3)
    x2, v2, _ = oracle.mts(m, s, x1, -v1, at.types, at.masses, at.box, 1.0, 4, 3)
    d = x2 - at.x
    d -= at.box * np.round(d / at.box)
    assert np.abs(d).max() < 1e-10 and np.abs(v2 + v).max() < 1e-12
    assert np.abs(x1 - at.x).max() > 1e-2


# ----------------------------------------------------------------------------- gradients, bf16, adam

def test_weight_gradient_fd(full_hp):
    hp = full_hp
    p = I.random_model(hp, 6)
    m = oracle.Model.from_hparams(hp, p)
    at = I.fcc_box(4, 0.17, 23)
    rng = np.random.default_rng(2)
    gF = rng.normal(size=(at.n, 3))
    gE = 0.7
    grad = oracle.weight_grad(m, at.x, at.types, at.box, gE, gF)
    off = hp.offsets()["W0"][0]

    def loss(pp):
        mm = oracle.Model.from_hparams(hp, pp)
        E, _, _, F = oracle.evaluate(mm, at.x, at.types, at.box)
        return gE * E + np.sum(gF * F)
    idx = list(rng.choice(hp.n_hidden * hp.n_desc, 6, replace=False))
    G = hp.n_hidden * hp.n_desc
    idx += [G + 3, G + hp.n_hidden + 5, G + 2 * hp.n_hidden]  # b0, w1, b1
    for k in idx:
        h = 1e-6
        pp = p.copy()
        pp[off + k] += h
        lp = loss(pp)
        pp[off + k] -= 2 * h
        lm = loss(pp)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) < 2e-6 * max(1.0, abs(grad[k])), (k, fd, grad[k])


@pytest.mark.parametrize("kind", ["full", "two_species", "surrogate"])
def test_param_gradient_fd(kind):
    """Gradient with respect to the expansion coefficients c (radial and angular, every
    species pair), the scaler and the network, against central differences of the
    oracle's own E and F; its network block equals weight_grad."""
    if kind == "two_species":
        hp = I.HParams(n_types=2)
        p = I.random_model(hp, 8)
        at = I.alloy_box(4, 1, 30, 2, 0.17, 3)
    elif kind == "surrogate":
        thp = I.FULL_HPARAMS
        hp = I.SURROGATE_HPARAMS
        p = I.surrogate_from_teacher(thp, I.random_model(thp, 0), hp, 3)
        at = I.fcc_box(4, 0.17, 23)
    else:
        hp = I.FULL_HPARAMS
        p = I.random_model(hp, 6)
        at = I.fcc_box(4, 0.17, 23)
    m = oracle.Model.from_hparams(hp, p)
    rng = np.random.default_rng(2)
    gF = rng.normal(size=(at.n, 3))
    gE = 0.7
    grad = oracle.param_grad(m, at.x, at.types, at.box, gE, gF)
    o = hp.offsets()
    off = o["W0"][0]
    ref = oracle.weight_grad(m, at.x, at.types, at.box, gE, gF)
    assert np.abs(grad[off:] - ref).max() < 1e-12 * np.abs(ref).max()
    grad0 = oracle.param_grad(m, at.x, at.types, at.box, gE, None)

    def loss(pp, with_f=True):
        E, _, _, F = oracle.evaluate(oracle.Model.from_hparams(hp, pp), at.x, at.types, at.box)
        return gE * E + (np.sum(gF * F) if with_f else 0.0)
    # entries from every block of cR and cA (each species pair) and the scaler
    idx = []
    for name in ("cR", "cA"):
        a, b = o[name]
        blk = (b - a) // hp.n_types ** 2
        for t in range(hp.n_types ** 2):
            idx += list(a + t * blk + rng.choice(blk, 3, replace=False))
    idx += list(o["sigma"][0] + rng.choice(hp.n_desc, 3, replace=False))
    for k in idx:
        for with_f, g in ((True, grad), (False, grad0)):
            h = 1e-6
            pp = p.copy()
            pp[k] += h
            lp = loss(pp, with_f)
            pp[k] -= 2 * h
            lm = loss(pp, with_f)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(g[k])), (kind, k, with_f, fd, g[k])


# ----------------------------------------------------------------------------- NVT (Nose-Hoover chain)

def _zero_force_model(hp):
    p = I.random_model(hp, 0)
    p[hp.offsets()["W0"][0]:] = 0.0    # constant network output: no forces
    return oracle.Model.from_hparams(hp, p)


@pytest.mark.parametrize("M", [1, 3])
def test_nvt_chain_follows_its_equations_of_motion(full_hp, M):
    """With zero forces the particles only feel the chain, and the state (KE, chain
    velocities and positions) obeys dKE/dt = -2 v_1 KE, dv_k/dt = G_k - v_k v_{k+1}
    (no damping term for the last), deta_k/dt = v_k. The integrator must converge to
    an independent high-accuracy solution of these equations at second order in dt."""
    from scipy.integrate import solve_ivp
    m0 = _zero_force_model(full_hp)
    at = I.fcc_box(3, 0.1, 3)
    at = I.Atoms(x=at.x * 1.5, types=at.types, box=at.box * 1.5, masses=at.masses)
    at.v = I.maxwell_boltzmann(at, 600.0, 4)
    n, T0, tau, kB = at.n, 300.0, 20.0, 8.617333262e-5
    Nf, kT = 3 * n - 3, kB * T0
    Q = np.full(M, kT * tau * tau)
    Q[0] *= Nf
    ke0 = 0.5 * np.sum(at.masses[at.types][:, None] * at.v ** 2) * 103.642697

    def rhs(t, y):
        ke, ve = y[0], y[1:1 + M]
        G = np.empty(M)
        G[0] = (2 * ke - Nf * kT) / Q[0]
        G[1:] = (Q[:-1] * ve[:-1] ** 2 - kT) / Q[1:]
        dve = G.copy()
        dve[:-1] -= ve[:-1] * ve[1:]
        return np.concatenate([[-2 * ve[0] * ke], dve, ve])
    ref = solve_ivp(rhs, (0, 100.0), np.concatenate([[ke0], np.zeros(2 * M)]), method="DOP853",
                    rtol=1e-12, atol=1e-14).y[:, -1]
    errs = []
    for dt in (0.25, 0.125):
        _, _, eta, ve, th = oracle.nvt(m0, at.x, at.v, at.types, at.masses, at.box, dt, int(100 / dt), T0, tau,
                                       np.zeros(M), np.zeros(M))
        errs.append(max(abs(th[-1, 1] - ref[0]) / ref[0],
                        np.abs(ve - ref[1:1 + M]).max() / np.abs(ref[1:1 + M]).max(),
                        np.abs(eta - ref[1 + M:]).max() / np.abs(ref[1 + M:]).max()))
    assert errs[1] < 2e-5, errs
    assert 3.8 < errs[0] / errs[1] < 4.2, errs


def test_nvt_with_a_stiff_chain_mass_is_nve(full_model):
    """tau -> infinity decouples the chain: the steps are velocity Verlet's."""
    at = I.fcc_box(4, 0.1, 7)
    at.v = I.maxwell_boltzmann(at, 600.0, 8)
    x1, v1, _ = oracle.velocity_verlet(full_model, at.x, at.v, at.types, at.masses, at.box, 1.0, 6)
    x2, v2, _, _, _ = oracle.nvt(full_model, at.x, at.v, at.types, at.masses, at.box, 1.0, 6, 300.0, 1e9,
                                 np.zeros(3), np.zeros(3))
    assert np.abs(x1 - x2).max() < 1e-10 and np.abs(v1 - v2).max() < 1e-12


def test_nvt_time_reversible_and_conserving(full_model):
    """Reversing particle and chain velocities retraces the trajectory, and the extended
    energy (PE + KE + chain energy) drifts as dt^2."""
    at = I.fcc_box(4, 0.1, 7)
    at.v = I.maxwell_boltzmann(at, 600.0, 8)
    x, v, eta, ve, _ = oracle.nvt(full_model, at.x, at.v, at.types, at.masses, at.box, 1.0, 12, 300.0, 10.0,
                                  np.zeros(3), np.zeros(3))
    xb, vb, _, _, _ = oracle.nvt(full_model, x, -v, at.types, at.masses, at.box, 1.0, 12, 300.0, 10.0, eta, -ve)
    d = xb - at.x
    d -= at.box * np.round(d / at.box)
    assert np.abs(d).max() < 1e-9 and np.abs(vb + at.v).max() < 1e-11
    drift = []
    for dt in (1.0, 0.5):
        th = oracle.nvt(full_model, at.x, at.v, at.types, at.masses, at.box, dt, int(40 / dt), 300.0, 20.0,
                        np.zeros(3), np.zeros(3))[4]
        drift.append(np.abs(th[:, 4] - th[0, 4]).max())
    assert 3.0 < drift[0] / drift[1] < 5.0, drift


def test_bf16_rounding_closed_forms():
    import torch
    assert oracle.round_bf16(1.0) == 1.0
    assert oracle.round_bf16(1 + 2 ** -8) == 1.0                 # tie -> even
    assert oracle.round_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # tie -> even
    assert oracle.round_bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert oracle.round_bf16(-0.1) == -0.10009765625
    rng = np.random.default_rng(4)
    vals = rng.normal(0, 3, 200).astype(np.float32).astype(np.float64)
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(v) for v in vals])
    assert np.array_equal(got, ref)


def test_bf16_model_error_is_bf16_sized(full_model):
    at = I.fcc_box(4, 0.1, 24)
    E, W, U, F = oracle.evaluate(full_model, at.x, at.types, at.box)
    Eb, Wb, Ub, Fb = oracle.evaluate(full_model, at.x, at.types, at.box, bf16=True)
    du = np.abs(Ub - U).max()
    assert 1e-6 < du < 5e-2
    assert np.abs(Fb - F).max() < 0.05 * np.abs(F).max()


def test_bf16_network_worked_example():
    """One hidden unit, values chosen so that each of the three bfloat16 roundings of the
    form (scaled descriptor, W0, w1 (1 - tanh^2)) moves a known bit: the expected U and
    dU/dq follow from the rounded values typed in below (8 significant bits each, so every
    product is exact in FP64), with the rounding of w1 (1 - tanh^2) taken by torch."""
    import math
    import torch
    hp = I.HParams(l_max_3b=2, l_max_4b=0, n_hidden=1)
    D = hp.n_desc
    p = np.zeros(hp.n_params())
    o = hp.offsets()
    sig = np.ones(D)
    sig[0] = 0.25
    sig[3] = 3.0
    p[o["sigma"][0]:o["sigma"][1]] = sig
    W0 = np.zeros(D)
    W0[0] = 0.5 + 2 ** -10 + 2 ** -12          # bf16: 0.5 (0.31 ulp below the midpoint)
    W0[3] = 1.0 - 2 ** -9 - 2 ** -12           # bf16: 1 - 2^-8
    p[o["W0"][0]:o["W0"][1]] = W0
    p[o["b0"][0]] = 0.1
    p[o["w1"][0]] = 1.7
    p[o["b1"][0]] = 0.3
    q = np.zeros(D)
    q[0] = 4.0 * (1.0 + 2 ** -8 + 2 ** -20)    # q~ = 1 + 2^-8 + 2^-20 -> bf16 1 + 2^-7
    q[3] = -(0.25 + 2 ** -11)                  # q~ = -(0.75 + 3 2^-11) -> bf16 -0.75
    m = oracle.Model.from_hparams(hp, p)
    U, Fp = oracle.network(m, q, bf16=True)
    h = 0.5 * (1.0 + 2 ** -7) + (1.0 - 2 ** -8) * (-0.75) - 0.1
    t = math.tanh(h)
    a1 = 1.7 * (1.0 - t * t)
    a1r = float(torch.tensor(a1, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).double())
    assert abs(a1r - a1) > 1e-4 * a1        # the rounding of a1 matters at this scale
    U_ref = 1.7 * t - 0.3
    Fp_ref = np.zeros(D)
    Fp_ref[0] = 0.25 * 0.5 * a1r
    Fp_ref[3] = 3.0 * (1.0 - 2 ** -8) * a1r
    assert abs(U - U_ref) <= 4e-16 * abs(U_ref)
    assert np.array_equal(Fp, Fp_ref)
    # the same model without rounding gives a different U and dU/dq
    U64, Fp64 = oracle.network(m, q)
    assert abs(U64 - U) > 1e-3 and abs(Fp64[0] - Fp[0]) > 1e-4 and abs(Fp64[3] - Fp[3]) > 1e-4


@pytest.mark.parametrize("betas,eps", [((0.9, 0.999), 1e-8), ((0.5, 0.9), 1e-8), ((0.95, 0.6), 1e-3)])
def test_adam_matches_torch_over_several_steps(betas, eps):
    """Seven Adam steps on non-uniform gradients against torch.optim.Adam in FP64 (the bias
    corrections of later steps, the order of beta1 and beta2 and where eps enters)."""
    import torch
    rng = np.random.default_rng(17)
    n = 37
    theta = rng.normal(size=n)
    grads = [rng.normal(size=n) * rng.uniform(0.01, 3.0, size=n) for _ in range(7)]
    pt = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=betas, eps=eps, foreach=False)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    for t, g in enumerate(grads, start=1):
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        oracle.adam(theta, g, m1, m2, t, lr=0.01, beta1=betas[0], beta2=betas[1], eps=eps)
        assert np.abs(theta - pt.detach().numpy()).max() < 1e-14, t


def test_adam_first_step_is_signed_lr():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -1e-3, 0.2])
    m1 = np.zeros(3)
    m2 = np.zeros(3)
    oracle.adam(theta, g, m1, m2, 1, lr=0.01, eps=1e-12)
    assert np.allclose(theta, [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01], atol=1e-9)


# ----------------------------------------------------------------------------- inputs

def test_maxwell_boltzmann_exact_temperature_and_zero_momentum():
    at = I.fcc_box(5, 0.05, 1)
    v = I.maxwell_boltzmann(at, 600.0, 2)
    m = at.masses[at.types]
    assert np.allclose((m[:, None] * v).sum(0), 0, atol=1e-12)
    ke = 0.5 * I.AMU_A2_FS2_IN_EV * np.sum(m[:, None] * v * v)
    T = 2 * ke / ((3 * at.n - 3) * I.BOLTZMANN_EV_PER_K)
    assert abs(T - 600.0) < 1e-9


def test_alloy_workload_counts():
    at = I.alloy_box(6, 31, 43, 32, 0.05, 33)
    assert at.n == 4 * 216 - 43
    assert abs(int((at.types == 1).sum()) - int((at.types == 0).sum())) <= 43
