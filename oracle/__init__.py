"""FP64 CPU oracle of the NEP evaluation (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path never calls it; the two
share no code. The arithmetic lives in ``nep_oracle.cpp`` (plain C++17, FP64,
built with ``-O2 -ffp-contract=off``); this module only marshals NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nep_oracle.cpp")
_LIB = os.path.join(_HERE, "_liboracle.so")

_lib = None

ERRORS = {0: "ok", -1: "bad argument", -2: "box too small", -3: "neighbour capacity exceeded"}


def build(force: bool = True) -> str:
    """Compile the oracle library in place (g++, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c++17", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_round_bf16.restype = ctypes.c_double
        _lib.orc_round_bf16.argtypes = [ctypes.c_double]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what}: {ERRORS.get(st, st)}")


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for the following oracle calls."""
    _check(_load().orc_set_num_threads(ctypes.c_int32(int(n))), "set_num_threads")


class Model:
    """Hyperparameters (8 ints, 2 reals) plus the packed FP64 parameter vector."""

    def __init__(self, int_hparams, real_hparams, params):
        self.ip = np.ascontiguousarray(int_hparams, dtype=np.int32)
        self.dp = _f64(real_hparams)
        self.params = _f64(params)
        n = ctypes.c_int64()
        d = ctypes.c_int32()
        _load().orc_n_params(_p(self.ip), ctypes.byref(n), ctypes.byref(d))
        if n.value != self.params.size:
            raise ValueError(f"parameter count {self.params.size} != {n.value}")
        self.n_desc = d.value
        self.n_hidden = int(self.ip[7])

    @classmethod
    def from_hparams(cls, hp, params):
        return cls(hp.int_array(), hp.real_array(), params)

    def _args(self):
        return (_p(self.ip), _p(self.dp), _p(self.params), ctypes.c_int64(self.params.size))


def neighbors(x, box, cut, brute=False, cap=256):
    """Lists with r^2 < cut^2, ascending ids: (counts [N], idx [N][cap])."""
    x = _f64(x)
    box = _f64(box)
    n = x.shape[0]
    counts = np.zeros(n, np.int64)
    idx = np.full((n, cap), -1, np.int32)
    st = _load().orc_neighbors(ctypes.c_int64(n), _p(x), _p(box), ctypes.c_double(cut),
                               ctypes.c_int(1 if brute else 0), _p(counts), _p(idx),
                               ctypes.c_int32(cap))
    _check(st, "neighbors")
    return counts, idx


def radial_basis(r, rc, K):
    f = np.zeros(K)
    df = np.zeros(K)
    _check(_load().orc_radial_basis(ctypes.c_double(r), ctypes.c_double(rc), ctypes.c_int32(K),
                                    _p(f), _p(df)), "radial_basis")
    return f, df


def legendre(c, L):
    P = np.zeros(L + 1)
    dP = np.zeros(L + 1)
    _check(_load().orc_legendre(ctypes.c_double(c), ctypes.c_int32(L), _p(P), _p(dP)), "legendre")
    return P, dP


def sph_harm(l, u):
    u = _f64(u)
    Y = np.zeros(2 * l + 1)
    _check(_load().orc_sph_harm(ctypes.c_int32(l), _p(u), _p(Y)), "sph_harm")
    return Y


def round_bf16(v: float) -> float:
    return float(_load().orc_round_bf16(float(v)))


def network(model: Model, q, bf16=False):
    """U and dU/dq of the network on one descriptor vector q [D] (bf16: the bfloat16 form)."""
    q = _f64(q)
    if q.size != model.n_desc:
        raise ValueError(f"q has {q.size} values, expected {model.n_desc}")
    U = ctypes.c_double()
    Fp = np.zeros(model.n_desc)
    st = _load().orc_network(*model._args(), _p(q), ctypes.c_int32(1 if bf16 else 0), ctypes.byref(U), _p(Fp))
    _check(st, "network")
    return U.value, Fp


def descriptors(model: Model, x, types, box, centers=None, path=0):
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    n = x.shape[0]
    cen = None if centers is None else np.ascontiguousarray(centers, np.int64)
    nc = n if cen is None else cen.size
    q = np.zeros((nc, model.n_desc))
    st = _load().orc_descriptors(*model._args(), ctypes.c_int64(n), _p(x), _p(types), _p(box),
                                 ctypes.c_int64(nc), _p(cen), ctypes.c_int32(path), _p(q))
    _check(st, "descriptors")
    return q


def evaluate(model: Model, x, types, box, bf16=False):
    """(E, W[3][3], U[N], F[N][3]) of the whole system."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    n = x.shape[0]
    E = ctypes.c_double()
    W = np.zeros(9)
    U = np.zeros(n)
    F = np.zeros((n, 3))
    st = _load().orc_evaluate(*model._args(), ctypes.c_int64(n), _p(x), _p(types), _p(box),
                              ctypes.c_int32(1 if bf16 else 0), ctypes.byref(E), _p(W), _p(U), _p(F))
    _check(st, "evaluate")
    return E.value, W.reshape(3, 3), U, F


def evaluate_sampled(model: Model, x, types, box, sel, bf16=False):
    """(U[sel], F[sel][3]) for the selected atoms only."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    sel = np.ascontiguousarray(sel, np.int64)
    U = np.zeros(sel.size)
    F = np.zeros((sel.size, 3))
    st = _load().orc_evaluate_sampled(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(types),
                                      _p(box), ctypes.c_int32(1 if bf16 else 0),
                                      ctypes.c_int64(sel.size), _p(sel), _p(U), _p(F))
    _check(st, "evaluate_sampled")
    return U, F


def energies(model: Model, x, types, box, centers=None, bf16=False):
    """(U, Fp, q) of the given centers (all atoms when None)."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    n = x.shape[0]
    cen = None if centers is None else np.ascontiguousarray(centers, np.int64)
    nc = n if cen is None else cen.size
    U = np.zeros(nc)
    Fp = np.zeros((nc, model.n_desc))
    q = np.zeros((nc, model.n_desc))
    st = _load().orc_energies(*model._args(), ctypes.c_int64(n), _p(x), _p(types), _p(box),
                              ctypes.c_int32(1 if bf16 else 0), ctypes.c_int64(nc), _p(cen),
                              _p(U), _p(Fp), _p(q))
    _check(st, "energies")
    return U, Fp, q


def center_work(model: Model, x, types, box, first, count):
    """Per-center work of a force evaluation for ``count`` centers; returns a checksum."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    cs = ctypes.c_double()
    st = _load().orc_center_work(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(types),
                                 _p(box), ctypes.c_int64(first), ctypes.c_int64(count),
                                 ctypes.byref(cs))
    _check(st, "center_work")
    return cs.value


def velocity_verlet(model: Model, x, v, types, masses, box, dt, n_steps):
    """Integrate n_steps; returns (x, v, thermo[n_steps+1][4] = PE, KE, T, P)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    types = np.ascontiguousarray(types, np.int32)
    masses = _f64(masses)
    box = _f64(box)
    thermo = np.zeros((n_steps + 1, 4))
    st = _load().orc_velocity_verlet(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(v),
                                     _p(types), _p(masses), _p(box), ctypes.c_double(dt),
                                     ctypes.c_int64(n_steps), _p(thermo))
    _check(st, "velocity_verlet")
    return x, v, thermo


def nvt(model: Model, x, v, types, masses, box, dt, n_steps, T0, tau, eta, ve):
    """NVT (Nose-Hoover chain) steps; returns (x, v, eta, ve, thermo[n_steps+1][5] =
    PE, KE, T, P, conserved energy). eta, ve: chain state of length M (copied)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    eta = _f64(eta).copy()
    ve = _f64(ve).copy()
    types = np.ascontiguousarray(types, np.int32)
    masses = _f64(masses)
    box = _f64(box)
    thermo = np.zeros((n_steps + 1, 5))
    st = _load().orc_nvt(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(v), _p(types), _p(masses),
                         _p(box), ctypes.c_double(dt), ctypes.c_int64(n_steps), ctypes.c_double(T0),
                         ctypes.c_double(tau), ctypes.c_int32(eta.size), _p(eta), _p(ve), _p(thermo))
    _check(st, "nvt")
    return x, v, eta, ve, thermo


def mts(full: Model, sur: Model, x, v, types, masses, box, dt, k, n_blocks):
    """r-RESPA blocks; returns (x, v, err[n_blocks][2] = rms, max of |F_full - F_s|)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    types = np.ascontiguousarray(types, np.int32)
    masses = _f64(masses)
    box = _f64(box)
    err = np.zeros((n_blocks, 2))
    st = _load().orc_mts(*full._args(), *sur._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(v),
                         _p(types), _p(masses), _p(box), ctypes.c_double(dt), ctypes.c_int32(k),
                         ctypes.c_int64(n_blocks), _p(err))
    _check(st, "mts")
    return x, v, err


def weight_grad(model: Model, x, types, box, gE, gF=None):
    """d(gE*E + sum gF.F)/d(W0, b0, w1, b1), packed in that order."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    H, D = model.n_hidden, model.n_desc
    grad = np.zeros(H * D + 2 * H + 1)
    gFa = None if gF is None else _f64(gF)
    st = _load().orc_weight_grad(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(types),
                                 _p(box), ctypes.c_double(gE), _p(gFa), _p(grad))
    _check(st, "weight_grad")
    return grad


def param_grad(model: Model, x, types, box, gE, gF=None):
    """d(gE*E + sum gF.F)/d(every packed parameter): [cR | cA | sigma | W0 | b0 | w1 | b1]."""
    x = _f64(x)
    types = np.ascontiguousarray(types, np.int32)
    box = _f64(box)
    grad = np.zeros(model.params.size)
    gFa = None if gF is None else _f64(gF)
    st = _load().orc_param_grad(*model._args(), ctypes.c_int64(x.shape[0]), _p(x), _p(types),
                                _p(box), ctypes.c_double(gE), _p(gFa), _p(grad))
    _check(st, "param_grad")
    return grad


def adam(theta, g, m1, m2, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on FP64 arrays."""
    for a in (theta, g, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _check(_load().orc_adam(ctypes.c_int64(theta.size), _p(theta), _p(g), _p(m1), _p(m2),
                            ctypes.c_int64(t), ctypes.c_double(lr), ctypes.c_double(beta1),
                            ctypes.c_double(beta2), ctypes.c_double(eps)), "adam")
