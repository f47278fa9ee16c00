"""Argument checks of the Python binding, on the host: arrays of the wrong shape, size,
dtype or device are refused with ValueError before anything reaches the library (a short
array would otherwise be read or written past its end). A stub stands in for libnep."""
import types

import numpy as np
import pytest
import torch

from paper_2604_24816_amd import inputs as I
from paper_2604_24816_amd import nep


class StubLib:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def call(*args):
            self.calls.append((name, args))
            return 0
        return call


def shell(n=4, n_types=1):
    s = object.__new__(nep.NEPSystem)
    s.lib = StubLib()
    s.n = n
    s.device = torch.device("cpu")
    s.handle = None
    s.generation = 0
    s._types = None
    s._masses = None
    s.full = types.SimpleNamespace(hp=I.HParams(n_types=n_types))
    s.surrogate = None
    return s


def test_set_state_checks_every_array():
    s = shell(n=4, n_types=2)
    x, t, m, v = np.zeros((4, 3)), np.zeros(4, np.int32), np.ones(2), np.zeros((4, 3))
    for bad in (dict(x=np.zeros((3, 3))), dict(types=np.zeros(5, np.int32)), dict(masses=np.ones(1)),
                dict(v=np.zeros((4, 2))), dict(x=torch.zeros(5, 3)), dict(x=torch.zeros(4, 3), v=torch.zeros(3, 3))):
        args = dict(x=x, types=t, masses=m, v=v)
        args.update(bad)
        with pytest.raises(ValueError):
            s.set_state(**args)
    assert s.lib.calls == []
    s.set_state(x, t, m, v)
    assert [c[0] for c in s.lib.calls] == ["nep_set_state"] and s.lib.calls[0][1][-1] == 0


def test_training_buffers_are_checked():
    s = shell(n=4)
    hp = s.full.hp
    n = hp.n_params()
    theta = torch.zeros(n)
    with pytest.raises(ValueError):
        s.train_backward_params(0, theta, 1.0, None, out=torch.zeros(n - 1))
    with pytest.raises(ValueError):
        s.train_backward_params(0, theta, 1.0, None, out=torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError):
        s.train_backward_params(0, theta, 1.0, torch.zeros(3, 3))
    with pytest.raises(ValueError):
        s.train_backward_params(0, torch.zeros(n + 1), 1.0, None)
    assert s.lib.calls == []
    g = s.train_backward_params(0, theta, 1.0, torch.zeros(4, 3))
    assert g.shape == (n,) and s.lib.calls[-1][0] == "nep_train_backward_params"


def test_adam_checks_sizes_and_dtypes():
    s = shell()
    a = torch.zeros(10)
    with pytest.raises(ValueError):
        s.adam(a, torch.zeros(9), torch.zeros(10), torch.zeros(10), 1)
    with pytest.raises(ValueError):
        s.adam(a, torch.zeros(10), torch.zeros(10, dtype=torch.float64), torch.zeros(10), 1)
    assert s.lib.calls == []
    s.adam(a, torch.zeros(10), torch.zeros(10), torch.zeros(10), 1)
    assert s.lib.calls[-1][0] == "nep_adam_update"


def test_unknown_precision_is_refused():
    s = shell()
    with pytest.raises(ValueError):
        s.compute(precision="fp16")
    with pytest.raises(ValueError):
        s.step(4, precision="half")
    assert s.lib.calls == []


def test_valid_calls_reach_the_library():
    s = shell()
    E, W, F, U = s.compute(precision="bf16", per_atom=True)
    assert F.shape == (4, 3) and U.shape == (4,) and W.shape == (3, 3)
    assert s.lib.calls[-1][0] == "nep_compute_energy_forces_virial" and s.lib.calls[-1][1][2] == nep.NEP_BF16
    th = s.step(8, mts_k=4, thermo_every=4, relative_judge=True)
    names = [c[0] for c in s.lib.calls]
    assert names[-2:] == ["nep_set_judge", "nep_step"] and th.shape == (0, 8)


def test_deterministic_switch_and_fp64_gradient_reach_the_library():
    s = shell(n=4)
    s.set_deterministic(True)
    s.set_deterministic(False)
    assert [(c[0], c[1][1]) for c in s.lib.calls] == [("nep_set_deterministic", 1), ("nep_set_deterministic", 0)]
    with pytest.raises(ValueError):
        s.train_backward64(0.5, np.zeros((3, 3)))
    assert len(s.lib.calls) == 2
    g = s.train_backward64(0.5, np.zeros((4, 3)))
    name, args = s.lib.calls[-1]
    assert name == "nep_train_backward64" and args[1] == 0 and args[2] == 0.5
    assert g.dtype == torch.float64 and g.numel() == s.full.hp.n_params()
