"""Python binding of the NEP C-ABI library (``libnep.so``, declared in ``include/nep.h``).

Argument marshalling only: every step of the evaluation and of the integrator
runs in the HIP kernels of the library. PyTorch provides device memory (the
workspace and device-side arrays) and the HIP stream. There is no fallback:
if the library is missing or no GPU is present, these classes raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

from . import inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep.so")

NEP_FP32 = 0
NEP_BF16 = 1
NEP_FP64 = 2   # evaluation only: FP64 throughout, for checks
_PREC = {"fp32": NEP_FP32, "bf16": NEP_BF16, "fp64": NEP_FP64, NEP_FP32: NEP_FP32, NEP_BF16: NEP_BF16,
         NEP_FP64: NEP_FP64}


def _prec(p) -> int:
    try:
        return _PREC[p]
    except (KeyError, TypeError):
        raise ValueError(f"precision {p!r}: expected 'fp32', 'bf16' or 'fp64'") from None

EXPORTED = [
    "nep_param_count", "nep_model_create", "nep_model_destroy", "nep_system_workspace_bytes",
    "nep_system_create", "nep_system_destroy", "nep_system_set_params", "nep_set_state",
    "nep_build_neighbors", "nep_export_neighbors", "nep_compute_energy_forces_virial", "nep_step",
    "nep_set_judge", "nep_set_deterministic", "nep_set_thermostat", "nep_set_thermostat_state", "nep_get_thermostat", "nep_get_state",
    "nep_get_stats", "nep_halo_stats",
    "nep_train_forward", "nep_train_backward", "nep_train_forward_params", "nep_train_backward_params",
    "nep_train_backward64",
    "nep_adam_update",
    "nep_surrogate_error", "nep_status_string", "nep_last_error", "nep_profile", "nep_profile_read",
    "nep_pair_counts", "nep_compute_energy_forces_virial_noalloc",
]


class NEPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"NEP status {status}: {message}")
        self.status = status


class _HParams(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int32), ("n_max_radial", ctypes.c_int32),
                ("n_max_angular", ctypes.c_int32), ("basis_radial", ctypes.c_int32),
                ("basis_angular", ctypes.c_int32), ("l_max_3b", ctypes.c_int32),
                ("l_max_4b", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("rc_radial", ctypes.c_double), ("rc_angular", ctypes.c_double),
                ("zbl_rc_inner", ctypes.c_double), ("zbl_rc_outer", ctypes.c_double),
                ("zbl_z", ctypes.c_double * 2)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnep.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "nep_param_count": [vp, vp, vp],
        "nep_model_create": [vp, vp, i64, vp],
        "nep_system_workspace_bytes": [vp, vp, i64, vp, i32, i32, vp],
        "nep_system_create": [vp, vp, i64, vp, i32, i32, vp, i64, vp, vp],
        "nep_system_set_params": [vp, i32, vp, i64],
        "nep_set_state": [vp, vp, vp, vp, vp, i32],
        "nep_build_neighbors": [vp, f64],
        "nep_export_neighbors": [vp, i32, vp, vp, i64],
        "nep_compute_energy_forces_virial": [vp, i32, i32, vp, vp, vp, vp, i32],
        "nep_step": [vp, i64, f64, i32, f64, i32, f64, f64, i32, vp, i32, i64, vp],
        "nep_get_state": [vp, vp, vp, vp, i32],
        "nep_set_judge": [vp, i32],
        "nep_set_deterministic": [vp, i32],
        "nep_set_thermostat": [vp, f64, f64, i32],
        "nep_get_thermostat": [vp, vp, vp, vp],
        "nep_set_thermostat_state": [vp, vp, vp],
        "nep_get_stats": [vp, vp],
        "nep_halo_stats": [vp, vp],
        "nep_train_forward": [vp, i32, vp, vp, vp],
        "nep_train_backward": [vp, i32, vp, f64, vp, vp, i32],
        "nep_train_forward_params": [vp, i32, vp, vp, vp],
        "nep_train_backward_params": [vp, i32, vp, f64, vp, vp, i32],
        "nep_train_backward64": [vp, i32, f64, vp, vp],
        "nep_adam_update": [vp, vp, vp, vp, vp, i64, i64, f64, f64, f64, f64],
        "nep_surrogate_error": [vp, i32, vp],
        "nep_profile": [vp, i32],
        "nep_profile_read": [vp, vp, vp],
        "nep_pair_counts": [vp, vp],
        "nep_compute_energy_forces_virial_noalloc": [vp, i64, vp, i32, i32, f64, vp, vp, i32, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nep_model_destroy.argtypes = [vp]
    lib.nep_model_destroy.restype = None
    lib.nep_system_destroy.argtypes = [vp]
    lib.nep_system_destroy.restype = None
    lib.nep_status_string.argtypes = [ctypes.c_int]
    lib.nep_status_string.restype = ctypes.c_char_p
    lib.nep_last_error.argtypes = [vp]
    lib.nep_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _hp_struct(hp: inputs.HParams) -> _HParams:
    z = list(hp.zbl_z) + [0.0] * (2 - len(hp.zbl_z))
    return _HParams(hp.n_types, hp.n_max_radial, hp.n_max_angular, hp.basis_radial, hp.basis_angular,
                    hp.l_max_3b, hp.l_max_4b, hp.n_hidden, hp.rc_radial, hp.rc_angular,
                    hp.zbl_inner, hp.zbl_outer, (ctypes.c_double * 2)(z[0], z[1]))


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _t_ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class NEPModel:
    """Host-side model handle (hyperparameters + packed FP64 parameters)."""

    def __init__(self, hp: inputs.HParams, params: np.ndarray):
        lib = load_library()
        self.hp = hp
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self._hps = _hp_struct(hp)
        h = ctypes.c_void_p()
        st = lib.nep_model_create(ctypes.byref(self._hps), _np_ptr(self.params),
                                  self.params.size, ctypes.byref(h))
        if st != 0:
            raise NEPError(st, lib.nep_status_string(st).decode())
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nep_model_destroy(self.handle)
            self.handle = None


class NEPSystem:
    """One periodic system on one GPU: workspace, state, neighbour lists, models."""

    def __init__(self, full: NEPModel, n_atoms: int, box, surrogate: Optional[NEPModel] = None,
                 cap_radial: int = 160, cap_angular: int = 96, device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("NEPSystem needs a HIP GPU; none is visible")
        self.lib = load_library()
        self.device = torch.device(device)
        self.full = full
        self.surrogate = surrogate
        self.n = int(n_atoms)
        self.box = np.ascontiguousarray(box, dtype=np.float64)
        self.cap_radial, self.cap_angular = cap_radial, cap_angular
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = ctypes.c_int64()
        self._check(self.lib.nep_system_workspace_bytes(
            full.handle, surrogate.handle if surrogate else None, self.n, _np_ptr(self.box),
            cap_radial, cap_angular, ctypes.byref(nb)), None)
        self.workspace_bytes = nb.value
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.nep_system_create(
            full.handle, surrogate.handle if surrogate else None, self.n, _np_ptr(self.box),
            cap_radial, cap_angular, _t_ptr(self.workspace), nb.value,
            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None)
        self.handle = h
        self.generation = 0      # bumped by every call that changes positions, lists or buffers
        self._types = None
        self._masses = None

    def _check(self, st, handle="self"):
        if st != 0:
            h = self.handle if handle == "self" else None
            msg = self.lib.nep_last_error(h).decode() if h else ""
            raise NEPError(st, f"{self.lib.nep_status_string(st).decode()}: {msg}")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.nep_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------------ state
    def set_params(self, slot: int, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float64)
        self._check(self.lib.nep_system_set_params(self.handle, slot, _np_ptr(p), p.size))

    def _shape(self, a, shape, name):
        if tuple(a.shape) != shape:
            raise ValueError(f"{name} has shape {tuple(a.shape)}, expected {shape}")

    def set_state(self, x, types, masses, v=None):
        """Positions [N][3] (A), species [N], one mass per species (amu), velocities [N][3]
        (A/fs, optional): host arrays, or device tensors for x, types and v."""
        self.generation += 1
        masses = np.ascontiguousarray(masses, dtype=np.float64).reshape(-1)
        self._shape(masses, (self.full.hp.n_types,), "masses")
        if isinstance(x, torch.Tensor):
            xt = x.to(self.device, torch.float64).contiguous()
            tt = torch.as_tensor(types, device=self.device, dtype=torch.int32).contiguous()
            vt = None if v is None else torch.as_tensor(v).to(self.device, torch.float64).contiguous()
            self._shape(xt, (self.n, 3), "x")
            self._shape(tt, (self.n,), "types")
            if vt is not None:
                self._shape(vt, (self.n, 3), "v")
            self._types, self._masses = types, masses
            self._check(self.lib.nep_set_state(self.handle, _t_ptr(xt), _t_ptr(vt) if vt is not None else None,
                                               _t_ptr(tt), _np_ptr(masses), 1))
            torch.cuda.synchronize(self.device)
            return
        x = np.ascontiguousarray(x, dtype=np.float64)
        t = np.ascontiguousarray(types, dtype=np.int32)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        self._shape(x, (self.n, 3), "x")
        self._shape(t, (self.n,), "types")
        if vv is not None:
            self._shape(vv, (self.n, 3), "v")
        self._types, self._masses = types, masses
        self._check(self.lib.nep_set_state(self.handle, _np_ptr(x), _np_ptr(vv) if vv is not None else None,
                                           _np_ptr(t), _np_ptr(masses), 0))

    def get_state(self):
        x = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        step = ctypes.c_int64()
        self._check(self.lib.nep_get_state(self.handle, _np_ptr(x), _np_ptr(v), ctypes.byref(step), 0))
        return x, v, step.value

    def set_positions(self, x):
        """New positions with the types and masses of the last set_state (velocities zero)."""
        if self._types is None:
            raise RuntimeError("set_state first")
        self.set_state(x, self._types, self._masses)

    def build_neighbors(self, skin: float = 1.0):
        self.generation += 1
        self._check(self.lib.nep_build_neighbors(self.handle, float(skin)))

    def export_neighbors(self, which: int = 0):
        cap = self.cap_radial if which == 0 else self.cap_angular
        offsets = np.zeros(self.n + 1, np.int64)
        idx = np.zeros(self.n * cap, np.int32)
        self._check(self.lib.nep_export_neighbors(self.handle, which, _np_ptr(offsets), _np_ptr(idx),
                                                  idx.size))
        return offsets, idx[: offsets[-1]].copy()

    # ------------------------------------------------------------------ evaluation
    def compute(self, slot: int = 0, precision="fp32", forces: bool = True, per_atom: bool = False,
                on_device: bool = False):
        """(E, W[3][3], F[N][3] or None, U[N] or None), FP64, original atom order."""
        self.generation += 1
        E = ctypes.c_double()
        W = np.zeros(9)
        if on_device:
            F = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if forces else None
            U = torch.empty(self.n, dtype=torch.float64, device=self.device) if per_atom else None
            fp = _t_ptr(F) if F is not None else None
            up = _t_ptr(U) if U is not None else None
        else:
            F = np.zeros((self.n, 3)) if forces else None
            U = np.zeros(self.n) if per_atom else None
            fp = _np_ptr(F) if F is not None else None
            up = _np_ptr(U) if U is not None else None
        self._check(self.lib.nep_compute_energy_forces_virial(
            self.handle, slot, _prec(precision), ctypes.byref(E), _np_ptr(W), fp, up, 1 if on_device else 0))
        return E.value, W.reshape(3, 3), F, U

    def set_deterministic(self, on: bool = True):
        """Fixed-order force accumulation without atomics (bitwise reproducible forces)."""
        self._check(self.lib.nep_set_deterministic(self.handle, 1 if on else 0))

    def step(self, n_steps: int, dt: float = 1.0, rebuild_every: int = 10, skin: float = 1.0,
             mts_k: int = 0, fallback_rms: float = 0.05, fallback_max: float = 1.0, precision="fp32",
             thermo_every: int = 0, max_rows: int = 4096, relative_judge: bool = False):
        """Advance n_steps; returns thermo rows [k][8] (step, PE, KE, T, P, err_rms, err_max, fallback).

        With ``relative_judge`` the MTS fallback thresholds are multiples of each block's rms
        full-model force instead of eV/A."""
        prec = _prec(precision)
        self.generation += 1
        self._check(self.lib.nep_set_judge(self.handle, 1 if relative_judge else 0))
        rows = ctypes.c_int64()
        th = np.zeros((max_rows, 8)) if thermo_every > 0 else None
        self._check(self.lib.nep_step(self.handle, int(n_steps), float(dt), int(rebuild_every), float(skin),
                                      int(mts_k), float(fallback_rms), float(fallback_max), prec,
                                      _np_ptr(th) if th is not None else None, int(max(thermo_every, 1)),
                                      int(max_rows), ctypes.byref(rows)))
        return th[: rows.value].copy() if th is not None else None

    def set_thermostat(self, temperature: float, tau: float = 100.0, chain: int = 3):
        """NVT with a Nose-Hoover chain (chain = 0: back to NVE); resets the chain state."""
        self._check(self.lib.nep_set_thermostat(self.handle, float(temperature), float(tau), int(chain)))
        self._chain = int(chain)

    def set_thermostat_state(self, eta, v_eta):
        """Restore the chain state (after set_thermostat), e.g. from a checkpoint."""
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        ve = np.ascontiguousarray(v_eta, dtype=np.float64)
        m = getattr(self, "_chain", 0)
        if eta.size != m or ve.size != m:
            raise ValueError(f"the chain has {m} thermostats")
        self._check(self.lib.nep_set_thermostat_state(self.handle, _np_ptr(eta), _np_ptr(ve)))

    def get_thermostat(self):
        """(eta, v_eta, chain energy in eV) of the Nose-Hoover chain."""
        m = getattr(self, "_chain", 0)
        eta, ve, e = np.zeros(max(m, 1)), np.zeros(max(m, 1)), ctypes.c_double()
        self._check(self.lib.nep_get_thermostat(self.handle, _np_ptr(eta), _np_ptr(ve), ctypes.byref(e)))
        return eta[:m], ve[:m], e.value

    def stats(self) -> dict:
        s = np.zeros(4, np.int64)
        self._check(self.lib.nep_get_stats(self.handle, _np_ptr(s)))
        return {"list_builds": int(s[0]), "mts_blocks": int(s[1]), "fallback_blocks": int(s[2]),
                "steps": int(s[3])}

    def halo_stats(self) -> dict:
        """Force-halo tables of the last list build: tiles, tiles on the global-atomic
        scatter (halo too large for LDS), largest halo in atoms and in cells."""
        s = np.zeros(4, np.int64)
        self._check(self.lib.nep_halo_stats(self.handle, _np_ptr(s)))
        return {"tiles": int(s[0]), "global_atomic_tiles": int(s[1]), "max_halo_atoms": int(s[2]),
                "max_halo_cells": int(s[3])}

    def profile(self, enable: bool):
        self._check(self.lib.nep_profile(self.handle, 1 if enable else 0))

    def profile_read(self) -> dict:
        """Summed ms and launch counts per kernel group (slot 0 = full model, slot 1 = surrogate)."""
        ms = np.zeros(6)
        cnt = np.zeros(6, np.int64)
        self._check(self.lib.nep_profile_read(self.handle, _np_ptr(ms), _np_ptr(cnt)))
        names = ["desc_net", "force", "rebuild", "integrate", "desc_net_surrogate", "force_surrogate"]
        return {n: (float(ms[k]), int(cnt[k])) for k, n in enumerate(names)}

    def pair_counts(self):
        """(radial pairs, angular pairs, radial skin-list entries) summed over atoms."""
        c = np.zeros(3, np.int64)
        self._check(self.lib.nep_pair_counts(self.handle, _np_ptr(c)))
        return int(c[0]), int(c[1]), int(c[2])

    def surrogate_error(self, precision="fp32"):
        e = np.zeros(2)
        self._check(self.lib.nep_surrogate_error(self.handle, _prec(precision), _np_ptr(e)))
        return float(e[0]), float(e[1])

    # ------------------------------------------------------------------ training
    def train_forward(self, slot: int, theta: torch.Tensor):
        """(E float, F torch [N][3] float32) with network parameters theta (device FP32)."""
        return self._train_forward(self.lib.nep_train_forward, slot, theta, False)

    def train_backward(self, slot: int, theta: torch.Tensor, gE: float, gF: Optional[torch.Tensor],
                       out: Optional[torch.Tensor] = None):
        """dL/dtheta for L = gE*E + sum gF.F (FP32, device); adds into ``out`` when given."""
        return self._train_backward(self.lib.nep_train_backward, slot, theta, gE, gF, out, False)

    def train_forward_params(self, slot: int, params: torch.Tensor):
        """As train_forward with every parameter (packed [cR | cA | sigma | W0 | b0 | w1 | b1])."""
        return self._train_forward(self.lib.nep_train_forward_params, slot, params, True)

    def train_backward_params(self, slot: int, params: torch.Tensor, gE: float, gF: Optional[torch.Tensor],
                              out: Optional[torch.Tensor] = None):
        """dL/dparams in the packed order, including the expansion coefficients and the scaler."""
        return self._train_backward(self.lib.nep_train_backward_params, slot, params, gE, gF, out, True)

    def train_backward64(self, gE: float, gF=None, slot: int = 0) -> torch.Tensor:
        """FP64 dL/dparams (packed order) of L = gE E + sum_i gF_i . F_i, with E and F those of
        the FP64 evaluation of the slot's own parameters; gF [N][3] in original order."""
        hp = (self.full if slot == 0 else self.surrogate).hp
        grad = torch.empty(hp.n_params(), dtype=torch.float64, device=self.device)
        gFc = None
        if gF is not None:
            gFc = torch.as_tensor(gF).detach().to(self.device, torch.float64).contiguous()
            self._shape(gFc, (self.n, 3), "gF")
        self._check(self.lib.nep_train_backward64(self.handle, slot, float(gE),
                                                  _t_ptr(gFc) if gFc is not None else None, _t_ptr(grad)))
        return grad

    def _expect(self, slot, theta, all_params):
        hp = (self.full if slot == 0 else self.surrogate).hp
        n = hp.n_params() if all_params else hp.n_hidden * hp.n_desc + 2 * hp.n_hidden + 1
        if theta.numel() != n:
            raise ValueError(f"parameter vector has {theta.numel()} values, the model in slot {slot} takes {n}")
        return theta.detach().to(self.device, torch.float32).contiguous()

    def _train_forward(self, fn, slot, theta, all_params):
        self.generation += 1
        theta = self._expect(slot, theta, all_params)
        F = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        E = ctypes.c_double()
        self._check(fn(self.handle, slot, _t_ptr(theta), ctypes.byref(E), _t_ptr(F)))
        return E.value, F

    def _device_f32(self, a, n, name):
        if not (isinstance(a, torch.Tensor) and a.dtype == torch.float32 and a.is_contiguous()
                and a.device == self.device and a.numel() == n):
            raise ValueError(f"{name} must be a contiguous float32 tensor of {n} values on {self.device}")

    def _train_backward(self, fn, slot, theta, gE, gF, out, all_params):
        theta = self._expect(slot, theta, all_params)
        acc = out is not None
        if acc:
            self._device_f32(out, theta.numel(), "out")
        grad = out if acc else torch.empty_like(theta)
        gFc = None if gF is None else gF.detach().to(self.device, torch.float32).contiguous()
        if gFc is not None:
            self._shape(gFc, (self.n, 3), "gF")
        self._check(fn(self.handle, slot, _t_ptr(theta), float(gE), _t_ptr(gFc) if gFc is not None else None,
                       _t_ptr(grad), 1 if acc else 0))
        return grad

    def adam(self, theta: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor, t: int,
             lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        for a, name in ((theta, "theta"), (grad, "grad"), (m1, "m1"), (m2, "m2")):
            self._device_f32(a, theta.numel(), name)
        self._check(self.lib.nep_adam_update(self.handle, _t_ptr(theta), _t_ptr(grad), _t_ptr(m1), _t_ptr(m2),
                                             theta.numel(), int(t), lr, beta1, beta2, eps))


def network_params(hp: inputs.HParams, params: np.ndarray) -> np.ndarray:
    """The network block (W0, b0, w1, b1) of a packed parameter vector, as one array."""
    b = inputs.unpack(hp, params)
    return np.concatenate([b["W0"], b["b0"], b["w1"], b["b1"]])


def compute_energy_forces_virial_noalloc(model: NEPModel, x: torch.Tensor, types: torch.Tensor, box,
                                         cap_radial: int = 160, cap_angular: int = 96, skin: float = 1.0,
                                         precision="fp32", forces: Optional[torch.Tensor] = None,
                                         per_atom_energy: Optional[torch.Tensor] = None,
                                         stream: Optional[torch.cuda.Stream] = None):
    """Energy, virial [3][3] and, into the given device tensors, forces [N][3] and per-atom
    energies [N] (FP64) of one configuration through the library's allocation-free call:
    x [N][3] FP64 and types [N] int32 are device tensors; the library's fixed device scratch
    replaces a system workspace. Returns (E, W)."""
    lib = load_library()
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.dim() == 2
            and x.shape[1] == 3 and x.is_contiguous()):
        raise ValueError("x must be a contiguous [N][3] float64 device tensor")
    n = x.shape[0]
    if not (isinstance(types, torch.Tensor) and types.is_cuda and types.dtype == torch.int32
            and tuple(types.shape) == (n,) and types.is_contiguous()):
        raise ValueError("types must be a contiguous [N] int32 device tensor")
    for t, shape, name in ((forces, (n, 3), "forces"), (per_atom_energy, (n,), "per_atom_energy")):
        if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                                  and tuple(t.shape) == shape and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {list(shape)} float64 device tensor")
    b = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    E = ctypes.c_double()
    W = np.zeros(9)
    st_obj = stream if stream is not None else torch.cuda.current_stream(x.device)
    st = lib.nep_compute_energy_forces_virial_noalloc(
        model.handle, n, _np_ptr(b), int(cap_radial), int(cap_angular), float(skin), _t_ptr(x), _t_ptr(types),
        _prec(precision), ctypes.byref(E), _np_ptr(W), _t_ptr(forces) if forces is not None else None,
        _t_ptr(per_atom_energy) if per_atom_energy is not None else None, ctypes.c_void_p(st_obj.cuda_stream))
    if st != 0:
        raise NEPError(st, lib.nep_status_string(st).decode())
    return E.value, W.reshape(3, 3)
