"""Distilled surrogate NEP: frame generation with full-NEP MD, training on the GPU with the
library's own forward/backward kernels and Adam, and the multiple-time-step driver.

The surrogate has 8 hidden units, n_max 4, l_max 2 and no four-body term; its
descriptor coefficients start as a copy of the full model's. By default they stay
frozen and only the network (8 x 15 + 8 + 8 + 1 = 137 parameters) is trained, on
energy and force MSE against the full model's labels; with ``train_coeffs`` the 90
radial and angular expansion coefficients are trained as well, as the paper's
description of c as trainable allows. Every arithmetic step of training runs in the
library's kernels (descriptors, network, forces, parameter gradients, Adam); torch
only holds the arrays and forms the loss residuals.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import inputs as I
from .nep import NEPModel, NEPSystem, network_params


@dataclasses.dataclass
class Frames:
    x: torch.Tensor        # [F][N][3] float64, device
    E: np.ndarray          # [F] float64 (full-model energies)
    F: torch.Tensor        # [F][N][3] float32, device (full-model forces)
    types: np.ndarray
    masses: np.ndarray
    box: np.ndarray
    temps: np.ndarray      # [F] target temperature of the trajectory each frame came from


def generate_frames(full_hp: I.HParams, full_params: np.ndarray, n_traj: int = 200, cells: int = 10,
                    steps: int = 100, every: int = 10, t_min: float = 300.0, t_max: float = 1200.0,
                    seed: int = 100, skin: float = 1.0, cap_radial: int = 256,
                    cap_angular: int = 160) -> Frames:
    """Full-NEP FP32 MD: n_traj trajectories at T_j = t_min + (t_max - t_min) j/(n_traj - 1), each
    started from an FCC box with displacements 0.083 sqrt(T/300) A and MB(T) velocities (the
    production workload's recipe); a frame every `every` steps. Many short trajectories keep the
    frames in the near-lattice regime the production runs sample (the default gives 2,000 frames)."""
    xs, es, fs, ts = [], [], [], []
    box = types = masses = None
    model = NEPModel(full_hp, full_params)
    for j in range(n_traj):
        T = t_min + (t_max - t_min) * j / max(n_traj - 1, 1)
        at = I.fcc_box(cells, 0.083 * np.sqrt(T / 300.0), seed + j)
        v = I.maxwell_boltzmann(at, T, seed + 1000 + j)
        s = NEPSystem(model, at.n, at.box, cap_radial=cap_radial, cap_angular=cap_angular)
        s.set_state(at.x, at.types, at.masses, v)
        s.build_neighbors(skin)
        for _ in range(steps // every):
            s.step(every, dt=1.0, rebuild_every=10, skin=skin)
            x, _, _ = s.get_state()
            E, _, F, _ = s.compute(forces=True, on_device=True)
            xs.append(torch.tensor(x, device=s.device))
            es.append(E)
            fs.append(F.to(torch.float32))
            ts.append(T)
        box, types, masses = at.box, at.types, at.masses
        s.close()
    return Frames(torch.stack(xs), np.array(es), torch.stack(fs), types, masses, box, np.array(ts))


@dataclasses.dataclass
class TrainResult:
    params: np.ndarray           # packed FP64 surrogate parameters after training
    history: List[float]         # mean training loss per epoch
    val_force_rmse_init: float   # eV/A, surrogate vs full on held-out frames, before training
    val_force_rmse: float        # after training
    val_energy_mae_init: float   # eV/atom
    val_energy_mae: float
    seconds: float


def _with_network(hp: I.HParams, params: np.ndarray, theta: np.ndarray) -> np.ndarray:
    p = params.copy()
    a = hp.offsets()["W0"][0]
    p[a:] = theta
    return p


def evaluate_frames(system: NEPSystem, frames: Frames, idx, theta: torch.Tensor, skin: float = 1.0,
                    all_params: bool = False):
    """(force RMSE eV/A, energy MAE eV/atom) of model theta (slot 0) against the labels;
    theta holds the network block, or every parameter when ``all_params``."""
    se, ae, cnt = 0.0, 0.0, 0
    n = frames.x.shape[1]
    fwd = system.train_forward_params if all_params else system.train_forward
    for f in idx:
        system.set_state(frames.x[f], frames.types, frames.masses)
        system.build_neighbors(skin)
        E, F = fwd(0, theta)
        d = (F - frames.F[f]).double()
        se += float((d * d).sum())
        ae += abs(E - frames.E[f]) / n
        cnt += 1
    return float(np.sqrt(se / (3 * n * cnt))), ae / cnt


def train_surrogate(frames: Frames, sur_hp: I.HParams, sur_params: np.ndarray, epochs: int = 10,
                    batch: int = 8, lr: float = 1e-3, lam_e: float = 1.0, lam_f: float = 1.0,
                    val_fraction: float = 0.1, seed: int = 0, skin: float = 1.0,
                    cap_radial: int = 256, cap_angular: int = 160, train_coeffs: bool = False,
                    lr_end: Optional[float] = None, log=None) -> TrainResult:
    """Adam on energy + force MSE, mini-batches of `batch` frames, on the GPU.

    The network block is trained; with ``train_coeffs`` the radial and angular expansion
    coefficients c are trained too (the descriptor scaler stays fixed). With ``lr_end`` the
    step size follows a cosine from ``lr`` down to ``lr_end`` over all steps."""
    t0 = time.perf_counter()
    nf, n = frames.x.shape[0], frames.x.shape[1]
    rng = np.random.default_rng(seed)
    order = rng.permutation(nf)
    nval = max(1, int(round(val_fraction * nf)))
    val, tr = order[:nval], order[nval:]
    s = NEPSystem(NEPModel(sur_hp, sur_params), n, frames.box, cap_radial=cap_radial, cap_angular=cap_angular)
    if train_coeffs:
        theta = torch.tensor(sur_params, dtype=torch.float32, device=s.device)
        fwd, bwd = s.train_forward_params, s.train_backward_params
        frozen = slice(*sur_hp.offsets()["sigma"])
    else:
        theta = torch.tensor(network_params(sur_hp, sur_params), dtype=torch.float32, device=s.device)
        fwd, bwd = s.train_forward, s.train_backward
        frozen = None
    m1 = torch.zeros_like(theta)
    m2 = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    rmse0, mae0 = evaluate_frames(s, frames, val, theta, skin, train_coeffs)
    history, step = [], 0
    total = epochs * max(1, len(tr) // batch)
    for ep in range(epochs):
        perm = rng.permutation(tr)
        tot = 0.0
        for b0 in range(0, len(perm) - batch + 1, batch):
            grad.zero_()
            for f in perm[b0:b0 + batch]:
                s.set_state(frames.x[f], frames.types, frames.masses)
                s.build_neighbors(skin)
                E, F = fwd(0, theta)
                de = (E - frames.E[f]) / n
                dF = F - frames.F[f]
                tot += lam_e * de * de + lam_f * float((dF.double() ** 2).sum()) / (3 * n)
                gE = 2.0 * lam_e * de / n / batch
                gF = (2.0 * lam_f / (3 * n * batch)) * dF
                bwd(0, theta, gE, gF, out=grad)
            if frozen is not None:
                grad[frozen] = 0.0   # Adam then leaves these entries unchanged
            lr_t = lr if lr_end is None else lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * step / total))
            step += 1
            s.adam(theta, grad, m1, m2, step, lr=lr_t)
        history.append(tot / max(1, (len(perm) // batch) * batch))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.4e}")
    rmse, mae = evaluate_frames(s, frames, val, theta, skin, train_coeffs)
    if train_coeffs:
        params = theta.double().cpu().numpy()
        params[frozen] = sur_params[frozen]
    else:
        params = _with_network(sur_hp, sur_params, theta.double().cpu().numpy())
    s.close()
    return TrainResult(params, history, rmse0, rmse, mae0, mae, time.perf_counter() - t0)


def judge_thresholds(system: NEPSystem, fraction: float = 0.75, max_factor: float = 10.0):
    """Fallback thresholds from the full model's force scale at the current positions:
    tau_rms = fraction * rms(F_full) per component, tau_max = max_factor * rms(F_full).

    An untrained surrogate has a force error at least as large as the forces themselves
    (errors and forces uncorrelated), so fraction < 1 separates it from a useful one."""
    _, _, F, _ = system.compute(slot=0, forces=True, on_device=True)
    rms = float(torch.sqrt(torch.mean(F * F)))
    return fraction * rms, max_factor * rms, rms
