"""Benchmark of the NEP molecular-dynamics step on one MI355X.

Default workload: FCC Cu-like box of 100 x 100 x 100 unit cells (4,000,000 atoms,
a = 3.615 A, Gaussian displacements sigma = 0.08 A, 600 K Maxwell-Boltzmann
velocities), the full NEP (radial 6 A / angular 5 A cutoffs, n_max 4, basis 8,
l_max 4 + four-body, 30 hidden units) with random N(0, 0.1) weights, FP32
descriptors and forces, FP32 MFMA network, FP64 integration; velocity Verlet at
1 fs, neighbour lists rebuilt every 10 steps with a 1 A skin, thermo output
every 100 steps. One "step" is one MD step of the whole path (integration,
conditional list rebuild, descriptors, network, forces, virial, reductions).

Prints one JSON line: atom-steps/s on one GPU, the roofline of the dominant
kernel (the force kernel, timed with HIP events on the library's stream over
the timed region) and the FP64 CPU oracle timed on this host's cores.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak (packed FMA)
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense bfloat16 matrix peak (no sparsity)

# Static FLOP counts per unit (FMA = 2 flops) of the method's definition, counted per
# pair inside the true cutoff or per atom (the basis and its derivative, the channel
# contractions, harmonics and their gradients, the network). Units are pairs inside
# the true cutoffs and atoms.
FLOPS = {
    "full": {
        "force_radial_pair": 346,
        "force_angular_pair": 1222,
        "desc_candidate_pair": 8,        # FP64 distance test of each skin-list entry
        "desc_radial_pair": 160,
        "desc_angular_pair": 460,
        "desc_per_atom": 5000,           # q_nl, four-body, network (2 x 2 x 30 x 30) and dU/ds
    },
    "surrogate": {                       # l_max 2 (8 harmonics), no four-body, 8 hidden units
        "force_radial_pair": 346,
        "force_angular_pair": 615,
        "desc_candidate_pair": 8,
        "desc_radial_pair": 160,
        "desc_angular_pair": 270,
        "desc_per_atom": 1000,
    },
}


FORCE_SOURCES = ("nep_eval.hip", "nep_kernels.h", "nep_poly.h", "nep_common.h")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_force_fcc4m_fp32_hbm_traffic.md")


def force_sources_digest():
    """SHA-256 of the code the force kernel is compiled from: its sources with // comments
    and blank lines removed, so that a comment edit does not disown the measured counters."""
    import hashlib
    h = hashlib.sha256()
    for name in FORCE_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_24816_amd", "csrc", name), encoding="utf-8") as f:
            for line in f:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode("utf-8") + b"\n")
    return h.hexdigest()


def force_traffic():
    """HBM bytes per k_force launch from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the same counter's reading for a plain copy of known
    size), or None when the force kernel's sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            lines = [ln for ln in f if ln.startswith("traffic-json: ")]
        rec = json.loads(lines[-1][len("traffic-json: "):])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("sources_sha256") != force_sources_digest():
        return None
    return rec["bytes_per_launch"]


def flops_per_atom(pairs_r, pairs_a, skin_entries, model="full"):
    f = FLOPS[model]
    force = f["force_radial_pair"] * pairs_r + f["force_angular_pair"] * pairs_a
    desc = (f["desc_candidate_pair"] * skin_entries + f["desc_radial_pair"] * pairs_r +
            f["desc_angular_pair"] * pairs_a + f["desc_per_atom"])
    return desc, force


def cpu_baseline(hp, params, at, seconds):
    """The FP64 oracle's per-center work on a bounded run of consecutive atoms of the same
    box. Two short calls separate the per-call cell-list setup from the per-atom cost; the
    timed call is then sized to take about `seconds`."""
    import oracle
    m = oracle.Model.from_hparams(hp, params)
    k0, k1 = 2000, 20000
    t = time.perf_counter()
    oracle.center_work(m, at.x, at.types, at.box, 0, k0)
    t0 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.center_work(m, at.x, at.types, at.box, k0, k1)
    t1 = time.perf_counter() - t
    per_atom = max((t1 - t0) / (k1 - k0), 1e-9)
    setup = max(t0 - k0 * per_atom, 0.0)
    k = int(min(at.n - k0 - k1, max(k1, (seconds - setup) / per_atom)))
    t = time.perf_counter()
    oracle.center_work(m, at.x, at.types, at.box, k0 + k1, k)
    dt = time.perf_counter() - t
    return {"value": k / dt, "unit": "atom-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"per-center work of one force evaluation (descriptors, network, every pair "
                      f"derivative) for {k} consecutive atoms of the same {at.n}-atom box, FP64 C++ "
                      f"oracle with OpenMP, {dt:.1f} s including the cell-list setup of the whole box "
                      f"({setup:.1f} s)"}


def run_form(form, hp, params, at, steps, warmup, sur=None, judge_fraction=0.75, mts_k=4):
    """Time one form on one box: 'fp32', 'bf16', 'mts' (mts_k surrogate inner steps per
    full-model step) or 'mts_bf16' (the same with the bfloat16 network in both models).
    An MTS run times the largest multiple of mts_k not above `steps`."""
    mts = form.startswith("mts")
    import torch
    from paper_2604_24816_amd import nep
    from paper_2604_24816_amd import surrogate as SG
    shp, sp = sur if sur is not None else (None, None)
    s = nep.NEPSystem(nep.NEPModel(hp, params), at.n, at.box,
                      surrogate=nep.NEPModel(shp, sp) if mts else None)
    s.set_state(at.x, at.types, at.masses, at.v)
    s.build_neighbors(1.0)
    prec = "bf16" if form in ("bf16", "mts_bf16") else "fp32"
    k = mts_k if mts else 0
    if mts:
        steps = k * (steps // k)
        warmup = k * max(1, warmup // k)
    kw = dict(dt=1.0, rebuild_every=10, skin=1.0, precision=prec, mts_k=k)
    extra = {}
    if mts:
        # each block is judged against its own full-model force scale
        _, _, rms = SG.judge_thresholds(s, judge_fraction)
        kw.update(fallback_rms=judge_fraction, fallback_max=10.0, relative_judge=True)
        extra["judge"] = {"mode": "relative to the block's rms full-model force", "fraction_rms": judge_fraction,
                          "factor_max": 10.0, "rms_force_full_at_start": rms}
    s.step(warmup, **kw)
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = s.step(steps, thermo_every=k if k else 100, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    n = at.n
    if mts:
        # pair counts are those of the last evaluation, which in an MTS run is the full
        # model's; the surrogate's roofline needs its own, at its own cutoffs
        s.compute(slot=1, precision=prec, on_device=True)
    pr, pa, sk = s.pair_counts()
    model_name = "surrogate" if mts else "full"
    grp = "force_surrogate" if mts else "force"
    desc_f, force_f = flops_per_atom(pr / n, pa / n, sk / n, model_name)
    fms, fcnt = prof[grp]
    out = {"atom_steps_per_s": n * steps / elapsed, "s_per_step_per_atom": elapsed / (n * steps),
           "ms_per_step": 1e3 * elapsed / steps, "n_atoms": n, "steps": steps,
           "kernels_ms_per_launch": {kk: (v[0] / v[1] if v[1] else None) for kk, v in prof.items()},
           "roofline": {"bound": "alu", "kernel": "k_force" + ("<surrogate>" if mts else ""),
                        "achieved": force_f * n / (fms / fcnt / 1e3) / 1e12, "peak": PEAK_FP32_VECTOR_TFLOPS,
                        "unit": "TFLOP/s"},
           "energy_drift_per_atom": float((th[-1, 1] + th[-1, 2] - th[0, 1] - th[0, 2]) / n) if len(th) > 1 else None}
    if mts:
        out["mts_k"] = k
    out["roofline"]["frac"] = out["roofline"]["achieved"] / PEAK_FP32_VECTOR_TFLOPS
    if mts:
        st = s.stats()
        out.update(extra)
        out["surrogate_force_error_rms_mean"] = float(np.mean(th[:, 5]))
        out["surrogate_force_error_max"] = float(np.max(th[:, 6]))
        out["block_error_rms"] = [round(float(e), 6) for e in th[:, 5]]
        out["block_error_max"] = [round(float(e), 5) for e in th[:, 6]]
        out["block_fallback"] = [int(e) for e in th[:, 7]]
        out["mts_blocks"] = st["mts_blocks"]
        out["fallback_blocks"] = st["fallback_blocks"]
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def run_forms(args):
    """32M-atom box: FP32, BF16 and MTS with a surrogate trained here on the GPU, plus the
    untrained-surrogate MTS run that shows what training gains."""
    import torch
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import surrogate as SG
    hp = I.FULL_HPARAMS
    params = I.random_model(hp, 0)
    shp = I.SURROGATE_HPARAMS
    sur0 = I.surrogate_from_teacher(hp, params, shp, 1)
    t = time.perf_counter()
    fr = SG.generate_frames(hp, params, n_traj=200, cells=10, steps=100, every=10)
    t_frames = time.perf_counter() - t
    n_frames = int(fr.x.shape[0])
    shp_s = I.SURROGATE_SHORT_HPARAMS   # the same surrogate with 5 / 4 A cutoffs (fewer pairs per step)
    sur0_s = I.surrogate_from_teacher(hp, params, shp_s, 1)
    shp_t = I.SURROGATE_SHORTER_HPARAMS  # 4 / 3 A: two radial shells, one angular shell
    sur0_t = I.surrogate_from_teacher(hp, params, shp_t, 1)

    def train(label, h, p0, coeffs):
        def log(msg):
            if msg.startswith("epoch") and int(msg.split()[1].rstrip(":")) % 10 == 9:
                print(f"  {label} {msg}", file=sys.stderr, flush=True)
        r = SG.train_surrogate(fr, h, p0, epochs=args.epochs, batch=8, lr=1e-2, lr_end=1e-4,
                               train_coeffs=coeffs, log=log)
        print(f"trained surrogate {label}: held-out force RMSE {r.val_force_rmse_init:.4f} -> "
              f"{r.val_force_rmse:.4f} eV/A ({r.seconds:.1f} s)", file=sys.stderr, flush=True)
        return r
    res = train("6/5 A", shp, sur0, False)
    res_c = train("6/5 A, coefficients", shp, sur0, True)
    res_s = train("5/4 A", shp_s, sur0_s, False)
    res_sc = train("5/4 A, coefficients", shp_s, sur0_s, True)
    res_tc = train("4/3 A, coefficients", shp_t, sur0_t, True)
    del fr
    torch.cuda.empty_cache()
    at = I.workload_32m(args.cells)
    forms = {}
    for form in ("fp32", "bf16"):
        forms[form] = run_form(form, hp, params, at, args.steps, args.warmup)
        print(f"form {form}: {forms[form]['atom_steps_per_s']:.3e} atom-steps/s", file=sys.stderr, flush=True)
    wm = 4 * max(1, args.warmup // 4)
    for name, sur in (("mts_trained_coeffs", (shp, res_c.params)), ("mts_trained", (shp, res.params)),
                      ("mts_untrained", (shp, sur0)), ("mts_short_trained_coeffs", (shp_s, res_sc.params)),
                      ("mts_short_trained", (shp_s, res_s.params)), ("mts_short_untrained", (shp_s, sur0_s)),
                      ("mts_short_trained_coeffs_bf16", (shp_s, res_sc.params)),
                      ("mts_short_trained_coeffs_k8", (shp_s, res_sc.params)),
                      ("mts_shorter_trained_coeffs", (shp_t, res_tc.params)),
                      ("mts_shorter_untrained", (shp_t, sur0_t))):
        # the last form: the full model every 8 steps instead of 4 (same judge)
        forms[name] = run_form("mts_bf16" if name.endswith("_bf16") else "mts", hp, params, at, args.steps, wm,
                               sur=sur, mts_k=8 if name.endswith("_k8") else 4)
        print(f"form {name}: {forms[name]['atom_steps_per_s']:.3e} atom-steps/s, "
              f"{forms[name]['mts_blocks']} MTS / {forms[name]['fallback_blocks']} fallback blocks",
              file=sys.stderr, flush=True)
    out = {"metric": "atom-steps/s per GPU (s/step/atom): plain FP32 NEP vs BF16/MTS surrogate",
           "value": forms["mts_shorter_trained_coeffs"]["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic (seeded FCC box, random-weight NEP)",
           "config": {"workload": f"fcc_cu_{args.cells}^3_cells_{at.n}_atoms_forms", "n_atoms": at.n,
                      "value_form": "mts_shorter_trained_coeffs (4/3 A surrogate, coefficients and network "
                                    "trained, k = 4, judged every block against 0.75 x the block's rms full-model "
                                    "force)"},
           "training": {"frames": n_frames, "frame_generation_s": t_frames, "epochs": args.epochs,
                        "lr": "cosine 1e-2 -> 1e-4",
                        **{name: {"seconds": r.seconds, "loss_history": r.history,
                                  "val_force_rmse_init": r.val_force_rmse_init, "val_force_rmse": r.val_force_rmse,
                                  "val_energy_mae_init": r.val_energy_mae_init, "val_energy_mae": r.val_energy_mae}
                           for name, r in (("teacher_cutoffs", res), ("teacher_cutoffs_coeffs", res_c),
                                           ("short_cutoffs", res_s), ("short_cutoffs_coeffs", res_sc),
                                           ("shorter_cutoffs_coeffs", res_tc))}},
           "forms": forms}
    print(json.dumps(out))


def mts_on_workload(args, hp, params, at, fp32_value):
    """The MTS form on the benchmark's own box: the 4 / 3 A surrogate (coefficients and
    network) trained here on the GPU from full-model frames, then r-RESPA with k = 4 and
    the relative judge, timed like the plain run. Reported beside `value`, not in it."""
    import torch
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import surrogate as SG
    shp = I.SURROGATE_SHORTER_HPARAMS
    sur0 = I.surrogate_from_teacher(hp, params, shp, 1)
    t = time.perf_counter()
    fr = SG.generate_frames(hp, params, n_traj=200, cells=10, steps=100, every=10)

    def log(msg):
        if msg.startswith("epoch") and int(msg.split()[1].rstrip(":")) % 10 == 9:
            print(f"  surrogate {msg}", file=sys.stderr, flush=True)
    r = SG.train_surrogate(fr, shp, sur0, epochs=args.epochs, batch=8, lr=1e-2, lr_end=1e-4, train_coeffs=True,
                           log=log)
    t_train = time.perf_counter() - t
    del fr
    torch.cuda.empty_cache()
    f = run_form("mts_bf16" if args.precision == "bf16" else "mts", hp, params, at, args.steps, args.warmup,
                 sur=(shp, r.params))
    return {"form": "r-RESPA k = 4, 4/3 A surrogate (coefficients and network trained on 2,000 full-model "
                    "frames, 40 epochs), relative judge 0.75 x the block's rms full-model force",
            "atom_steps_per_s": f["atom_steps_per_s"], "ms_per_step": f["ms_per_step"],
            "s_per_step_per_atom": f["s_per_step_per_atom"], "vs_plain": f["atom_steps_per_s"] / fp32_value,
            "mts_blocks": f["mts_blocks"], "fallback_blocks": f["fallback_blocks"],
            "surrogate_force_error_rms_mean": f["surrogate_force_error_rms_mean"],
            "energy_drift_per_atom": f["energy_drift_per_atom"],
            "surrogate_val_force_rmse": r.val_force_rmse, "frames_and_training_s": t_train,
            "kernels_ms_per_launch": f["kernels_ms_per_launch"]}


def network_mfma(hp, n, desc_ms, precision):
    """MFMA use of the network inside the descriptor kernel: the forward product W0 q~ and
    the backward product W0^T (w1 (1 - t^2)), 2 * 2 * H * D flops per atom (unpadded),
    over the whole descriptor+network launch, against the dense MFMA peak of the
    operand type."""
    flops = 4.0 * hp.n_hidden * hp.n_desc
    achieved = flops * n / (desc_ms * 1e-3) / 1e12
    peak = PEAK_BF16_MFMA_TFLOPS if precision == "bf16" else PEAK_FP32_MFMA_TFLOPS
    return {"kernel": "k_desc_net (network part)", "flops_per_atom": flops, "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}


def integrator_hbm(n, integrate, steps):
    """HBM bandwidth of the velocity-Verlet kernels: k_kick_drift reads type, v, F, x and
    the build positions and writes v, x and the record's position (88 + 72 B per atom);
    k_kick reads type, F, v and writes v (40 + 24 B)."""
    total_ms, launches = integrate
    per_step_s = total_ms * 1e-3 / steps
    nbytes = 224.0 * n
    achieved = nbytes / per_step_s / 1e9
    return {"kernels": "k_kick_drift + k_kick", "bytes_per_atom_step": 224, "achieved": achieved,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "timed_segments": launches}


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain copy of known size: reads nbytes and writes nbytes per launch."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                                           "launches": reps}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cells", type=int, default=100, help="FCC cells per side")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", action="store_true",
                    help="time FP32, BF16 and surrogate MTS on the 200^3-cell (32M-atom) box instead")
    ap.add_argument("--epochs", type=int, default=40, help="surrogate training epochs")
    ap.add_argument("--nvt", type=float, default=0.0,
                    help="run NVT at this temperature (K) with a Nose-Hoover chain of 3, tau 100 fs")
    ap.add_argument("--zbl", type=float, default=0.0,
                    help="add the ZBL repulsion with this outer radius in A (the paper's Cu model uses 2.0)")
    ap.add_argument("--no-mts", action="store_true",
                    help="skip the MTS form on the benchmark box (trains a surrogate first, about a minute)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference kernel "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the library computes one GPU's share; the spatial decomposition with a halo "
              f"exchange across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    if args.forms:
        if args.cells == 100:
            args.cells = 200
        run_forms(args)
        return

    import torch
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import nep

    hp = I.FULL_HPARAMS
    if args.zbl > 0:
        hp = dataclasses.replace(hp, zbl_outer=args.zbl)
    params = I.random_model(hp, 0)
    at = I.workload_4m(args.cells)
    s = nep.NEPSystem(nep.NEPModel(hp, params), at.n, at.box)
    s.set_state(at.x, at.types, at.masses, at.v)
    s.build_neighbors(1.0)
    if args.nvt > 0:
        s.set_thermostat(args.nvt, tau=100.0, chain=3)
    s.step(args.warmup, dt=1.0, rebuild_every=10, skin=1.0, precision=args.precision)
    # timed region
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps, dt=1.0, rebuild_every=10, skin=1.0, precision=args.precision, thermo_every=100)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    elapsed = t1 - t0
    n = at.n
    value = n * args.steps / elapsed
    pairs_r, pairs_a, skin_total = s.pair_counts()
    skin_entries = skin_total / n
    desc_f, force_f = flops_per_atom(pairs_r / n, pairs_a / n, skin_entries)
    force_ms, force_cnt = prof["force"]
    desc_ms, desc_cnt = prof["desc_net"]
    avg_force_s = force_ms / force_cnt / 1e3
    achieved = force_f * n / avg_force_s / 1e12
    out = {
        "metric": "atom-steps/s per GPU (s/step/atom): plain FP32 NEP vs BF16/MTS surrogate",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "s_per_step_per_atom": elapsed / (n * args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if args.precision == "fp32" else "fp32+bf16-mfma",
        "data": "synthetic (seeded FCC box, random-weight NEP)",
        "config": {"workload": f"fcc_cu_{args.cells}x{args.cells}x{args.cells}_cells_{n}_atoms_"
                               + (f"nvt_{args.nvt:g}K" if args.nvt > 0 else "nve"),
                   "n_atoms": n, "model": "NEP rc 6/5 A, n_max 4, basis 8, l_max 4 + 4-body, 30 hidden"
                   + (f", ZBL outer {args.zbl} A" if args.zbl > 0 else ""),
                   "precision": args.precision, "dt_fs": 1.0, "rebuild_every": 10, "skin_A": 1.0,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_force", "achieved": achieved,
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": force_traffic(),
                     "flops_per_atom": force_f, "avg_launch_ms": avg_force_s * 1e3},
        "network_mfma": network_mfma(hp, n, desc_ms / desc_cnt, args.precision),
        "integrator_hbm": integrator_hbm(n, prof["integrate"], args.steps),
        "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
        "pairs_per_atom": {"radial": pairs_r / n, "angular": pairs_a / n, "skin_list": skin_entries},
        "flops_per_atom_step": desc_f + force_f,
        "sustained_tflops": (desc_f + force_f) * value / 1e12,
        "paper_context": {"note": "Table 5, CNIS GPGPU, trained Cu model, 4,499,456 atoms, FP32",
                          "atom_steps_per_s": 46.19e6},
    }
    if not args.no_mts and args.nvt <= 0 and args.zbl <= 0 and args.steps >= 4:
        s.close()
        del s
        torch.cuda.empty_cache()
        out["mts"] = mts_on_workload(args, hp, params, at, value)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(hp, params, at, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
