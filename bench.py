"""Benchmark of the NEP molecular-dynamics step on one MI355X.

Default workload: FCC Cu-like box of 200 x 200 x 200 unit cells (32,000,000 atoms,
a = 3.615 A, Gaussian displacements sigma = 0.08 A, 600 K Maxwell-Boltzmann
velocities), the full NEP (radial 6 A / angular 5 A cutoffs, n_max 4, basis 8,
l_max 4 + four-body, 30 hidden units) with random N(0, 0.1) weights, FP64
integration; velocity Verlet at 1 fs, neighbour lists rebuilt every 10 steps with
a 1 A skin. One "step" is one MD step of the whole path (integration, conditional
list rebuild, descriptors, network, forces, virial, reductions).

The same box is timed in four forms, each from the same initial state:
  fp32      FP32 descriptors and forces, FP32 MFMA network (the line's `value`);
  bf16      the network's matrix operands in bfloat16 (FP32 accumulation);
  mts       r-RESPA with k = 4: a 4/3 A surrogate (l_max 2, 8 hidden units; expansion
            coefficients and network trained here on the GPU from full-model frames)
            for the inner steps, the full model every 4 steps, every block judged
            against 0.75 x the block's rms full-model force (fallback to the full model);
  mts_bf16  the same with the bfloat16 network in both models;
plus the untrained surrogate in the same MTS run (what training gains).

Prints one JSON line: atom-steps/s of the fp32 form on one GPU, the roofline of its
dominant kernel (HIP events on the library's stream over the timed region), every
form with its own per-kernel rooflines, and the FP64 CPU oracle timed on this
host's cores.
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

METRIC = "atom-steps/s per GPU (s/step/atom): plain FP32 NEP vs BF16/MTS surrogate"

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

# profile groups of nep_profile_read: (group, model, kernel part, kernel name)
KERNEL_GROUPS = (("desc_net", "full", "desc", "k_desc_net<full>"),
                 ("force", "full", "force", "k_force<full>"),
                 ("desc_net_surrogate", "surrogate", "desc", "k_desc_net<surrogate>"),
                 ("force_surrogate", "surrogate", "force", "k_force<surrogate>"))

FORCE_SOURCES = ("nep_eval.hip", "nep_kernels.h", "nep_poly.h", "nep_common.h", "nep_fast.h")


def workload_tag(cells):
    n = 4 * cells ** 3
    return f"fcc{n // 1000000}m" if n % 1000000 == 0 else f"fcc{n}"


def traffic_summary_path(cells):
    return os.path.join(ROOT, "profiles", f"k_force_{workload_tag(cells)}_fp32_hbm_traffic.md")


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


def force_traffic(cells):
    """HBM bytes per k_force launch on this workload from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a plain
    copy of known size), or None when there is none for this box or the force kernel's
    sources changed since the counters were taken."""
    try:
        with open(traffic_summary_path(cells)) as f:
            lines = [ln for ln in f if ln.startswith("traffic-json: ")]
        rec = json.loads(lines[-1][len("traffic-json: "):])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("sources_sha256") != force_sources_digest() or rec.get("n_atoms") != 4 * cells ** 3:
        return None
    return rec["bytes_per_launch"]


def flops_per_atom(pairs_r, pairs_a, skin_entries, model="full"):
    f = FLOPS[model]
    force = f["force_radial_pair"] * pairs_r + f["force_angular_pair"] * pairs_a
    desc = (f["desc_candidate_pair"] * skin_entries + f["desc_radial_pair"] * pairs_r +
            f["desc_angular_pair"] * pairs_a + f["desc_per_atom"])
    return desc, force


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(hp, params, at_big, seconds):
    """The FP64 oracle as it stands, on this host's cores.

    value: the small 10^3-cell box (4,000 atoms, sigma 0.05 A, 300 K) end to end, ten
    velocity-Verlet steps (force evaluations with cell lists, integration), on every core
    the oracle uses; the same on one core; and, beside them, the per-center work of a force
    evaluation (descriptors, network, every pair derivative) on a bounded run of consecutive
    atoms of the benchmark box itself, sized to take about `seconds`."""
    import oracle
    from paper_2604_24816_amd import inputs as I
    m = oracle.Model.from_hparams(hp, params)
    small = I.workload_small()
    all_threads = oracle.num_threads()
    runs = {}
    for label, nt in (("one_core", 1), ("all_cores", all_threads)):
        oracle.set_num_threads(nt)
        t = time.perf_counter()
        oracle.velocity_verlet(m, small.x, small.v, small.types, small.masses, small.box, 1.0, 0)
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        oracle.velocity_verlet(m, small.x, small.v, small.types, small.masses, small.box, 1.0, 10)
        t_run = time.perf_counter() - t
        steps_s = max(t_run - t_setup, 1e-9)   # ten steps without the initial evaluation
        runs[label] = {"threads": nt, "seconds_10_steps": steps_s, "atom_steps_per_s": small.n * 10 / steps_s,
                       "s_per_step_per_atom": steps_s / (small.n * 10)}
    oracle.set_num_threads(all_threads)
    # per-center work on the benchmark box
    k0, k1 = 2000, 20000
    t = time.perf_counter()
    oracle.center_work(m, at_big.x, at_big.types, at_big.box, 0, k0)
    t0 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.center_work(m, at_big.x, at_big.types, at_big.box, k0, k1)
    t1 = time.perf_counter() - t
    per_atom = max((t1 - t0) / (k1 - k0), 1e-9)
    setup = max(t0 - k0 * per_atom, 0.0)
    k = int(min(at_big.n - k0 - k1, max(k1, (seconds - setup) / per_atom)))
    t = time.perf_counter()
    oracle.center_work(m, at_big.x, at_big.types, at_big.box, k0 + k1, k)
    dt = time.perf_counter() - t
    per_center = {"threads": all_threads, "atoms": k, "seconds": dt, "cell_list_setup_s": setup,
                  "atom_evaluations_per_s": k / max(dt - setup, 1e-9)}
    return {"value": runs["all_cores"]["atom_steps_per_s"], "unit": "atom-steps/s", "cores": all_threads,
            "kind": "oracle",
            "sample": f"FP64 C++ oracle (OpenMP) on the {small.n}-atom 10^3-cell FCC box, ten velocity-Verlet "
                      f"steps end to end (cell lists, descriptors, network, forces, integration) timed without "
                      f"the initial evaluation, {all_threads} threads; the same on 1 thread, and the per-center "
                      f"work of one force evaluation for {k} consecutive atoms of the {at_big.n}-atom box",
            "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": cpu_model_name(),
            "end_to_end": runs, "per_center_benchmark_box": per_center}


def kernel_rooflines(prof, steps, n, counts):
    """Per-kernel achieved FP32 rate (algorithmic flops per launch / average launch time,
    HIP events on the library's stream) for the evaluation kernels that ran, with each
    model's own pair counts."""
    out = {}
    for grp, model, part, name in KERNEL_GROUPS:
        ms, cnt = prof[grp]
        if not cnt or model not in counts:
            continue
        pr, pa, sk = counts[model]
        desc_f, force_f = flops_per_atom(pr / n, pa / n, sk / n, model)
        f = desc_f if part == "desc" else force_f
        avg_ms = ms / cnt
        ach = f * n / (avg_ms * 1e-3) / 1e12
        out[grp] = {"kernel": name, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_VECTOR_TFLOPS,
                    "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VECTOR_TFLOPS, "flops_per_atom": f,
                    "avg_launch_ms": avg_ms, "launches": cnt, "ms_per_step": ms / steps}
    return out


def run_form(form, hp, params, at, steps, warmup, sur=None, judge_fraction=0.75, mts_k=4, traffic=None):
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
    st0 = s.stats()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = s.step(steps, thermo_every=k if k else 100, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    st1 = s.stats()
    n = at.n
    # each model's pair counts at its own cutoffs, from one evaluation after the timed steps
    counts = {}
    s.compute(slot=0, precision=prec, forces=False)
    counts["full"] = s.pair_counts()
    if mts:
        s.compute(slot=1, precision=prec, forces=False)
        counts["surrogate"] = s.pair_counts()
    kr = kernel_rooflines(prof, steps, n, counts)
    dom = max(kr.values(), key=lambda r: r["ms_per_step"])
    roof = {k_: dom[k_] for k_ in ("kernel", "bound", "achieved", "peak", "unit", "frac", "flops_per_atom",
                                   "avg_launch_ms")}
    if dom["kernel"] == "k_force<full>" and not mts:
        roof["traffic"] = traffic
    out = {"atom_steps_per_s": n * steps / elapsed, "s_per_step_per_atom": elapsed / (n * steps),
           "ms_per_step": 1e3 * elapsed / steps, "n_atoms": n, "steps": steps, "warmup": warmup,
           "precision": prec, "roofline": roof, "kernels": kr,
           "kernels_ms_per_step": {kk: v[0] / steps for kk, v in prof.items() if v[1]},
           "pairs_per_atom": {m_: {"radial": c[0] / n, "angular": c[1] / n, "skin_list": c[2] / n}
                              for m_, c in counts.items()},
           "list_builds": st1["list_builds"] - st0["list_builds"],
           "energy_drift_per_atom": float((th[-1, 1] + th[-1, 2] - th[0, 1] - th[0, 2]) / n) if len(th) > 1 else None}
    if not mts:
        desc_f, force_f = flops_per_atom(*(c / n for c in counts["full"]))
        out["flops_per_atom_step"] = desc_f + force_f
        out["sustained_tflops"] = (desc_f + force_f) * out["atom_steps_per_s"] / 1e12
        desc_ms, desc_cnt = prof["desc_net"]
        out["network_mfma"] = network_mfma(hp, n, desc_ms / desc_cnt, prec)
        out["integrator_hbm"] = integrator_hbm(n, prof["integrate"], steps)
    else:
        out["mts_k"] = k
        out.update(extra)
        out["surrogate_force_error_rms_mean"] = float(np.mean(th[:, 5]))
        out["surrogate_force_error_max"] = float(np.max(th[:, 6]))
        out["block_error_rms"] = [round(float(e), 6) for e in th[:, 5]]
        out["block_fallback"] = [int(e) for e in th[:, 7]]
        out["mts_blocks_timed"] = st1["mts_blocks"] - st0["mts_blocks"]
        out["fallback_blocks_timed"] = st1["fallback_blocks"] - st0["fallback_blocks"]
        out["mts_blocks"] = st1["mts_blocks"]
        out["fallback_blocks"] = st1["fallback_blocks"]
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def train_shorter_surrogate(hp, params, epochs, n_traj=200):
    """The 4/3 A surrogate (coefficients and network) trained on the GPU from full-model
    frames: n_traj trajectories of 100 steps on 10^3-cell boxes at 300..1200 K, a frame
    every 10 steps; Adam with a cosine step size from 1e-2 to 1e-4, batch 8 frames."""
    import torch
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import surrogate as SG
    shp = I.SURROGATE_SHORTER_HPARAMS
    sur0 = I.surrogate_from_teacher(hp, params, shp, 1)
    t = time.perf_counter()
    fr = SG.generate_frames(hp, params, n_traj=n_traj, cells=10, steps=100, every=10)
    t_frames = time.perf_counter() - t

    def log(msg):
        if msg.startswith("epoch") and int(msg.split()[1].rstrip(":")) % 10 == 9:
            print(f"  surrogate {msg}", file=sys.stderr, flush=True)
    r = SG.train_surrogate(fr, shp, sur0, epochs=epochs, batch=8, lr=1e-2, lr_end=1e-4, train_coeffs=True,
                           log=log)
    n_frames = int(fr.x.shape[0])
    del fr
    torch.cuda.empty_cache()
    info = {"surrogate": "rc 4/3 A, n_max 4, basis 8, l_max 2, no four-body, 8 hidden units; coefficients "
                         "and network trained", "frames": n_frames, "frame_generation_s": t_frames,
            "training_s": r.seconds, "epochs": epochs, "val_force_rmse_init": r.val_force_rmse_init,
            "val_force_rmse": r.val_force_rmse, "val_energy_mae_init": r.val_energy_mae_init,
            "val_energy_mae": r.val_energy_mae}
    return shp, sur0, r.params, info


def run_forms(args):
    """Extended comparison on the 32M-atom box: surrogates with three cutoff pairs, network
    only and with trained coefficients, untrained, k = 4 and 8 (five trainings)."""
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
        # the _k8 form: the full model every 8 steps instead of 4 (same judge)
        forms[name] = run_form("mts_bf16" if name.endswith("_bf16") else "mts", hp, params, at, args.steps, wm,
                               sur=sur, mts_k=8 if name.endswith("_k8") else 4)
        print(f"form {name}: {forms[name]['atom_steps_per_s']:.3e} atom-steps/s, "
              f"{forms[name]['mts_blocks']} MTS / {forms[name]['fallback_blocks']} fallback blocks",
              file=sys.stderr, flush=True)
    out = {"metric": METRIC,
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
    the build positions and writes v, x and the 16-byte box-fraction position (88 + 64 B
    per atom); k_kick reads type, F, v and writes v (40 + 24 B)."""
    total_ms, launches = integrate
    per_step_s = total_ms * 1e-3 / steps
    nbytes = 216.0 * n
    achieved = nbytes / per_step_s / 1e9
    return {"kernels": "k_kick_drift + k_kick", "bytes_per_atom_step": 216, "achieved": achieved,
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


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cells", type=int, default=200, help="FCC cells per side (200: 32M atoms)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16 forms")
    ap.add_argument("--no-mts", action="store_true",
                    help="skip the MTS forms (they train a surrogate first, about a minute)")
    ap.add_argument("--forms", action="store_true",
                    help="extended comparison: five surrogates (three cutoff pairs, with and without "
                         "trained coefficients), k = 4 and 8")
    ap.add_argument("--epochs", type=int, default=40, help="surrogate training epochs")
    ap.add_argument("--nvt", type=float, default=0.0,
                    help="fp32 form only, NVT at this temperature (K) with a Nose-Hoover chain of 3, tau 100 fs")
    ap.add_argument("--zbl", type=float, default=0.0,
                    help="fp32 form only, with the ZBL repulsion of this outer radius in A (the paper's Cu "
                         "model uses 2.0)")
    ap.add_argument("--deterministic", action="store_true",
                    help="fp32 form only, with fixed-order force accumulation (no atomics)")
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
        run_forms(args)
        return

    import torch
    from paper_2604_24816_amd import inputs as I

    hp = I.FULL_HPARAMS
    if args.zbl > 0:
        hp = dataclasses.replace(hp, zbl_outer=args.zbl)
    params = I.random_model(hp, 0)
    at = I.workload_4m(args.cells) if args.cells == 100 else I.workload_32m(args.cells)
    n = at.n
    variant = ((f"nvt_{args.nvt:g}K" if args.nvt > 0 else "nve") + (f"_zbl_{args.zbl:g}A" if args.zbl > 0 else "")
               + ("_deterministic" if args.deterministic else ""))
    say(f"bench: {n} atoms ({args.cells}^3 FCC cells), {args.steps} timed + {args.warmup} warm-up steps")
    forms = {}
    if args.nvt > 0 or args.deterministic:
        from paper_2604_24816_amd import nep
        # NVT (a Nose-Hoover chain) or deterministic accumulation: the fp32 form alone,
        # timed like the others
        s = nep.NEPSystem(nep.NEPModel(hp, params), n, at.box)
        s.set_state(at.x, at.types, at.masses, at.v)
        s.build_neighbors(1.0)
        if args.nvt > 0:
            s.set_thermostat(args.nvt, tau=100.0, chain=3)
        if args.deterministic:
            s.set_deterministic(True)
        s.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"metric": METRIC, "value": n * args.steps / el, "unit": "atom-steps/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
                          "data": "synthetic (seeded FCC box, random-weight NEP)",
                          "config": {"workload": f"fcc_cu_{args.cells}x{args.cells}x{args.cells}_cells_{n}"
                                                 f"_atoms_{variant}", "n_atoms": n}}))
        return
    traffic = force_traffic(args.cells) if args.zbl <= 0 else None
    forms["fp32"] = run_form("fp32", hp, params, at, args.steps, args.warmup, traffic=traffic)
    say(f"form fp32: {forms['fp32']['atom_steps_per_s']:.3e} atom-steps/s, {forms['fp32']['ms_per_step']:.2f} ms/step")
    if not args.no_bf16:
        forms["bf16"] = run_form("bf16", hp, params, at, args.steps, args.warmup)
        say(f"form bf16: {forms['bf16']['atom_steps_per_s']:.3e} atom-steps/s")
    training = None
    if not args.no_mts and args.zbl <= 0 and args.steps >= 4:
        shp, sur0, sur_t, training = train_shorter_surrogate(hp, params, args.epochs)
        say(f"surrogate trained: held-out force RMSE {training['val_force_rmse_init']:.4f} -> "
            f"{training['val_force_rmse']:.4f} eV/A")
        for name, form, p in (("mts", "mts", sur_t), ("mts_bf16", "mts_bf16", sur_t),
                              ("mts_untrained", "mts", sur0)):
            forms[name] = run_form(form, hp, params, at, args.steps, args.warmup, sur=(shp, p))
            forms[name]["vs_fp32"] = forms[name]["atom_steps_per_s"] / forms["fp32"]["atom_steps_per_s"]
            say(f"form {name}: {forms[name]['atom_steps_per_s']:.3e} atom-steps/s, "
                f"{forms[name]['mts_blocks']} MTS / {forms[name]['fallback_blocks']} fallback blocks")
    f32 = forms["fp32"]
    out = {
        "metric": METRIC,
        "value": f32["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "s_per_step_per_atom": f32["s_per_step_per_atom"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (seeded FCC box, random-weight NEP)",
        "config": {"workload": f"fcc_cu_{args.cells}x{args.cells}x{args.cells}_cells_{n}_atoms_{variant}",
                   "n_atoms": n, "model": "NEP rc 6/5 A, n_max 4, basis 8, l_max 4 + 4-body, 30 hidden"
                   + (f", ZBL outer {args.zbl} A" if args.zbl > 0 else ""),
                   "value_form": "fp32", "dt_fs": 1.0, "rebuild_every": 10, "skin_A": 1.0,
                   "parallelism": "single GPU"},
        "roofline": f32["roofline"],
        "forms": forms,
        "paper_context": {"note": "Table 5, CNIS GPGPU, trained Cu model, 4,499,456 atoms, FP32",
                          "atom_steps_per_s": 46.19e6},
    }
    if training is not None:
        out["surrogate_training"] = training
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(hp, params, at, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
