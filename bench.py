#!/usr/bin/env python
"""Benchmark: induced-dipole solves per second to 1e-5 D rms on one MI355X.

Headline workload (the largest single-GPU configuration): 288,000 rigid waters (864,000 atoms)
in a 205.0 A box, 7 A real-space cutoff with a 2 A list buffer, Ewald beta 0.545 1/A, PME grid
216^3 of order 5 (synthetic, seeded).  One step processes one configuration end to end on the
GPU with inputs resident in HBM: block-list build, permanent field E_perm, the learned initial
guess (features and network of its delta kind: the previous configuration's converged dipoles
corrected by the network's response to the change of the permanent field) and the
mixed-precision PCG solve of (alpha^-1 - T) mu = E_perm from that guess to the stopping
tolerance, E_pol included.  The configurations are held-out frames of a 0.02 A-step trajectory
of the box; the network was trained beforehand on the GPU (its own kernels) on the solver's
converged dipoles of the preceding frames.  `value` is steps (= solves) per second over the
timed steps; the per-step median, p10 and p90 are reported too.  Beside it, on the same frames:
mixed precision from the previous step's dipoles (the method without the network), from the
zero guess, and the plain FP64 PCG from the zero guess (the baseline the speed-ups refer to).

Accuracy: the converged dipoles of every variant on the 864,000-atom box are compared with the
FP64 GPU solve, and on a periodic ~4,000-atom subcell of the same box with the FP64 oracle's
exact solution (rms and max |mu - mu*|, E_pol error).  Secondary legs: the 648-, 23,558- and
96,000-atom workloads (FP64 and mixed), and the 288,000-atom trajectory (train on 150 frames,
evaluate 50 from the zero, previous-step, learned and judged starts, with both network kinds).

The roofline entry is the dominant kernel of the headline leg, timed with HIP events on the
stream it runs on; the CPU baseline times the FP64 oracle on this host (one full matrix-vector
product and one permanent field of the headline box, scaled by the iteration count).
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "induced-dipole solves/s to 1e-5 D rms (FP64 vs mixed vs learned guess)"
# Stopping tolerance of every timed solve (rms of the preconditioned residual alpha r, Debye),
# the same for the FP64, mixed and learned-start variants.  The GPU tests check at exactly this
# tolerance that the converged dipoles lie within 1e-5 D rms of the oracle's exact solution.
TOL_DEBYE = 1e-5
DEBYE = 4.80320
PEAK_FP32_VALU = 157.3     # TFLOP/s, MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_NONPACKED = 78.6 # TFLOP/s: 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz (packed FP32 is disabled)
PEAK_HBM = 8000.0          # GB/s
# Algorithmic FLOPs per in-cutoff pair of the real-space dipole kernel: FMA counted as 2, each
# of the four hardware transcendentals (rsq, rcp, exp2, exp2) as 1; fixed-point conversion,
# loop control and masked slots not counted.
FLOPS_PER_PAIR = 80
STAGES = ["list", "perm", "real", "spread", "fft", "gather", "pcg", "guess"]
DTYPE = ("f32 pair/PME math; tile and grid-row sums as 64-bit integer fixed point (2^-38 e/A^2) in LDS, "
         "per-atom fields as integer-valued f64 fixed point (2^-40 e/A^2); f64 PCG vectors, dot products "
         "and convergence test; f32 network")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=TOL_DEBYE)
    ap.add_argument("--workload", default="water_864000", choices=["water_864000", "water_96000"],
                    help="headline workload (the other sizes run as secondary legs)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing leg")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 648/23,558/96,000-atom legs")
    ap.add_argument("--no-trajectory", action="store_true", help="skip the 288,000-atom trajectory leg")
    ap.add_argument("--no-subcell", action="store_true", help="skip the oracle accuracy check on the subcell")
    ap.add_argument("--pair-store", default="auto", choices=["auto", "compute", "stored"],
                    help="how the real-space dipole products get their pair coefficients")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain 256 MiB device-to-device copies (the reference dispatch that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters of a profiling run)")
    return ap.parse_args()


def pstats(times_ms):
    """median, p10, p90 and mean of per-step times (ms), linear interpolation between ranks."""
    v = sorted(times_ms)

    def q(p):
        x = p * (len(v) - 1)
        lo = int(math.floor(x))
        hi = min(lo + 1, len(v) - 1)
        return v[lo] + (v[hi] - v[lo]) * (x - lo)
    return {"median_ms": q(0.5), "p10_ms": q(0.1), "p90_ms": q(0.9), "mean_ms": statistics.fmean(v)}


def tensors(s, dev="cuda:0"):
    import torch
    t = {k: torch.tensor(getattr(s, k), device=dev) for k in ("pos", "q", "dip", "quad", "alpha", "thole", "sc_s")}
    t["sc_ptr"] = torch.tensor(s.sc_ptr, dtype=torch.int32, device=dev)
    t["sc_j"] = torch.tensor(s.sc_j, dtype=torch.int32, device=dev)
    return t


def new_context(s, t, precision, pair_store="auto"):
    from paper_2011_01207_amd import amoeba
    ctx = amoeba.Context(s.n, s.box, cutoff=s.cutoff, buffer=s.buffer, ewald_alpha=s.ewald_alpha, grid=s.grid,
                         order=s.order, precision=precision)
    ctx.set_pair_store(pair_store)
    ctx.set_atoms(t["alpha"], t["thole"], t["sc_ptr"], t["sc_j"], t["sc_s"])
    return ctx


def run_steps(ctx, t, frames, steps, warmup, tol, guess="zero", prev=None, timing_live=False, stage_pass=False,
              rebuild_each_step=False):
    """`steps` steps cycling over `frames` (device position tensors): list + E_perm + solve from
    `guess` ('zero'; 'given' with prev[k] = (dipoles, field) of the frame before frame k;
    'learned' with the network of the context's kind, whose delta kind takes prev[k] as its
    reference; 'best' judges the learned guess against the given one).  The list is kept while
    every atom stays within buffer/2 of its position at the last build (the masks are refreshed
    for each frame) and rebuilt otherwise, or rebuilt at every step with rebuild_each_step.
    Returns per-step times, iterations, list rebuilds, the last frame's outputs and the timers."""
    import torch
    from paper_2011_01207_amd import amoeba
    e_perm = torch.empty_like(frames[0])
    mu = torch.empty_like(frames[0])
    delta = guess in ("learned", "best") and ctx.guess_kind == "delta"
    rebuilds = [0]

    def step(k):
        # amoeba_polarize_configuration: list kept (or rebuilt), E_perm, the solve
        pos = frames[k % len(frames)]
        if rebuild_each_step:
            ctx.build_blocklist(pos)
            rebuilds[0] += 1
        g = prev[k % len(frames)][0] if guess in ("given", "best") else None
        if delta:
            ctx.guess_set_reference(*prev[k % len(frames)])
        _, _, ep, it, st, rebuilt = ctx.polarize_configuration(pos, t["q"], t["dip"], t["quad"], mu_guess=g,
                                                                guess_mode=guess, tol_debye=tol, max_iter=1000,
                                                                out=mu, e_perm_out=e_perm)
        rebuilds[0] += int(rebuilt)
        if st != amoeba.AMOEBA_OK:
            raise RuntimeError(f"{guess} solve did not converge (status {st})")
        return ep, it

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    if timing_live:
        ctx.set_timing("live")
    times, its, picks, eps = [], [], [], []
    rebuilds[0] = 0
    t_all = time.perf_counter()
    for k in range(steps):
        t0 = time.perf_counter()
        ep, it = step(k)
        times.append(1e3 * (time.perf_counter() - t0))
        its.append(it)
        eps.append(ep)
        picks.append(ctx.info()["last_guess"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    out = {"step_ms": 1e3 * total / steps, "solves_per_s": steps / total, **pstats(times),
           "list_rebuilds": rebuilds[0],
           "iterations": its[-1], "mean_iterations": statistics.fmean(its), "e_pol_kcal": eps[-1],
           "learned_picked": sum(1 for p in picks if p == amoeba.AMOEBA_GUESS_LEARNED),
           # real-space products per pass of `steps` steps besides the PCG products: the
           # Neumann-kind guess's two basis products per step (the delta kind needs none)
           "extra_real_products": 2 * steps if guess in ("learned", "best") and not delta else 0}
    out["timing_live"] = ctx.timing() if timing_live else None
    ctx.set_timing("off")
    if stage_pass:
        # the same steps again with every launch bracketed by HIP events on the library's stream
        # (each stage alone): the per-stage kernel times; not part of `value`
        ctx.set_timing("stages")
        for k in range(steps):
            step(k)
        out["timing"] = ctx.timing()
        ctx.set_timing("off")
        out["kernel_ms_per_step"] = {k: v / steps for k, v in out["timing"]["ms"].items()}
        out["matvecs_per_step"] = out["timing"]["matvecs"] / steps
    inf = ctx.info()
    out.update({k: inf[k] for k in ("n_pairs", "n_tiles", "n_blocks", "pme_planes", "pair_min_image", "pair_store",
                                    "pair_store_bytes")})
    # outputs of the last timed frame (for the accuracy comparisons)
    ep, _ = step(steps - 1)
    out["e_pol_kcal"] = ep
    out["mu"] = mu.clone()
    return out


def reference_solves(ctx, t, frames, tol_ref=1e-6):
    """The solver's own converged dipoles (to tol_ref) and permanent field of every frame."""
    from paper_2011_01207_amd import amoeba
    out = []
    for pos in frames:
        ctx.build_blocklist(pos)
        e = ctx.perm_field(pos, t["q"], t["dip"], t["quad"])
        mu, _, _, st = ctx.polarize(pos, e, tol_debye=tol_ref, max_iter=1000)
        if st != amoeba.AMOEBA_OK:
            raise RuntimeError("reference solve did not converge")
        out.append({"pos": pos, "e": e, "mu": mu.clone()})
    return out


def with_features(ctx, sol, first, last):
    """Training data of frames first..last-1: the network's features and bases of each frame
    (GPU kernels; the delta kind takes the frame before as its reference) and its converged
    dipoles as the target."""
    data = []
    for k in range(first, last):
        d = sol[k]
        ctx.build_blocklist(d["pos"])
        if ctx.guess_kind == "delta":
            ctx.guess_set_reference(sol[k - 1]["mu"], sol[k - 1]["e"])
        feat, basis = ctx.guess_features(d["pos"], d["e"])
        data.append({**d, "feat": feat, "basis": basis})
    return data


def train(ctx, data, train_steps, batch, lr=2e-3, seed=5):
    """Fit the network on the GPU: feature statistics, then Adam steps on random batches."""
    import numpy as np
    import torch
    from paper_2011_01207_amd import synth
    feat = torch.cat([d["feat"] for d in data])
    basis = torch.cat([d["basis"] for d in data])
    target = torch.cat([d["mu"] for d in data]).float()
    ctx.guess_set_model(synth.guess_init_model(seed=7))
    ctx.guess_fit_norm(feat)
    rng = np.random.default_rng(seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for k in range(train_steps):
        idx = torch.tensor(rng.integers(0, feat.shape[0], batch).astype(np.int32), device=feat.device)
        losses.append(ctx.guess_train_step(feat, basis, target, lr, idx=idx))
    torch.cuda.synchronize()
    return {"train_samples": int(feat.shape[0]), "train_steps": train_steps, "batch": batch,
            "loss_first_d2": float(np.mean(losses[:20])), "loss_last_d2": float(np.mean(losses[-20:])),
            "train_s": time.perf_counter() - t0}


def amoeba_ok():
    from paper_2011_01207_amd import amoeba
    return amoeba.AMOEBA_OK


def mu_errors(a, b):
    """rms and max over atoms of |a_i - b_i| in Debye (device or host arrays)."""
    import numpy as np
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = b.cpu().numpy() if hasattr(b, "cpu") else np.asarray(b)
    d = np.linalg.norm(a.reshape(-1, 3) - b.reshape(-1, 3), axis=1)
    return {"mu_rms_debye": float(DEBYE * np.sqrt(np.mean(d * d))), "mu_max_debye": float(DEBYE * np.max(d))}


def strip(res):
    return {k: v for k, v in res.items() if k not in ("mu", "timing")}


def guess_errors(ctx, data):
    """Mean rms error (Debye) of the network's guess and of the previous-step guess against the
    converged dipoles of held-out frames."""
    err_l = statistics.fmean(
        mu_errors(ctx.guess_forward(d["feat"], d["basis"]).double(), d["mu"])["mu_rms_debye"] for d in data)
    return err_l


def headline(s, t, a):
    """The headline box: the delta-kind network trained on the GPU, then mixed + learned,
    mixed + previous step, mixed (zero) and FP64 (zero) on the same held-out frames."""
    import torch
    from paper_2011_01207_amd import synth
    n_train, n_eval = 8, 4
    frames = [torch.tensor(p, device="cuda:0") for p in synth.trajectory(s, n_train + n_eval + 1, 0.02, seed=504)]
    eval_frames = frames[n_train + 1:]
    log(f"{s.name}: training the learned guess on {n_train} frames")
    ctx = new_context(s, t, "mixed", a.pair_store)
    ctx.guess_set_kind("delta")
    t0 = time.perf_counter()
    sol = reference_solves(ctx, t, frames)
    t_ref = time.perf_counter() - t0
    data = with_features(ctx, sol, 1, n_train + 1)
    tr = train(ctx, data, train_steps=600, batch=65536)
    del data
    tr.update({"kind": "delta", "reference_solves_s": t_ref, "train_configs": n_train, "eval_configs": n_eval})
    held = with_features(ctx, sol, n_train + 1, n_train + n_eval + 1)
    tr["guess_rms_err_debye"] = guess_errors(ctx, held)
    tr["prev_rms_err_debye"] = statistics.fmean(
        mu_errors(sol[k - 1]["mu"], sol[k]["mu"])["mu_rms_debye"] for k in range(n_train + 1, n_train + n_eval + 1))
    del held
    model = ctx.guess_save()
    prev = [(sol[k - 1]["mu"], sol[k - 1]["e"]) for k in range(n_train + 1, n_train + n_eval + 1)]
    log(f"{s.name}: mixed + learned guess")
    learned = run_steps(ctx, t, eval_frames, a.steps, a.warmup, a.tol, guess="learned", prev=prev,
                        timing_live=True, stage_pass=True)
    log(f"{s.name}: mixed + learned {learned['step_ms']:.3f} ms/step (median {learned['median_ms']:.3f}), "
        f"{learned['mean_iterations']:.1f} it")
    given = run_steps(ctx, t, eval_frames, a.steps, a.warmup, a.tol, guess="given", prev=prev)
    log(f"{s.name}: mixed + previous step {given['step_ms']:.3f} ms/step, {given['mean_iterations']:.1f} it")
    rebuilt = run_steps(ctx, t, eval_frames, a.steps, a.warmup, a.tol, guess="learned", prev=prev,
                        rebuild_each_step=True)
    learned["rebuild_each_step"] = {k: rebuilt[k] for k in ("step_ms", "solves_per_s", "median_ms", "p10_ms",
                                                             "p90_ms", "mean_iterations", "list_rebuilds")}
    log(f"{s.name}: mixed + learned, list rebuilt every step {rebuilt['step_ms']:.3f} ms/step")
    del rebuilt
    ctx.close()
    ctx = new_context(s, t, "mixed", a.pair_store)
    mixed = run_steps(ctx, t, eval_frames, a.steps, a.warmup, a.tol, guess="zero", stage_pass=True)
    ctx.close()
    log(f"{s.name}: mixed {mixed['step_ms']:.3f} ms/step, {mixed['mean_iterations']:.1f} it")
    ctx = new_context(s, t, "fp64", a.pair_store)
    fp64 = run_steps(ctx, t, eval_frames, a.steps, a.warmup, a.tol, guess="zero")
    # the last timed frame solved in FP64 far below the tolerance: the exact dipoles of this
    # discretization to about 1e-9 D, against which every leg's converged dipoles are measured
    pos_last = eval_frames[(a.steps - 1) % len(eval_frames)]
    ctx.update_blocklist(pos_last)
    e_last = ctx.perm_field(pos_last, t["q"], t["dip"], t["quad"])
    mu_tight, ep_tight, it_tight, st_tight = ctx.polarize(pos_last, e_last, tol_debye=1e-9, max_iter=1000)
    if st_tight != amoeba_ok():
        raise RuntimeError("tightly converged reference solve did not converge")
    ctx.close()
    log(f"{s.name}: fp64 {fp64['step_ms']:.3f} ms/step, {fp64['mean_iterations']:.1f} it")
    del sol, prev
    acc = {"reference": "FP64 GPU solve of the same frame (zero start, the same tolerance)"}
    tight = {"reference": f"FP64 GPU solve of the same frame to 1e-9 D ({it_tight} iterations)"}
    for name, r in (("mixed_learned", learned), ("mixed_previous_step", given), ("mixed", mixed), ("fp64", fp64)):
        tight[name] = mu_errors(r["mu"], mu_tight)
        tight[name]["e_pol_rel"] = abs(r["e_pol_kcal"] - ep_tight) / abs(ep_tight)
    del mu_tight, e_last
    for name, r in (("mixed_learned", learned), ("mixed_previous_step", given), ("mixed", mixed)):
        acc[name] = mu_errors(r["mu"], fp64["mu"])
        acc[name]["e_pol_abs_kcal"] = abs(r["e_pol_kcal"] - fp64["e_pol_kcal"])
        acc[name]["e_pol_rel"] = acc[name]["e_pol_abs_kcal"] / abs(fp64["e_pol_kcal"])
    acc["vs_tightly_converged"] = tight
    return learned, given, mixed, fp64, acc, tr, model


def subcell_accuracy(parent, model, tol):
    """Every variant against the FP64 oracle's exact solution on the periodic subcell of the
    headline box (full oracle solve: smooth PME on the same grid spacing, PCG to 1e-9 D).  The
    subcell takes one 0.02 A trajectory step; the learned start (the headline's delta network)
    uses the GPU's converged solution of the configuration before the step as its reference."""
    import dataclasses
    import torch
    import oracle as O
    from paper_2011_01207_amd import synth
    s0 = synth.subcell(parent)
    p0, p1 = list(synth.trajectory(s0, 2, 0.02, seed=604))
    s = dataclasses.replace(s0, pos=p1)
    e_ref = O.perm_field(s, "spme")
    mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-9)
    ep_ref = O.e_pol(mu_ref, e_ref)
    t = tensors(s)
    pos0 = torch.tensor(p0, device="cuda:0")
    out = {"workload": f"{s.name}: periodic {s.box[0]:.2f} A cube of the headline box, PME {s.grid[0]}^3, one "
                       "0.02 A step after the reference configuration",
           "n_atoms": s.n, "e_pol_oracle_kcal": ep_ref}
    for name, prec, guess in (("fp64", "fp64", "zero"), ("mixed", "mixed", "zero"),
                              ("mixed_learned", "mixed", "learned")):
        ctx = new_context(s, t, prec)
        if guess == "learned":
            ctx.guess_load(model)
            ctx.build_blocklist(pos0)
            e0 = ctx.perm_field(pos0, t["q"], t["dip"], t["quad"])
            mu0, _, _, _ = ctx.polarize(pos0, e0, tol_debye=1e-6, max_iter=1000)
            ctx.guess_set_reference(mu0, e0)
        ctx.build_blocklist(t["pos"])
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        mu, ep, it, st = ctx.polarize(t["pos"], e, guess_mode=guess, tol_debye=tol, max_iter=1000)
        ctx.close()
        r = mu_errors(mu, mu_ref)
        r.update({"iterations": it, "e_pol_kcal": ep, "e_pol_abs_kcal": abs(ep - ep_ref),
                  "e_pol_rel": abs(ep - ep_ref) / abs(ep_ref)})
        out[name] = r
    return out


def secondary(a):
    """FP64 and mixed zero-guess steps of the smaller workloads (one configuration, the list
    rebuilt at every step), with the oracle's exact solution where it is cheap (648 and 23,558
    atoms)."""
    import oracle as O
    from paper_2011_01207_amd import synth
    out = {}
    for s in (synth.water648(), synth.solvated_chain(), synth.water96k()):
        t = tensors(s)
        res = {}
        for prec in ("fp64", "mixed"):
            ctx = new_context(s, t, prec, a.pair_store)
            res[prec] = run_steps(ctx, t, [t["pos"]], a.steps, a.warmup, a.tol, rebuild_each_step=True)
            ctx.close()
        entry = {p: strip(r) for p, r in res.items()}
        entry["speedup_mixed_vs_fp64"] = res["fp64"]["step_ms"] / res["mixed"]["step_ms"]
        if s.n <= 30000:
            e_ref = O.perm_field(s, "spme")
            mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-9)
            ep_ref = O.e_pol(mu_ref, e_ref)
            for p, r in res.items():
                entry[p]["vs_oracle"] = {**mu_errors(r["mu"], mu_ref),
                                         "e_pol_rel": abs(r["e_pol_kcal"] - ep_ref) / abs(ep_ref)}
        else:
            entry["mixed"]["vs_fp64_gpu"] = mu_errors(res["mixed"]["mu"], res["fp64"]["mu"])
        out[s.name] = entry
        log(f"{s.name}: fp64 {res['fp64']['step_ms']:.3f} ms, mixed {res['mixed']['step_ms']:.3f} ms")
        del t
    return out


def trajectory_leg(a, n_train=150, n_eval=50):
    """288,000 atoms, 201 configurations of cumulative 0.02 A steps: the network of each kind
    trained on frames 1..150 (the solver's own converged dipoles; the delta kind with each
    frame's predecessor as its reference), then frames 151..200 solved once each from the zero,
    previous-step, learned and judged starts."""
    import torch
    from paper_2011_01207_amd import synth
    s = synth.water288k()
    t = tensors(s)
    frames = [torch.tensor(p, device="cuda:0") for p in synth.trajectory(s, n_train + n_eval + 1, 0.02, seed=304)]
    ctx = new_context(s, t, "mixed", a.pair_store)
    t0 = time.perf_counter()
    sol = reference_solves(ctx, t, frames)
    out = {"workload": "water_288000: 96,000 waters, 142.3 A box, PME 144^3; 201 configurations of cumulative "
                       "0.02 A per-atom steps; train on 1-150, evaluate 151-200 once per start",
           "reference_solves_s": time.perf_counter() - t0,
           "prev_rms_err_debye": statistics.fmean(
               mu_errors(sol[k - 1]["mu"], sol[k]["mu"])["mu_rms_debye"]
               for k in range(n_train + 1, n_train + n_eval + 1))}
    ev = frames[n_train + 1:]
    prev = [(sol[k - 1]["mu"], sol[k - 1]["e"]) for k in range(n_train + 1, n_train + n_eval + 1)]
    modes = {}
    for mode in ("zero", "given"):
        r = run_steps(ctx, t, ev, n_eval, 2, a.tol, guess=mode, prev=prev, stage_pass=True)
        modes[{"given": "previous_step"}.get(mode, mode)] = strip(r)
        log(f"288k trajectory {mode}: {r['step_ms']:.3f} ms, {r['mean_iterations']:.2f} it")
    for kind in ("neumann", "delta"):
        ctx.guess_set_kind(kind)
        data = with_features(ctx, sol, 1, n_train + 1)
        tr = train(ctx, data, train_steps=2000, batch=65536)
        del data
        held = with_features(ctx, sol, n_train + 1, n_train + n_eval + 1)
        tr["guess_rms_err_debye"] = guess_errors(ctx, held)
        del held
        out[f"training_{kind}"] = tr
        for mode in ("learned", "best"):
            r = run_steps(ctx, t, ev, n_eval, 2, a.tol, guess=mode, prev=prev, stage_pass=True)
            modes[f"{mode}_{kind}"] = strip(r)
            log(f"288k trajectory {mode} ({kind}): {r['step_ms']:.3f} ms, {r['mean_iterations']:.2f} it, "
                f"learned picked {r['learned_picked']}")
    ctx.close()
    del sol, prev
    out["modes"] = modes
    return out


def roofline(s, res):
    """Per-stage achieved rates of a leg's stage pass; the dominant stage is reported, with the
    real-space tiles timed live in the timed region when they dominate."""
    tim = res["timing"]
    n = s.n
    K = s.grid
    mv = tim["matvecs"]
    stages = {}
    # real-space dipole tiles: FP32 VALU bound; the productive launches are the PCG products and
    # the learned guess's basis products (launches queued after convergence return at entry)
    extra = res.get("extra_real_products", 0)
    n_real = mv + extra
    ms = tim["ms"]["real"]
    flops = FLOPS_PER_PAIR * res["n_pairs"] * n_real
    mi = "true" if res.get("pair_min_image") else "false"
    cm = 2 if res.get("pair_store") else 0
    stages["real"] = {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP32_VALU,
                      "unit": "TFLOP/s", "ms_total": ms, "launches": tim["launches"]["real"],
                      "productive_launches": n_real,
                      "kernel": f"k_block_tiles<float, true, DipoleKind<float>, {mi}, {cm}>",
                      "algorithmic_per_launch": FLOPS_PER_PAIR * res["n_pairs"],
                      "peak_nonpacked": PEAK_FP32_NONPACKED,
                      "frac_nonpacked": flops / (ms * 1e-3) / 1e12 / PEAK_FP32_NONPACKED}
    kh = K[2] // 2 + 1
    nc = K[0] * K[1] * kh
    # plane path.  spread stage = k_pme_spread_z: per atom its binned record (16 B), spline
    # arguments (16 B) and FP32 dipole (16 B) read once, the z half spectra (8 B per point) written
    b_spread = n * 48 + nc * 8
    # fft stage = forward y-lines, x-lines with the influence function, inverse y-lines: the half
    # grid read and written by each pass, the influence function read once
    b_fft = 3 * nc * (8 + 8) + nc * 4
    # gather stage = k_pme_z_gather + k_plane_combine: half grid read once, atom records read,
    # five field shares written and read (16 B each); combine: i-field 24 B, direction 24 B,
    # 1/alpha 8 B read and A p 24 B written per atom, every tile j-field slot (16 B) read
    b_gather = nc * 8 + n * (32 + 2 * 80 + 24 + 24 + 8 + 24) + res["n_tiles"] * 64 * 16
    nt = "256" if K[0] >= 200 else "512"   # threads of the row passes (their shapes follow the grid)
    for name, b, kern in (("spread", b_spread, f"k_pme_spread_z<float, true, false, {nt}>"),
                          ("fft", b_fft, "k_pme_ylines<float, -1> + k_pme_xconv<float> + k_pme_ylines<float, 1>"),
                          ("gather", b_gather, f"k_pme_z_gather<float, {nt}> + k_plane_combine<float, 1>")):
        ms = tim["ms"][name]
        stages[name] = {"bound": "hbm", "achieved": b * mv / (ms * 1e-3) / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                        "ms_total": ms, "launches": tim["launches"][name], "kernel": kern,
                        "algorithmic_per_launch": b}
    for v in stages.values():
        v["frac"] = v["achieved"] / v["peak"]
    dom = max(["real", "spread", "gather", "fft"], key=lambda k: stages[k]["ms_total"])
    d = stages[dom]
    from paper_2011_01207_amd import profiling
    traffic = profiling.traffic_lookup(os.path.join(ROOT, "profiles", f"hbm_traffic_{s.name}_mixed.md"), d["kernel"])
    avg_us = 1e3 * d["ms_total"] / max(1, d["launches"])
    top = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
           "frac": d["frac"], "traffic": traffic, "kernel": d["kernel"], "stage": dom,
           "avg_launch_us": avg_us, "launches": d["launches"], "productive_launches": d.get("productive_launches", mv),
           "timed_in": "stage pass (each stage alone on one stream)"}
    live = res.get("timing_live")
    if dom == "real" and live and live["launches"]["real"]:
        # the tiles as they run in the timed region: on the second stream beside the reciprocal
        # passes (HIP events on that stream); the stage-pass figures are kept beside them
        ms_l, n_l = live["ms"]["real"], live["launches"]["real"]
        prod_l = live["matvecs"] + extra
        ach = d["algorithmic_per_launch"] * prod_l / (ms_l * 1e-3) / 1e12
        top.update({"achieved_alone": top["achieved"], "frac_alone": top["frac"], "avg_launch_us_alone": avg_us,
                    "achieved": ach, "frac": ach / d["peak"], "avg_launch_us": 1e3 * ms_l / n_l, "launches": n_l,
                    "productive_launches": prod_l,
                    "timed_in": "timed region (second stream, beside the reciprocal passes)"})
        avg_us = top["avg_launch_us"]
        d = dict(d, frac_nonpacked=ach / d["peak_nonpacked"])
    if traffic is not None:
        top["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        top["traffic_rate_gbs"] = traffic / (avg_us * 1e-6) / 1e9
    for k in ("peak_nonpacked", "frac_nonpacked"):
        if k in d:
            top[k] = d[k]
    top["algorithmic_unit"] = (f"{FLOPS_PER_PAIR} FLOP per in-cutoff pair x {res['n_pairs']} pairs per launch"
                               if dom == "real" else "bytes per launch")
    return top, stages


def cpu_baseline(s, iters):
    """FP64 oracle on this host: one full matrix-vector product (real space over the cell grid +
    smooth-PME reciprocal field + self) and one permanent field of the headline box; a solve =
    iterations x matvec + permanent field."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(0)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    n_thr = O.num_threads()
    t0 = time.perf_counter()
    O.matvec(s, mu, "spme")
    t_mv = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.perm_field(s, "spme")
    t_perm = time.perf_counter() - t0
    t_step = iters * t_mv + t_perm
    return {"value": 1.0 / t_step, "unit": "solves/s", "cores": n_thr, "kind": "oracle",
            "sample": (f"{s.name}: one full oracle matrix-vector product ({t_mv:.2f} s: real space over a cell "
                       f"grid, smooth-PME field, self) and one permanent field ({t_perm:.2f} s), timed; solve = "
                       f"{iters} PCG iterations x matvec + E_perm"),
            "seconds_per_solve": t_step}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 (multi-GPU sharding is "
                                   "a design note, not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2011_01207_amd import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    s = synth.water864k() if a.workload == "water_864000" else synth.water96k()
    log(f"workload {s.name}: N={s.n} box={s.box[0]} grid={s.grid} rc={s.cutoff}+{s.buffer}")
    t = tensors(s)
    learned, given, mixed, fp64, acc, tr, model = headline(s, t, a)
    top, stages = roofline(s, learned)
    res = {
        "metric": METRIC,
        "value": learned["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": learned["step_ms"],
        "median_ms": learned["median_ms"], "p10_ms": learned["p10_ms"], "p90_ms": learned["p90_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": (f"{s.name}: {s.n // 3:,} rigid waters ({s.n:,} atoms), {s.box[0]:.2f} A cubic box, "
                                f"rc 7 A + 2 A list buffer, beta 0.545/A, PME {s.grid[0]}^3 order 5; one step = "
                                "block list (kept while every atom stays within buffer/2 of its position at the last "
                                "build, tested on the device at every step; the in-cutoff masks refreshed for the "
                                "frame) + E_perm + learned initial guess + mixed-precision PCG to the tolerance, "
                                "as one amoeba_polarize_configuration call per step, on held-out frames of a "
                                "0.02 A-step trajectory"),
                   "list_rebuilds_timed": learned["list_rebuilds"],
                   "precision": "mixed", "guess": "learned (delta kind)", "tol_debye": a.tol},
        "roofline": top,
        "roofline_stages": stages,
        "mixed_learned": strip(learned),
        "mixed_previous_step": strip(given),
        "mixed": strip(mixed),
        "fp64": strip(fp64),
        "speedup_vs_fp64": {"mixed_learned": fp64["step_ms"] / learned["step_ms"],
                            "mixed_previous_step": fp64["step_ms"] / given["step_ms"],
                            "mixed": fp64["step_ms"] / mixed["step_ms"]},
        "accuracy_vs_fp64_gpu": acc,
        "learned_guess_training": tr,
    }
    if not a.no_subcell:
        log("subcell accuracy against the oracle")
        res["accuracy_vs_oracle_subcell"] = subcell_accuracy(s, model, a.tol)
    fp64_iters = fp64["iterations"]
    del t, learned, given, mixed, fp64
    torch.cuda.empty_cache()
    if not a.no_secondary:
        log("secondary workloads")
        res["secondary"] = secondary(a)
    if not a.no_trajectory:
        log("288,000-atom trajectory leg")
        res["trajectory_288000"] = trajectory_leg(a)
        torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(s, fp64_iters)
    if a.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
