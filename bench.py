#!/usr/bin/env python3
"""Throughput of the randomized Tucker compression + FFCP hot path on one GPU.

One step is one pass of the whole path over a resident synthetic tensor, in
the precision form: rt_tucker_rand with BF16 streaming passes (statistics,
the scaled BF16 copy of the FP32 tensor, the first sketch sweep and one power
sweep and the core pass on that copy; FP64 sketch QR; truncation to the
Tucker ranks) followed by rt_ffcp (CP-ALS through the compressed core, started
from the learned initializer's factors, guarded by the HOSVD start, run to
the stated fit-change tolerance).  The plain FP32 path (the same two sweeps,
HOSVD start) is timed beside it on the same tensor, and one FP32 sweep for
context.  The initializer is trained before the timed region on cores the
pipeline makes from seeded 300^3 CP tensors.

Workload (synthetic, seeded): 1000 x 1000 x 1000 FP32 CP tensor of rank 20
with per-mode column congruence drawn from U[0.5, 0.95], Gaussian noise at
SNR 30 dB; Omega_n 1000 x 30, Omega~_n 900 x 30; Tucker ranks (20, 20, 20);
FFCP with R = 20, ALS, stop when the fit changes by less than 1e-7.

Printed: one JSON line.  ``value`` is the algorithmic HBM rate of the Tucker
stage of the step (bytes of Y the method must stream per call / its time);
``roofline`` prices the dominant kernel against the chip's peak from HIP
events recorded live on the library's stream; ``cpu_baseline`` is the FP64
NumPy oracle on the same tensor (same unit; --cpu-slab bounds it to a
mode-3 slab).
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Tucker sketch+project HBM GB/s (% peak); FFCP time-to-fit, "
          "mixed vs plain FP32")
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=1000,
                    help="I for the I x I x I tensor")
    ap.add_argument("--precision", choices=("bf16", "f32"), default="bf16",
                    help="form timed as the step (bf16: precision form, two sweeps)")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--max-it", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (profiling runs)")
    ap.add_argument("--cpu-slab", type=int, default=1000,
                    help="mode-3 slab of the tensor the oracle runs on")
    ap.add_argument("--train-cores", type=int, default=2048,
                    help="pipeline cores the learned initializer trains on "
                         "(0: precision form starts from HOSVD)")
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--no-hals", action="store_true",
                    help="skip the 10^4-per-mode FFCP-HALS side measurement")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the Algorithm 2 side measurement")
    ap.add_argument("--tucker-only", action="store_true",
                    help="time only the Tucker stage of the chosen form (short "
                         "runs under a profiler) and print its stage times")
    ap.add_argument("--ffcp-only", action="store_true",
                    help="the 1000^3 workload's Tucker stage once, then only the "
                         "timed FFCP-ALS calls from the HOSVD start (for the profiler)")
    ap.add_argument("--hals-only", action="store_true",
                    help="run only the FFCP-HALS fits on the 10^4-per-mode workload (short "
                         "runs under a profiler) and print their record")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="K",
                    help="also run K plain device copies of Y (HBM counter "
                         "calibration under a profiler)")
    return ap.parse_args()


# source file of each kernel whose HBM traffic is stored in profiles/
KERNEL_SOURCE = {"dual_f32_kernel": "stream.hip",
                 "bf16_convert_kernel": "stream_bf16.hip",
                 "bf16_stream_kernel": "stream_bf16.hip",
                 "bf16_cs_kernel": "stream_bf16.hip"}


def source_digest(kernel):
    """Digest of the kernel's source file; stored traffic counters are only
    valid for the kernel they were taken on."""
    p = os.path.join(ROOT, "paper_1412_1885_amd", "csrc", KERNEL_SOURCE[kernel])
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(kernel, workload):
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        tab = json.load(f)
    e = tab.get(kernel, {}).get(workload)
    if not e or e.get("source_digest") != source_digest(kernel):
        return None
    return float(e["bytes_per_launch"])


def cpu_baseline(Y, omegas, omega_tildes, ranks, slab, sweeps, bytes_per_elem, reps=3):
    """The FP64 oracle (untuned) on Y[:, :, :slab] with Omega_3 rows
    0..slab-1, with the step's number of sweeps; rate in the metric's unit
    (the step's algorithmic bytes per element x elements / wall time), the
    median of ``reps`` runs with the BLAS threads pinned to the process's
    CPU affinity set.  Also returns the oracle's last result."""
    from oracle import randtucker as RT
    cores = len(os.sched_getaffinity(0))
    limiter = None
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=cores, user_api="blas")
    except Exception:  # threadpoolctl missing: BLAS keeps its own count
        pass
    try:
        Ys = Y[:, :, :slab].cpu().numpy().astype(np.float64)
        om = [o.astype(np.float64) for o in omegas]
        om[2] = om[2][:slab]
        omt = [[o.astype(np.float64) for o in lst] for lst in omega_tildes[:sweeps]]
        times, res = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = RT.rand_tucker(Ys, om, omt, sweeps=sweeps, ranks=ranks)
            times.append(time.perf_counter() - t0)
    finally:
        if limiter is not None:
            limiter.unregister()
    dt = float(np.median(times))
    nbytes = bytes_per_elem * Ys.size
    where = ("the whole tensor" if slab >= Y.shape[2] else
             f"the {Ys.shape[0]}x{Ys.shape[1]}x{slab} mode-3 slab of the tensor")
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"RandTucker2i S={sweeps} (sketches, QR, core, truncation) "
                       f"in FP64 NumPy on {where}; median of {reps} runs "
                       f"({', '.join(f'{t:.2f}' for t in times)} s), BLAS threads "
                       f"pinned to the {cores} CPUs of the affinity set")}, res, Ys


def run_form(P, torch, Y, om_d, omt_d, ranks, R, precision, sweeps, steps,
             warmup, tol, max_it, ybf16, net=None, A_random=None, order="jacobi"):
    """Time `steps` calls of tucker_rand [+ MLP start] + ffcp in one form;
    returns timings, the last outputs and the per-stage event totals.
    Start: the network's (guarded by HOSVD) when net is given, the given
    random factors when A_random is, else HOSVD."""
    stream = torch.cuda.current_stream()

    def step(tws, fws, ev):
        ev[0].record(stream)
        out = P.tucker_rand(Y, om_d, omt_d[:sweeps], ranks=ranks, sweeps=sweeps,
                            precision=precision, workspace=tws, ybf16=ybf16,
                            sync=False, order=order)
        ev[1].record(stream)
        if net is not None:     # learned start, kept only if it beats HOSVD's
            V = net.forward(out["G"].reshape((1,) + tuple(ranks)))
            init = dict(init="coeff_guarded", A_init=[v[0] for v in net.split(V)])
        elif A_random is not None:
            init = dict(init="user", A_init=A_random)
        else:
            init = dict(init="hosvd")
        ev[2].record(stream)
        f = P.ffcp(out["U"], out["G"], R, update="als", max_it=max_it, tol=tol,
                   workspace=fws, sync=False, **init)
        ev[3].record(stream)
        return out, f

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tws = fws = None
    for _ in range(max(warmup, 1)):      # the first call sizes the workspaces
        out, f = step(tws, fws, mk())
        tws, fws = out["workspace"], f["workspace"]
    torch.cuda.synchronize()
    P.profile_enable(True)
    evs = [mk() for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out, f = step(tws, fws, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = P.profile_read()
    P.profile_enable(False)
    finfo = np.frombuffer(f["info_dev"].cpu().numpy().tobytes(), P.FFCP_INFO_DTYPE)[0]
    tinfo = np.frombuffer(out["info_dev"].cpu().numpy().tobytes(),
                          P.TUCKER_INFO_DTYPE)[0]
    fit_y = P.cp_fit_dense(Y, f["A"], f["lam"])[0]
    return {
        "tucker_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
        "init_ms": float(np.mean([e[1].elapsed_time(e[2]) for e in evs])),
        "ffcp_ms": float(np.mean([e[2].elapsed_time(e[3]) for e in evs])),
        "wall_ms": wall / steps * 1e3,
        "prof": prof, "iterations": int(finfo["iterations"]),
        "converged": int(finfo["converged"]), "fit_core": float(finfo["fit"]),
        "init_used": int(finfo["init_used"]),
        "fit_y": float(fit_y), "normY2": float(tinfo["normY2"]),
        # Fit of the Tucker format against Y (orthonormal U):
        # 1 - sqrt(||Y||^2 - ||G||^2) / ||Y||
        "tucker_fit": float(1.0 - np.sqrt(max(tinfo["normY2"] - tinfo["normG2"], 0.0) /
                                          tinfo["normY2"])),
        "U": [u.double().cpu().numpy() for u in out["U"]],
        "G": out["G"].double().cpu().numpy(),
    }


def run_hals_1e4(P, torch, synth, reps):
    """FFCP-HALS on Section V-A's noise-free nonnegative example at its own
    size: four modes of 10^4, R = 10, exponential (mean 10) factors with
    20 % zeros, handed over as its exact Tucker format (U_n 10^4 x 10, G
    10^4 entries; the tensor itself is never formed).  Times fits of a
    fixed 30 iterations from a U[0,1] start (the fit reaches the rounding
    floor of its closed form by about 17, after which a tolerance test is
    decided by rounding) and reports the recovered components' SIR against
    the generating factors."""
    from scipy.optimize import linear_sum_assignment
    dims, R = (10000,) * 4, 10
    d = synth.nonneg_tucker_format(27, dims, R, "exp", 10.0, 0.2)
    dev = torch.device("cuda:0")
    up = lambda a: torch.from_numpy(synth.f32(a)).to(dev)
    U, G, A0 = [up(u) for u in d["U"]], up(d["G"]), [up(a) for a in d["A0"]]
    stream = torch.cuda.current_stream()

    def fit(ws):
        return P.ffcp(U, G, R, update="hals", A_init=A0, max_it=30, tol=0.0,
                      workspace=ws, sync=False)

    f = fit(None)                      # sizes the workspace
    ws = f["workspace"]
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        f = fit(ws)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    info = np.frombuffer(f["info_dev"].cpu().numpy().tobytes(), P.FFCP_INFO_DTYPE)[0]
    it = int(info["iterations"])
    # SIR (footnote of Section V-A) of zero-mean, unit-variance components,
    # each estimate matched to a true component by the best total correlation
    sirs = []
    for n in range(len(dims)):
        A = d["A"][n]
        B = f["A"][n].double().cpu().numpy()
        za = (A - A.mean(0)) / A.std(0)
        zb = (B - B.mean(0)) / B.std(0)
        rows, cols = linear_sum_assignment(-np.abs(za.T @ zb))
        for r, c in zip(rows, cols):
            b = zb[:, c] * (1.0 if za[:, r] @ zb[:, c] >= 0 else -1.0)
            err = max(float(np.linalg.norm(za[:, r] - b)), 1e-300)
            sirs.append(20.0 * np.log10(np.linalg.norm(za[:, r]) / err))
    return {"workload": "nonneg CP rank 10, 10^4 x 10^4 x 10^4 x 10^4 as its exact "
                        "Tucker format (FP32 U_n, G)",
            "update": "hals", "fits_timed": reps,
            "ms": round(ms, 4), "iterations": it,
            "us_per_iteration": round(ms * 1e3 / max(it, 1), 2),
            "converged": int(info["converged"]), "fit": float(info["fit"]),
            "sir_min_db": round(float(np.min(sirs)), 1),
            "sir_median_db": round(float(np.median(sirs)), 1)}


def train_learned_init(P, torch, synth, cores, epochs, I=300, R=20, rt=30):
    """Untimed setup: cores from the pipeline itself (seeded I^3 CP tensors,
    rank R, congruence U[0.5, 0.95], SNR U[20, 40] dB, precision form with two
    sweeps), then Adam on rt_mlp_train_step (batch 256, lr 1e-3 halved every
    quarter of the epochs)."""
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    Gs = []
    for k in range(cores):
        snr = synth.rngs((5, k))["noise"].uniform(20.0, 40.0)
        d = synth.cp_congruent_device((5, k), (I, I, I), R, 0.5, 0.95, snr, (rt,) * 3,
                                      sweeps=2, device=dev)
        om = [torch.from_numpy(o).to(dev) for o in synth.f32(d["omegas"])]
        omt = [[torch.from_numpy(o).to(dev) for o in synth.f32(lst)]
               for lst in d["omega_tildes"]]
        Gs.append(P.tucker_rand(d["Y"], om, omt, ranks=(R, R, R), sweeps=2,
                                precision="bf16", sync=False)["G"])
    Gtr = torch.stack(Gs)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    net = P.MLP((R, R, R), R, (1024, 1024))
    W, b = synth.mlp_weights(77, net.dims)
    W[2] = W[2] * 0.1
    net.load(W, b)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    t0 = time.perf_counter()
    first = last = None
    for ep in range(epochs):
        perm = torch.randperm(cores, device=dev, generator=gen)
        lr = 1e-3 * 0.5 ** (ep // max(1, epochs // 4))
        ls = [net.train_step(Gtr[perm[i:i + 256]].contiguous(), lr)
              for i in range(0, cores - 255, 256)]
        m = float(torch.cat(ls).mean())
        first = m if first is None else first
        last = m
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # matrix-product work of one sample: forward x W1..W3, backward dX and dW
    # of each layer (3 products of 2 d_l d_{l+1} flop per layer)
    dims = net.dims
    per_sample = 3 * sum(2.0 * dims[l] * dims[l + 1] for l in range(3))
    samples = net.step * 256
    return net, {"cores": cores, "core_tensor": f"{I}^3 CP rank {R}", "epochs": epochs,
                 "steps": net.step, "batch": 256, "generate_s": round(t_gen, 2),
                 "train_s": round(train_s, 3),
                 "train_tflops": round(per_sample * samples / train_s / 1e12, 2),
                 "train_mfma_frac_bf16": round(per_sample * samples / train_s / 1e12 /
                                               PEAK_TFLOPS["bf16"], 5),
                 "loss_first_epoch": round(first, 5), "loss_last_epoch": round(last, 5)}


def bf16_rounding_rms(Y):
    """RMS of bf16_rne(Y) - Y (torch's round-to-nearest-even conversion),
    mode-1 slab by slab."""
    import torch
    e2 = 0.0
    for a in range(0, Y.shape[0], 100):
        blk = Y[a:a + 100]
        e2 += float(((blk.to(torch.bfloat16).to(torch.float32) - blk).double() ** 2).sum())
    return (e2 / Y.numel()) ** 0.5


def errors_vs_oracle(res, forms, ores, Y64, R, tol, max_it, rms_bf16=None):
    """Error of each form's Tucker format and final fit against the FP64
    oracle on the whole tensor (same Omega): projector distance of each U_n,
    the aligned core error e_G, and |Fit_Y - Fit_Y(oracle)| where the oracle
    fits its own core by FFCP-ALS from its HOSVD start to the same tolerance
    and Fit_Y is evaluated against the tensor."""
    from oracle import ffcp as F
    from oracle.metrics import aligned_core_error, projector_distance
    A0 = F.hosvd_init(ores["U"], ores["G"], R)
    f = F.ffcp(ores["U"], ores["G"], A0, update="als", max_it=max_it, tol=tol)
    fit_o = F.cp_fit_mttkrp(Y64, f["A"], f["lam"])
    out = {"oracle_fit_y": fit_o, "oracle_ffcp_iterations": int(f["iterations"])}
    for form in ("bf16", "f32", "f32_one_sweep"):
        if form not in res or forms[form][1] != 2:
            continue
        r = res[form]
        d = [projector_distance(r["U"][k], ores["U"][k]) for k in range(len(r["U"]))]
        eG = aligned_core_error(r["G"], r["U"], ores["G"], ores["U"])
        out[form] = {"d_U_max": max(d), "e_G": eG,
                     "fit_y_abs_diff": abs(r["fit_y"] - fit_o)}
    out["bounds"] = {"f32": {"d_U": 1e-4, "e_G": 1e-4, "fit_y": 1e-5},
                     "bf16": {"fit_y": 1e-4}}
    if rms_bf16 is not None:
        # Wedin: d_n <= s_n / (gap_n - s_n), gap_n from the oracle's G~_(n),
        # s_n = rms(E) (sqrt(I_n) + sqrt(prod_{p != n} I_p)) the norm of the
        # BF16 rounding unfolded; the reported bound is twice the estimate
        Gt = ores["Gt"]
        est = []
        for k in range(Gt.ndim):
            sv = np.linalg.svd(np.moveaxis(Gt, k, 0).reshape(Gt.shape[k], -1),
                               compute_uv=False)
            gap = sv[R - 1] - sv[R]
            In = Y64.shape[k]
            s_n = rms_bf16 * (In ** 0.5 + (Y64.size / In) ** 0.5)
            est.append(s_n / (gap - s_n) if gap > s_n else float("inf"))
        out["bounds"]["bf16"]["d_U"] = 2.0 * max(est)
        out["bounds"]["bf16"]["e_G"] = 2.0 * float(np.sqrt(np.sum(np.square(est)))) + 2.0 ** -9
        out["bounds"]["bf16"]["wedin_estimates"] = est
        out["bounds"]["bf16"]["rounding_rms"] = rms_bf16
    return out


def tucker_only(args, P, torch, Y, om_d, omt_d, ranks, ybf16):
    """The Tucker stage alone (two sweeps in the chosen form), then the
    calibration copies: the command the kernel-trace and counter profiles
    under profiles/ were taken with."""
    kw = dict(ranks=ranks, sweeps=2, precision=args.precision, ybf16=ybf16)
    out = None
    for _ in range(max(args.warmup, 1)):
        out = P.tucker_rand(Y, om_d, omt_d, workspace=out and out["workspace"], **kw)
    torch.cuda.synchronize()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = P.tucker_rand(Y, om_d, omt_d, workspace=out["workspace"], sync=False, **kw)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    prof = P.profile_read()
    P.profile_enable(False)
    if args.copy_calibration:
        dst = torch.empty(Y.shape, dtype=torch.float64, device=Y.device)
        for _ in range(args.copy_calibration):
            dst.copy_(Y)
        torch.cuda.synchronize()
        del dst
    print(json.dumps({"tucker_only": args.precision, "steps": args.steps,
                      "ms_per_step": round(wall, 4),
                      "stages_ms": {k: round(v[0] / max(v[1], 1), 4)
                                    for k, v in prof.items() if v[1] > 0}}), flush=True)


def ffcp_only(args, P, torch, Y, om_d, omt_d, ranks, R, ybf16):
    """The precision form's Tucker stage once, then `steps` FFCP-ALS calls
    on its core from the HOSVD start: the command the FFCP-ALS kernel-trace
    profile under profiles/ was taken with."""
    out = P.tucker_rand(Y, om_d, omt_d, ranks=ranks, sweeps=2, precision="bf16",
                        ybf16=ybf16)
    kw = dict(update="als", max_it=args.max_it, tol=args.tol, init="hosvd")
    f = P.ffcp(out["U"], out["G"], R, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        f = P.ffcp(out["U"], out["G"], R, workspace=f["workspace"], sync=False, **kw)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    info = np.frombuffer(f["info_dev"].cpu().numpy().tobytes(), P.FFCP_INFO_DTYPE)[0]
    print(json.dumps({"ffcp_only": "als", "steps": args.steps, "ms": round(ms, 4),
                      "iterations": int(info["iterations"]),
                      "us_per_iteration_incl_start": round(1e3 * ms / int(info["iterations"]), 2),
                      "fit": float(info["fit"])}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not "
              "supported (the sharded path is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1412_1885_amd as P
    import synth

    P.lib()  # raises if the HIP library is missing: no fallback
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.hals_only:
        print(json.dumps({"hals_1e4_4way": run_hals_1e4(P, torch, synth, args.steps)}),
              flush=True)
        return

    I, R, rt = args.size, 20, 30
    dims = (I, I, I)
    ranks = (R, R, R)
    d = synth.cp_congruent_device(1885, dims, R, 0.5, 0.95, 30.0, (rt,) * 3,
                                  sweeps=2, device=dev)
    Y = d["Y"]
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    om_d = [torch.from_numpy(o).to(dev) for o in om32]
    omt_d = [[torch.from_numpy(o).to(dev) for o in lst] for lst in omt32]
    ybf16 = torch.empty(P.bf16_copy_shape(dims), dtype=torch.int16, device=dev)
    torch.cuda.synchronize()

    if args.tucker_only:
        tucker_only(args, P, torch, Y, om_d, omt_d, ranks, ybf16)
        return
    if args.ffcp_only:
        ffcp_only(args, P, torch, Y, om_d, omt_d, ranks, R, ybf16)
        return

    net, learned = None, None
    if args.train_cores > 0:
        net, learned = train_learned_init(P, torch, synth, args.train_cores,
                                          args.train_epochs)
    A_random = [torch.from_numpy(a).to(dev) for a in
                synth.f32(synth.init_factors(d["init_rng"], dims, R))]

    # (precision, sweeps, learned start).  The plain FP32 path runs the same
    # two sweeps as the precision form, so both reach the same subspaces and
    # the same fit; one FP32 sweep is timed as well, for context (on this
    # workload its subspaces, and so its fit, are clearly worse).  The
    # precision form from the HOSVD start isolates what the learned start
    # gains.
    forms = {"bf16": ("bf16", 2, "learned"), "bf16_hosvd": ("bf16", 2, "hosvd"),
             "bf16_random": ("bf16", 2, "random"), "f32": ("f32", 2, "hosvd"),
             "f32_one_sweep": ("f32", 1, "hosvd"),
             "f32_gauss_seidel": ("f32", 2, "hosvd")}
    main_form = args.precision
    order = [f for f in forms if f != main_form] + [main_form]   # the step's form last
    res = {}
    for form in order:
        prec, sw, start = forms[form]
        res[form] = run_form(P, torch, Y, om_d, omt_d, ranks, R, prec, sw,
                             args.steps, args.warmup, args.tol, args.max_it, ybf16,
                             net if start == "learned" else None,
                             A_random if start == "random" else None,
                             "gauss_seidel" if form.endswith("gauss_seidel") else "jacobi")
    m = res[main_form]

    # algorithmic HBM bytes of the Tucker stage (each pass reads Y once):
    # plain FP32: 4 B per element per sweep + 4 B for the core pass;
    # precision form: FP32 read + BF16 write (first sweep), then 2 B per
    # element per later sweep and for the core pass
    n = Y.numel()

    def alg_bytes(form):
        prec, sw, _ = forms[form]
        passes = 2 * sw + 1 if form.endswith("gauss_seidel") else sw + 1
        return (4 * passes if prec == "f32" else 4 + 2 + 2 * (passes - 1)) * n

    value = alg_bytes(main_form) / (m["tucker_ms"] * 1e-3) / 1e9

    # The dominant contraction kernel: the first sweep's streaming kernel
    # (two mode products in one read of Y).  Every Y-streaming kernel of the
    # step's form is priced beside it.
    workload = f"cp{R}_congruent_{I}x{I}x{I}_f32"

    def per_launch(stage):
        ms_k, n_k = m["prof"].get(stage, (0.0, 0))
        return ms_k / max(n_k, 1) * 1e-3 if n_k else None

    kernels = {}
    if main_form == "f32":
        t_k = per_launch("first_pass")
        flops = 2.0 * n * (rt + rt)   # Y x_3 Omega_3^T and Y x_2 Omega_2^T
        achieved = flops / t_k / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2),
                "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS["f32"], 4),
                "traffic": stored_traffic("dual_f32_kernel", workload),
                "kernel": "dual_f32_kernel (first sweep: Y x_3 Omega_3^T and "
                          "Y x_2 Omega_2^T in one read of Y)",
                "avg_ms": round(t_k * 1e3, 4)}
        for stage, b in (("first_pass", 4), ("sweep_pass", 4), ("core_pass", 4)):
            t = per_launch(stage)
            if t:
                kernels[stage] = {"bytes": b * n, "avg_ms": round(t * 1e3, 4),
                                  "gbs": round(b * n / t / 1e9, 1),
                                  "hbm_frac": round(b * n / t / 1e9 / HBM_PEAK_GBS, 4)}
    else:
        # bytes each pass must move: Y (FP32 in the first pass, BF16 after),
        # the BF16 copy written by a fused first pass, the FP32 outputs TA
        # (A I_2 R~_3), TB (A R~_2 I_3) and C (A R~_2 R~_3)
        A_, I1_, I2_ = n // (dims[-2] * dims[-1]), dims[-2], dims[-1]
        ta, tb, cc = 4 * A_ * I1_ * rt, 4 * A_ * rt * I2_, 4 * A_ * rt * rt
        fused = per_launch("convert") is None   # wide slabs: conversion in the first pass
        if fused:
            passes = (("first_pass", 6 * n + ta + tb,
                       "bf16_cs_kernel<true,true,2>: FP32 Y read once; BF16 copy, "
                       "TA = Y x_3 Omega_3^T and TB = Y x_2 Omega_2^T"),
                      ("sweep_pass", 2 * n + ta + tb + cc,
                       "bf16_cs_kernel<false,true,2>: second sweep from the copy; TA, TB "
                       "and C = TA x_2 Q_2^T"),
                      ("core_pass", 2 * n + cc,
                       "bf16_cs_kernel<false,false,2>: core pass, C = Y x_3 Q_3^T x_2 Q_2^T "
                       "per slab"))
        else:
            passes = (("convert", 6 * n, "bf16_convert_kernel (FP32 read, BF16 write)"),
                      ("first_pass", 2 * n + ta + tb, "bf16_stream_kernel, first sweep"),
                      ("sweep_pass", 2 * n + ta + tb, "bf16_stream_kernel, second sweep"),
                      ("core_pass", 2 * n + ta, "bf16_stream_kernel, core pass"))
        kname = "bf16_cs_kernel" if fused else "bf16_stream_kernel"
        kbytes = dict((st, b) for st, b, _ in passes)["first_pass"]
        t_k = per_launch("first_pass")
        achieved = kbytes / t_k / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(kname, workload),
                "kernel": dict((st, k) for st, _, k in passes)["first_pass"],
                "bytes_per_launch": kbytes,
                "avg_ms": round(t_k * 1e3, 4)}
        for stage, b, kn in passes:
            t = per_launch(stage)
            if t:
                kernels[stage] = {"kernel": kn, "bytes": b,
                                  "avg_ms": round(t * 1e3, 4),
                                  "gbs": round(b / t / 1e9, 1),
                                  "hbm_frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}

    if args.copy_calibration:
        # plain elementwise copy kernel of known traffic (reads 4 B, writes
        # 8 B per element): the scale for the HBM byte counters
        dst = torch.empty(Y.shape, dtype=torch.float64, device=dev)
        for _ in range(args.copy_calibration):
            dst.copy_(Y)
        torch.cuda.synchronize()
        del dst

    hals = None if args.no_hals else run_hals_1e4(P, torch, synth, 3)

    # Algorithm 2 (sequential RandTucker, dense counter-based Gaussian test
    # matrices) on the same tensor, R~ = 30 in every mode: time, bytes and
    # the captured energy beside the Jacobi RandTucker2i's at the same width
    seq = None
    if not args.no_sequential:
        stream = torch.cuda.current_stream()
        out_s = P.tucker_sequential(Y, (rt,) * 3, 14121885)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(3)]
        for a, b in evs:
            a.record(stream)
            out_s = P.tucker_sequential(Y, (rt,) * 3, 14121885, sync=False)
            b.record(stream)
        torch.cuda.synchronize()
        ms_s = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        g2 = float((out_s["G"].double() ** 2).sum())
        y2 = m["normY2"]
        rows1 = I * I
        seq = {"workload": f"{I}^3 FP32, R~ = {rt} per mode, no truncation",
               "ms": round(ms_s, 4),
               "bytes": {"tensor_passes": 2 * 4 * n, "omega_1": 2 * 4 * rows1 * rt},
               "tucker_fit_rt": 1.0 - float(np.sqrt(max(y2 - g2, 0.0) / y2)),
               "note": "two passes over Y (sketch, then projection) and the dense "
                       "Omega_1 written and read; RandTucker2i reads Y (S + 1) times "
                       "with Kronecker-structured test matrices"}
        del out_s

    cpu, errors = None, None
    if not args.no_cpu_baseline:
        cpu, ores, Ys = cpu_baseline(Y, om32, omt32, ranks, args.cpu_slab,
                                     forms[main_form][1], alg_bytes(main_form) // n)
        if args.cpu_slab >= I:
            errors = errors_vs_oracle(res, forms, ores, Ys, R, args.tol, args.max_it,
                                      bf16_rounding_rms(Y))
        del Ys

    def summary(form):
        r = res[form]
        learned_start = forms[form][2] == "learned" and net is not None
        start = {"learned": "learned (guarded by HOSVD)", "hosvd": "HOSVD",
                 "random": "seeded N(0,1) factors"}[forms[form][2]]
        return {"precision": forms[form][0], "sweeps": forms[form][1],
                "order": "gauss_seidel" if form.endswith("gauss_seidel") else "jacobi",
                "tucker_fit": r["tucker_fit"],
                "tucker_ms": round(r["tucker_ms"], 4),
                "tucker_gbs": round(alg_bytes(form) / (r["tucker_ms"] * 1e-3) / 1e9, 1),
                "start": start,
                "start_kept": r["init_used"] if learned_start else None,
                "init_ms": round(r["init_ms"], 4),
                "ffcp_ms": round(r["ffcp_ms"], 4),
                "time_to_fit_ms": round(r["tucker_ms"] + r["init_ms"] + r["ffcp_ms"], 4),
                "ffcp_iterations": r["iterations"], "ffcp_converged": r["converged"],
                "fit_core": r["fit_core"], "fit_y": r["fit_y"],
                "stages_ms": {k: round(v[0] / max(v[1], 1), 4)
                              for k, v in r["prof"].items() if v[1] > 0}}

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["wall_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_form,
        "data": "synthetic",
        "config": {
            "workload": workload,
            "description": (f"{I}^3 FP32 CP rank {R}, column congruence "
                            "U[0.5,0.95], SNR 30 dB; Omega_n "
                            f"{I}x{rt}, Omega~_n {rt * rt}x{rt}; Tucker ranks "
                            f"{ranks}; FFCP ALS R={R}, tol {args.tol}; precision "
                            "form: BF16 passes, two sweeps, learned start; plain "
                            "FP32: two sweeps, HOSVD start"),
            "dims": list(dims), "ranks": list(ranks), "ranks_tilde": [rt] * 3,
            "sweeps": forms[main_form][1], "R": R, "update": "als",
        },
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        **{f: summary(f) for f in forms},
        "fit_y_rel_diff_mixed_vs_plain": abs(res["bf16"]["fit_y"] - res["f32"]["fit_y"]) /
            max(abs(res["f32"]["fit_y"]), 1e-300),
        "time_to_fit_mixed_over_plain": round(
            (res["bf16"]["tucker_ms"] + res["bf16"]["init_ms"] + res["bf16"]["ffcp_ms"]) /
            (res["f32"]["tucker_ms"] + res["f32"]["init_ms"] + res["f32"]["ffcp_ms"]), 4),
        "learned_gain": {
            "ffcp_iterations_learned": res["bf16"]["iterations"],
            "ffcp_iterations_hosvd": res["bf16_hosvd"]["iterations"],
            "ffcp_iterations_random": res["bf16_random"]["iterations"],
            "ffcp_ms_learned_incl_inference": round(res["bf16"]["init_ms"] +
                                                    res["bf16"]["ffcp_ms"], 4),
            "ffcp_ms_hosvd": round(res["bf16_hosvd"]["init_ms"] +
                                   res["bf16_hosvd"]["ffcp_ms"], 4),
            "ffcp_ms_random": round(res["bf16_random"]["ffcp_ms"], 4),
            "fit_y": {k: res[k]["fit_y"] for k in ("bf16", "bf16_hosvd", "bf16_random")},
            "note": "all arms: precision form, two sweeps, same tensor; the learned "
                    "arm includes the network's inference and the HOSVD guard"},
        "gauss_seidel_vs_jacobi": {
            "note": "plain FP32, two sweeps: the printed loop order of Algorithm 3 "
                    "takes two passes over Y per sweep, the Jacobi order one",
            "bytes": {"jacobi": alg_bytes("f32"), "gauss_seidel": alg_bytes("f32_gauss_seidel")},
            "tucker_ms": {"jacobi": round(res["f32"]["tucker_ms"], 4),
                          "gauss_seidel": round(res["f32_gauss_seidel"]["tucker_ms"], 4)},
            "tucker_fit": {"jacobi": res["f32"]["tucker_fit"],
                           "gauss_seidel": res["f32_gauss_seidel"]["tucker_fit"]},
            "fit_y": {"jacobi": res["f32"]["fit_y"],
                      "gauss_seidel": res["f32_gauss_seidel"]["fit_y"]}},
        "errors_vs_fp64_oracle": errors,
        "kernels": kernels,
        "learned_init": learned,
        "hals_1e4_4way": hals,
        "sequential_alg2": seq,
        "normY2": m["normY2"],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
