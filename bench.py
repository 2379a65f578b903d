"""Benchmark of the marching-on-in-time step of the fast TDBEM on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp64|fp32] [--nrhs R]

A step is one full marching step (incident field read from HBM, near-field
history sum, far-field passes at the time gates, Z0 solve, history update).
The workload is the 20480-triangle PEC sphere of radius 1 m (c dt = 0.02 m,
modulated Gaussian 300/200 MHz, p_s = p_t = 4, leaves of at most 64 edges).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MOT steps/s and M2L roofline %, chosen vs plain FP64 IFMM at rel err 1e-4"
PEAK_HBM = 8.0e12          # B/s
PEAK_FP64 = 78.6e12        # FLOP/s, dense FP64 on the matrix cores
PEAK_FP32 = 157.3e12       # FLOP/s, dense FP32 on the matrix cores
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_m2l_off_sphere20480_traffic.json")


def gate_schedule(Mt, lmax, first, last):
    """Per level, the time gates alpha in [first, last] (alpha % M_t(l) == 0)."""
    out = {}
    for l in range(2, lmax + 1):
        M = Mt[l]
        out[l] = [a for a in range(first, last + 1) if a % M == 0]
    return out


def m2l_traffic(form):
    """HBM bytes per M2L launch from the committed counter summary, or None when
    the M2L source has changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        src = os.path.join(ROOT, rec["source"])
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if sha != rec["source_sha256"] or form not in rec["bytes_per_launch"]:
            return None
        return rec["bytes_per_launch"][form]
    except (OSError, KeyError, ValueError):
        return None


def copy_probe(torch, mib=512):
    """One plain device copy of known size (read mib MiB, write mib MiB): the
    reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    return {"bytes_read": n * 8, "bytes_written": n * 8}


def cpu_baseline(workload, rows=8):
    """Oracle (conventional method) history sum per step on a sample of rows."""
    from oracle import oracle as O
    from paper_2303_05006_amd.inputs import C0
    m = O.Mesh(workload.verts, workload.tris)
    cdt = workload.dt * C0
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(m.ne, rows, replace=False))
    nthreads = min(16, os.cpu_count() or 1)
    Z = O.zrows(m, sample, cdt, workload.theta, workload.zeta, nthreads=nthreads)     # untimed: coefficients
    # sparse lag strips of the sampled rows, as the oracle's history routine takes them
    r_, c_, g0, ln, off, vals = [], [], [], [], [], []
    pos = 0
    for ri in range(rows):
        nz = np.nonzero(np.abs(Z[ri]).max(axis=1))[0]
        for j in nz:
            g = np.nonzero(Z[ri, j])[0]
            a, b = g.min(), g.max()
            r_.append(ri); c_.append(j); g0.append(a); ln.append(b - a + 1); off.append(pos)
            vals.append(Z[ri, j, a:b + 1]); pos += b - a + 1
    import ctypes
    L = O.lib()
    arr = lambda x, t: np.ascontiguousarray(np.array(x, dtype=t))
    r_, c_, g0, ln = (arr(x, np.int32) for x in (r_, c_, g0, ln))
    off = arr(off, np.int64)
    vals = np.ascontiguousarray(np.concatenate(vals))
    G = Z.shape[2]
    nb = G + 2
    hist = rng.standard_normal((nb, m.ne))
    out = np.zeros(m.ne)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    reps = 0
    t0 = time.perf_counter()
    while True:
        L.orc_history(len(r_), P(r_), P(c_), P(g0), P(ln), P(off), P(vals), m.ne, P(hist), nb, nb, 2, P(out))
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 and reps >= 3:
            break
    per_sample = el / reps
    per_step = per_sample * m.ne / rows
    return {"value": 1.0 / per_step, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"conventional-method history sum sum_g Zt^(g) J^(a-g) over all 30720 source edges and all "
                       f"lags for {rows} target rows ({pos} stored coefficients; coefficients precomputed, "
                       f"untimed), {reps} repetitions, scaled by {m.ne}/{rows} rows")}


def make_solver(torch, tdbem, w, form, guess, rtol):
    nr = len(w.pulses)
    prec = tdbem.FP64 if form == "fp64" else tdbem.FP32
    cfg = tdbem.Config(dt=w.dt, nt=w.nt, theta=w.theta, zeta=w.zeta, leaf_max=w.leaf_max, mode=tdbem.MODE_IFMM,
                       precision=prec, n_rhs=nr, gmres_rtol=rtol, gmres_maxit=60,
                       guess=tdbem.GUESS_LEARNED if guess == "learned" else tdbem.GUESS_EXTRAP)
    t0 = time.perf_counter()
    S = tdbem.Solver(w.verts, w.tris, cfg)
    if guess == "learned":
        from paper_2303_05006_amd.train_guess import DEFAULT_OUT
        S.guess_weights(np.load(DEFAULT_OUT))
    torch.cuda.synchronize()
    return S, time.perf_counter() - t0


def march(torch, S, V, W, K, traj):
    """W untimed + K timed steps on the resident incident fields V [W+K][rhs][N_e];
    traj (or None) receives J of every step.  Returns (seconds, GMRES iterations)."""
    J = torch.zeros(V.shape[1:], dtype=torch.float64, device="cuda")
    for a in range(1, W + 1):
        S.step(V[a - 1], J)
        if traj is not None:
            traj[a - 1].copy_(J)
    torch.cuda.synchronize()
    S.profile(True)
    iters = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for a in range(W + 1, W + K + 1):
        S.step(V[a - 1], J)
        if traj is not None:
            traj[a - 1].copy_(J)
        iters.append(S.gmres_iters())
    torch.cuda.synchronize()
    return time.perf_counter() - t1, iters


def kernel_rooflines(info, ph, W, K, nr, prec_fp64, form):
    """Achieved rates of the M2L and near-field kernels over the timed steps."""
    lmax = info["lmax"]
    gates = gate_schedule(info["Mt"], lmax, W + 1, W + K)
    win = info["window"]
    m2l_flops = 0.0
    for l in range(2, lmax + 1):
        for a in gates[l]:
            k = a // info["Mt"][l] - 1
            lags = min(win, k + 1)
            m2l_flops += info["nilist"][l] * lags * 7 * 2.0 * 256 * 256 * nr
    vb = 8 if prec_fp64 else 4
    near_bytes = K * (info["near_nnz"] * vb + info["near_pairs"] * 8 + info["ne"] * 8 * nr)
    kernels = {}
    t_m2l = ph["m2l"][0] * 1e-3
    t_near = ph["near"][0] * 1e-3
    if t_m2l > 0:
        kernels["m2l"] = {"bound": "mfma", "achieved": m2l_flops / t_m2l / 1e12, "unit": "TFLOP/s",
                          "peak": (PEAK_FP64 if prec_fp64 else PEAK_FP32) / 1e12,
                          "launches": ph["m2l"][1], "ms_total": ph["m2l"][0],
                          "ms_per_launch": ph["m2l"][0] / max(ph["m2l"][1], 1),
                          "flop_per_launch": m2l_flops / max(ph["m2l"][1], 1)}
    if t_near > 0:
        kernels["near"] = {"bound": "hbm", "achieved": near_bytes / t_near / 1e9, "unit": "GB/s",
                           "peak": PEAK_HBM / 1e9, "launches": ph["near"][1], "ms_total": ph["near"][0]}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"]) if kernels else None
    roof = None
    if dom:
        kd = kernels[dom]
        traffic = m2l_traffic(form) if (dom == "m2l" and nr == 1) else None
        roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["achieved"] / kd["peak"], "traffic": traffic}
    return roof, kernels


def batched_runs(torch, tdbem, W, K, rtol, single_fp64_steps_per_s):
    """64 incident fields (Fibonacci directions, seeded polarisations) marched
    together: the plain FP64 form and the chosen form (FP32 near values and
    M2L, learned initial guess), W + K steps each with the fields resident in
    HBM, K timed; the chosen form's error is taken against the FP64 batch over
    all W + K steps (the pulse crosses the sphere from about step 200)."""
    from paper_2303_05006_amd.inputs import workload
    w = workload("sphere20480x64", n_rhs=64)
    nr = len(w.pulses)
    last = W + K
    out = {"workload": f"sphere20480x64: the same sphere, {nr} incident fields, steps {W + 1}..{last} timed",
           "n_rhs": nr, "steps": K, "warmup": W}
    trajs = {}
    for key, form, guess in (("fp64", "fp64", "extrap"), ("chosen", "fp32", "learned")):
        S, setup = make_solver(torch, tdbem, w, form, guess, rtol)
        V = torch.zeros((last, nr, S.ne), dtype=torch.float64, device="cuda")
        for a in range(1, last + 1):
            S.incident(w.pulses, a, V[a - 1])
        traj = torch.zeros((last, nr, S.ne), dtype=torch.float64, device="cuda")
        el, iters = march(torch, S, V, W, K, traj)
        ph = S.phase_times()
        roof, _ = kernel_rooflines(S.info(), ph, W, K, nr, form == "fp64", form)
        out[key] = {"form": form + (" + learned initial guess" if guess == "learned" else ""),
                    "steps_per_s": K / el, "rhs_steps_per_s": nr * K / el, "ms_per_step": el / K * 1e3,
                    "gmres_iters_mean": float(np.mean(iters)), "roofline": roof,
                    "phase_ms": {k: v[0] for k, v in ph.items()}, "setup_s": setup}
        trajs[key] = traj
        S.close()
        del V
    a, b = trajs["chosen"], trajs["fp64"]
    out["chosen"]["rel_l2_err_vs_fp64"] = float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt())
    out["chosen"]["err_over_steps"] = f"1..{last}"
    out["chosen"]["speedup_vs_fp64_batched"] = out["chosen"]["steps_per_s"] / out["fp64"]["steps_per_s"]
    out["chosen"]["rhs_throughput_vs_fp64_single"] = out["chosen"]["rhs_steps_per_s"] / single_fp64_steps_per_s
    del trajs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=480)
    ap.add_argument("--warmup", type=int, default=240)
    ap.add_argument("--form", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-chosen", action="store_true",
                    help="skip the chosen-form run (FP32 + learned guess) and its error against FP64")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--guess", default="extrap", choices=["extrap", "learned"],
                    help="initial guess of the Z0 solve (learned: the committed network parameters)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched runs (64 incident fields, FP64 and FP32 + learned guess)")
    ap.add_argument("--batched-steps", type=int, default=60)
    ap.add_argument("--batched-warmup", type=int, default=240)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, run one 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_05006_amd import tdbem
    from paper_2303_05006_amd.inputs import workload

    torch.cuda.set_device(0)
    name = "sphere20480" if args.nrhs == 1 else "sphere20480x64"
    w = workload(name, n_rhs=args.nrhs)
    nr = len(w.pulses)
    W, K = args.warmup, args.steps
    last = W + K
    chosen = not args.no_chosen and nr == 1 and args.form == "fp64" and args.guess == "extrap"

    S, setup_s = make_solver(torch, tdbem, w, args.form, args.guess, args.rtol)
    info = S.info()
    ne = S.ne
    # incident fields of every step resident in HBM before timing
    V = torch.zeros((last, nr, ne), dtype=torch.float64, device="cuda")
    for a in range(1, last + 1):
        S.incident(w.pulses, a, V[a - 1])
    traj = torch.zeros((last, nr, ne), dtype=torch.float64, device="cuda") if chosen else None
    el, iters = march(torch, S, V, W, K, traj)
    ph = S.phase_times()
    prec_fp64 = args.form == "fp64"
    roof, kernels = kernel_rooflines(info, ph, W, K, nr, prec_fp64, args.form)
    res = {
        "metric": METRIC,
        "value": K / el,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: PEC sphere r=1 m, 20480 triangles / {ne} RWG edges, c dt = 0.02 m, "
                               f"IFMM p_s=p_t=4, leaves <= 64 edges, {nr} incident field(s), steps {W + 1}..{last} of 1000",
                   "form": args.form, "n_rhs": nr, "gmres_rtol": args.rtol, "guess": args.guess},
        "roofline": roof,
        "kernels": kernels,
        "rhs_steps_per_s": nr * K / el,
        "near_interactions_per_s": info["near_nnz"] * nr * K / el,
        "phase_ms": {k: v[0] for k, v in ph.items()},
        "phase_launches": {k: v[1] for k, v in ph.items()},
        "gmres_iters_mean": float(np.mean(iters)),
        "setup_s": setup_s,
        "hierarchy": {k: info[k] for k in ("lmax", "Mt", "ncells", "nilist", "near_nnz", "near_pairs", "z0_nnz", "window")},
        "device_gb": info["device_bytes"] / 1e9,
    }
    S.close()
    if chosen:
        # chosen form on the same incident fields: FP32 near values and M2L
        # products, learned initial guess; error of its march against FP64's
        S2, setup2 = make_solver(torch, tdbem, w, "fp32", "learned", args.rtol)
        traj32 = torch.zeros_like(traj)
        el2, iters2 = march(torch, S2, V, W, K, traj32)
        ph2 = S2.phase_times()
        roof2, kernels2 = kernel_rooflines(S2.info(), ph2, W, K, nr, False, "fp32")
        err = float(((traj32 - traj) ** 2).sum().sqrt() / (traj ** 2).sum().sqrt())
        res["chosen"] = {"form": "fp32 near values and M2L + learned initial guess", "value": K / el2,
                         "unit": "steps/s", "ms_per_step": el2 / K * 1e3, "speedup_vs_fp64": el / el2,
                         "rel_l2_err_vs_fp64": err, "err_over_steps": f"1..{last}",
                         "roofline": roof2, "kernels": kernels2,
                         "phase_ms": {k: v[0] for k, v in ph2.items()},
                         "gmres_iters_mean": float(np.mean(iters2)), "setup_s": setup2}
        S2.close()
    if chosen and not args.no_batched:
        res["batched"] = batched_runs(torch, tdbem, args.batched_warmup, args.batched_steps, args.rtol, K / el)
    if args.copy_probe:
        res["copy_probe"] = copy_probe(torch)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
