"""Benchmark of the marching-on-in-time step of the fast TDBEM on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp64|fp32] [--nrhs R]

A step is one full marching step (incident field read from HBM, near-field
history sum, far-field passes at the time gates, Z0 solve, history update).
The workload is the 20480-triangle PEC sphere of radius 1 m (c dt = 0.02 m,
modulated Gaussian 300/200 MHz, p_s = p_t = 4, leaves of at most 64 edges),
marched 1000 steps.  The timed steps always lie in the steady state: the
lead-in before them is at least the coarsest level's full M2L window (W
intervals of M_t(2) steps) and the pulse's arrival on the sphere, and their
number is a whole number of coarsest time gates; --warmup and --steps are
raised to those floors.  Both forms are marched on to step 1000 (untimed) for
the error of the chosen form.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MOT steps/s and M2L roofline %, chosen vs plain FP64 IFMM at rel err 1e-4"
PEAK_HBM = 8.0e12          # B/s
PEAK_FP64 = 78.6e12        # FLOP/s, dense FP64 on the matrix cores
PEAK_FP32 = 157.3e12       # FLOP/s, dense FP32 on the matrix cores
PEAK_BF16 = 2.5e15         # FLOP/s, dense bf16 on the matrix cores
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_m2l_off_sphere20480_traffic.json")
NT = 1000                  # steps of the workload


def gate_schedule(Mt, lmax, first, last):
    """Per level, the time gates alpha in [first, last] (alpha % M_t(l) == 0)."""
    out = {}
    for l in range(2, lmax + 1):
        M = Mt[l]
        out[l] = [a for a in range(first, last + 1) if a % M == 0]
    return out


def steady_window(W, K, Mt2, window, arrival):
    """Lead-in and timed step count raised to the steady state: the lead-in
    covers the coarsest level's full window (window * Mt2 steps) and the
    pulse's arrival step, rounded up to whole coarsest intervals; the timed
    steps are a whole number of coarsest intervals (every level's gates in
    proportion)."""
    lead = max(W, window * Mt2, arrival)
    lead = -(-lead // Mt2) * Mt2
    K = max(Mt2, -(-K // Mt2) * Mt2)
    return lead, K


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


def near_traffic():
    """HBM bytes per launch of the one-rhs per-leaf near-field kernel (FP64)
    from the same counter summary, or None when its source has changed."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        for name, k in rec.get("other_kernels", {}).items():
            if name.startswith("k_near_leaf<double"):
                with open(os.path.join(ROOT, k["source"]), "rb") as f:
                    if hashlib.sha256(f.read()).hexdigest() == k["source_sha256"]:
                        return k["bytes_per_launch"]
        return None
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


def physical_cores():
    """Physical cores from lscpu (unique core, socket pairs), capped by the
    OpenMP thread count the host grants (its CPU share)."""
    n = 0
    try:
        out = subprocess.run(["lscpu", "-p=core,socket"], capture_output=True, text=True, timeout=10).stdout
        n = len({ln for ln in out.splitlines() if ln and not ln.startswith("#")})
    except (OSError, subprocess.SubprocessError):
        pass
    n = n or (os.cpu_count() or 1)
    cap = int(os.environ.get("OMP_NUM_THREADS", n))
    return n, max(1, min(n, cap))


def cpu_baseline(workload, min_seconds=10.0):
    """The oracle's conventional (all-pairs) marching step on the host, from a
    bounded sample: its history sum sum_g Zt^(g) J^(a-g) over every source edge
    and lag for a sample of target rows (the rows split over the cores, one
    oracle call per core, as the paper parallelises over targets), scaled by
    N_e / rows; plus its Z0 solve (back-substitution with the dense LU factors,
    as the oracle's march does), timed at n = 6144 and scaled by (N_e/6144)^2.
    Coefficients and factors are precomputed and untimed."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor
    import scipy.linalg as sla
    from oracle import oracle as O
    from oracle.constants import C0
    phys, cores = physical_cores()
    m = O.Mesh(workload.verts, workload.tris)
    cdt = workload.dt * C0
    rng = np.random.default_rng(0)
    rows = 4 * cores
    sample = np.sort(rng.choice(m.ne, rows, replace=False))
    Z = O.zrows(m, sample, cdt, workload.theta, workload.zeta, nthreads=cores)     # untimed
    G = Z.shape[2]
    nb = G + 2
    hist = rng.standard_normal((nb, m.ne))
    L = O.lib()
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    groups = []
    nnz = 0
    for part in np.array_split(np.arange(rows), cores):
        r_, c_, g0, ln, off, vals = [], [], [], [], [], []
        pos = 0
        for ri in part:
            for j in np.nonzero(np.abs(Z[ri]).max(axis=1))[0]:
                g = np.nonzero(Z[ri, j])[0]
                a, b = g.min(), g.max()
                r_.append(ri); c_.append(j); g0.append(a); ln.append(b - a + 1); off.append(pos)
                vals.append(Z[ri, j, a:b + 1]); pos += b - a + 1
        arr = lambda x, t: np.ascontiguousarray(np.array(x, dtype=t))
        grp = (arr(r_, np.int32), arr(c_, np.int32), arr(g0, np.int32), arr(ln, np.int32), arr(off, np.int64),
               np.ascontiguousarray(np.concatenate(vals)), np.zeros(m.ne))
        groups.append(grp)
        nnz += pos
    del Z

    def run(grp):
        r_, c_, g0, ln, off, vals, out = grp
        L.orc_history(len(r_), P(r_), P(c_), P(g0), P(ln), P(off), P(vals), m.ne, P(hist), nb, nb, 2, P(out))

    reps = 0
    with ThreadPoolExecutor(max_workers=cores) as ex:
        t0 = time.perf_counter()
        while True:
            list(ex.map(run, groups))
            reps += 1
            el = time.perf_counter() - t0
            if el > min_seconds and reps >= 2:
                break
    t_hist = el / reps * m.ne / rows
    # solve: dense LU back-substitution (the oracle's march_dense), O(n^2)
    n_s = 6144
    A = rng.standard_normal((n_s, n_s)) + n_s * np.eye(n_s)
    lu = sla.lu_factor(A)
    x = rng.standard_normal(n_s)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < 2.0 or k < 3:
        sla.lu_solve(lu, x)
        k += 1
    t_solve = (time.perf_counter() - t0) / k * (m.ne / n_s) ** 2
    per_step = t_hist + t_solve
    return {"value": 1.0 / per_step, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "physical_cores_lscpu": phys,
            "sample": (f"conventional-method step: history sum over all {m.ne} source edges and all lags for "
                       f"{rows} sampled target rows ({nnz} stored coefficients) on {cores} threads, {reps} "
                       f"repetitions, scaled by {m.ne}/{rows} rows ({t_hist:.3f} s); Z0 solve as dense LU "
                       f"back-substitution timed at n = {n_s} and scaled by (n/{n_s})^2 ({t_solve:.3f} s); "
                       f"coefficients and LU factors precomputed, untimed")}


NEAR_FORMS = [(2, 1), (1, 1), (3, 1), (2, 2), (1, 2), (2, 0), (1, 0), (0, 0)]   # TDBEM_Q_TUNED shapes, near_kernel 1..8


def make_solver(torch, tdbem, w, form, guess, rtol, same_as=None, graph=0):
    """A context of the workload; the set-up autotuner picks the near-field
    form and the solve's blocks, unless same_as (a TDBEM_Q_TUNED record) fixes
    them to another context's choice."""
    nr = len(w.pulses)
    prec = tdbem.FP64 if form == "fp64" else tdbem.FP32
    fix = {}
    if same_as is not None:
        fix = dict(autotune=0, near_kernel=NEAR_FORMS.index((int(same_as[0]), int(same_as[1]))) + 1,
                   gmres_blocks=int(same_as[2]))
    else:
        fix = dict(autotune=1)
    cfg = tdbem.Config(dt=w.dt, nt=w.nt, theta=w.theta, zeta=w.zeta, leaf_max=w.leaf_max, mode=tdbem.MODE_IFMM,
                       precision=prec, n_rhs=nr, gmres_rtol=rtol, gmres_maxit=60,
                       guess=tdbem.GUESS_LEARNED if guess == "learned" else tdbem.GUESS_EXTRAP, graph=graph, **fix)
    t0 = time.perf_counter()
    S = tdbem.Solver(w.verts, w.tris, cfg)
    if guess == "learned":
        from paper_2303_05006_amd.train_guess import DEFAULT_OUT
        S.guess_weights(np.load(DEFAULT_OUT))
    torch.cuda.synchronize()
    return S, time.perf_counter() - t0


def march(torch, S, V, lead, K, last, traj, deferred=False, profile=True):
    """Untimed steps 1..lead, timed steps lead+1..lead+K, untimed steps up to
    last, on the resident incident fields V [last][rhs][N_e]; traj (or None)
    receives J of every step.  deferred: the timed steps in one tdbem_march
    call (the same kernels; each step's solver status read once at the end)
    instead of K tdbem_step calls.  Returns (seconds, GMRES iterations of the
    timed steps, phase times)."""
    J = torch.zeros(V.shape[1:], dtype=torch.float64, device="cuda")

    def run(a):
        S.step(V[a - 1], J)
        if traj is not None:
            traj[a - 1].copy_(J)

    for a in range(1, lead + 1):
        run(a)
    torch.cuda.synchronize()
    S.profile(profile)
    iters = []
    out = traj[lead:lead + K] if traj is not None else (
        torch.zeros((K,) + tuple(V.shape[1:]), dtype=torch.float64, device="cuda") if deferred else None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if deferred:
        rc, st, its = S.march(V[lead:lead + K], out, with_iters=True)
        if rc != tdbem_codes()["OK"]:
            raise RuntimeError(f"march returned {rc}")
        iters.extend(int(x) for x in its)
    else:
        for a in range(lead + 1, lead + K + 1):
            run(a)
            iters.append(S.gmres_iters())
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    if deferred:
        J.copy_(out[-1])
    ph = S.phase_times()
    S.profile(False)
    for a in range(lead + K + 1, last + 1):
        run(a)
    torch.cuda.synchronize()
    return el, iters, ph


def tdbem_codes():
    from paper_2303_05006_amd import tdbem
    return {"OK": tdbem.OK}


def kernel_rooflines(info, ph, lead, K, nr, prec_fp64, form, near_mm=False, near_leaf=False):
    """Achieved rates of the M2L and near-field kernels over the timed steps.
    near_mm: the batched near field runs as per-leaf matrix-core products
    (priced by its algorithmic FLOP, 2 per stored coefficient and rhs)."""
    lmax = info["lmax"]
    gates = gate_schedule(info["Mt"], lmax, lead + 1, lead + K)
    m2l_flops = 0.0
    for l in range(2, lmax + 1):
        for a in gates[l]:
            k = a // info["Mt"][l] - 1
            lags = min(info["windows"][l], k + 1)
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
    if t_near > 0 and near_mm:
        near_flops = K * 2.0 * info["near_nnz"] * nr
        kernels["near"] = {"bound": "mfma", "achieved": near_flops / t_near / 1e12, "unit": "TFLOP/s",
                           "peak": (PEAK_FP64 if prec_fp64 else PEAK_FP32) / 1e12, "launches": ph["near"][1],
                           "ms_total": ph["near"][0], "flop_per_launch": near_flops / max(ph["near"][1], 1)}
    elif t_near > 0:
        kernels["near"] = {"bound": "hbm", "achieved": near_bytes / t_near / 1e9, "unit": "GB/s",
                           "peak": PEAK_HBM / 1e9, "launches": ph["near"][1], "ms_total": ph["near"][0],
                           "bytes_per_launch": near_bytes / max(ph["near"][1], 1),
                           "traffic": near_traffic() if (nr == 1 and prec_fp64 and near_leaf) else None}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"]) if kernels else None
    roof = None
    if dom:
        kd = kernels[dom]
        traffic = m2l_traffic(form) if (dom == "m2l" and nr == 1) else None
        roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["achieved"] / kd["peak"], "traffic": traffic}
    return roof, kernels


def rel_l2(a, b):
    return float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt())


def batched_runs(torch, tdbem, lead, K, rtol, single_fp64_steps_per_s, deferred=True):
    """64 incident fields (Fibonacci directions, seeded polarisations) marched
    together: the plain FP64 form and the chosen form (FP32 near values and
    M2L, learned initial guess), timed over K steady-state steps after the
    lead-in; the chosen form's error is taken against the FP64 batch over
    every step marched."""
    from paper_2303_05006_amd.inputs import workload
    w = workload("sphere20480x64", n_rhs=64)
    nr = len(w.pulses)
    last = lead + K
    out = {"workload": f"sphere20480x64: the same sphere, {nr} incident fields, steps {lead + 1}..{last} timed "
                       f"after a {lead}-step lead-in",
           "n_rhs": nr, "steps": K, "lead_in": lead}
    trajs = {}
    for key, form, guess in (("fp64", "fp64", "extrap"), ("chosen", "fp32", "learned")):
        S, setup = make_solver(torch, tdbem, w, form, guess, rtol)
        V = torch.zeros((last, nr, S.ne), dtype=torch.float64, device="cuda")
        for a in range(1, last + 1):
            S.incident(w.pulses, a, V[a - 1])
        traj = torch.zeros((last, nr, S.ne), dtype=torch.float64, device="cuda")
        tuned = S.query_array(tdbem.Q_TUNED, 4, np.int32)
        el, iters, ph = march(torch, S, V, lead, K, last, traj, deferred=deferred)
        near_mm = (int(tuned[0]), int(tuned[1])) == (0, 0)
        roof, kern = kernel_rooflines(S.info(), ph, lead, K, nr, form == "fp64", form, near_mm=near_mm)
        out[key] = {"form": form + (" + learned initial guess" if guess == "learned" else ""),
                    "steps_per_s": K / el, "rhs_steps_per_s": nr * K / el, "ms_per_step": el / K * 1e3,
                    "near_form": "matrix cores, per leaf" if near_mm else "row kernel",
                    "near_leaf_gb": S.info()["near_leaf_bytes"] / 1e9,
                    "gmres_iters_mean": float(np.mean(iters)), "roofline": roof, "kernels": kern,
                    "phase_ms": {k: v[0] for k, v in ph.items()}, "setup_s": setup}
        trajs[key] = traj
        S.close()
        del V
    out["chosen"]["rel_l2_err_vs_fp64"] = rel_l2(trajs["chosen"], trajs["fp64"])
    out["chosen"]["err_over_steps"] = f"1..{last}"
    out["chosen"]["speedup_vs_fp64_batched"] = out["chosen"]["steps_per_s"] / out["fp64"]["steps_per_s"]
    out["chosen"]["rhs_throughput_vs_fp64_single"] = out["chosen"]["rhs_steps_per_s"] / single_fp64_steps_per_s
    del trajs
    torch.cuda.empty_cache()
    return out


def far_study(torch, tdbem):
    """Dense (matrix cores) against Fourier-domain M2L at p = 4, 6, 8: the M2L
    phase per launch over the potentials of a seeded random history (the far
    field's gates of every level), with the dense form's algorithmic FLOP and
    the Fourier form's algorithmic bytes (diagonal products: transformed
    moments and kernels read once per (target, entry, lag), sums written once)
    per launch.  Also the relative difference of the two forms' potentials."""
    from paper_2303_05006_amd.inputs import icosphere, C0
    out = []
    for p, level, cdt, n_hist in ((4, 4, 0.02, 120), (6, 4, 0.02, 120), (8, 3, 0.04, 60)):
        v, f = icosphere(level)
        rng = np.random.default_rng(p)
        hist = torch.tensor(rng.standard_normal((n_hist, 3 * len(f) // 2)), device="cuda")
        pots = {}
        forms = [("dense", tdbem.M2L_AUTO), ("fft", tdbem.M2L_FFT)]
        if p == 4:
            forms.append(("bf16", tdbem.M2L_BF16))
        for name, m2l in forms:
            S = tdbem.Solver(v, f, tdbem.Config(dt=cdt / C0, mode=tdbem.MODE_IFMM, p_s=p, p_t=p, leaf_max=64, m2l=m2l))
            info = S.info()
            o = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
            S.profile(True)
            t0 = time.perf_counter()
            S.potentials(hist, n_hist, o)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ph = S.phase_times()
            S.profile(False)
            pots[name] = o.clone()
            nn, nf = p ** 4, (2 * p) ** 3 * (p + 1)
            work, nl = 0.0, 0
            for l in range(2, info["lmax"] + 1):
                M = info["Mt"][l]
                for a in range(M, n_hist + 1, M):
                    lags = min(info["windows"][l], a // M)
                    nl += 1
                    if name != "fft":
                        work += info["nilist"][l] * lags * 7 * 2.0 * nn * nn
                    else:
                        work += (info["nilist"][l] * lags * (7 + 2) + info["ncells"][l] * 7) * nf * 16.0
            ms = ph["m2l"][0] / max(ph["m2l"][1], 1)
            rate = work / max(ph["m2l"][1], 1) / (ms * 1e-3)
            r = {"p": p, "m2l": name, "triangles": len(f), "c_dt": cdt, "history_steps": n_hist,
                 "m2l_ms_total": ph["m2l"][0], "launches": ph["m2l"][1], "ms_per_launch": ms,
                 "potentials_wall_s": wall, "device_gb": info["device_bytes"] / 1e9}
            if name == "dense":
                r.update({"flop_per_launch": work / max(nl, 1), "achieved_tflops": rate / 1e12,
                          "frac_fp64_mfma": rate / PEAK_FP64})
            elif name == "bf16":
                r.update({"flop_per_launch": work / max(nl, 1), "achieved_tflops": rate / 1e12,
                          "frac_bf16_mfma": rate / PEAK_BF16})
            else:
                r.update({"bytes_per_launch": work / max(nl, 1), "achieved_gbs": rate / 1e9,
                          "frac_hbm": rate / PEAK_HBM})
            out.append(r)
            S.close()
            torch.cuda.empty_cache()
        for r in out[-len(forms):]:
            if r["m2l"] != "dense":
                r["rel_diff_vs_dense"] = float((pots[r["m2l"]] - pots["dense"]).abs().max() /
                                               pots["dense"].abs().max())
            print(json.dumps(r), flush=True)
    return out


def guess_study(torch, tdbem, nt=1000, n_pulses=2):
    """The learned initial guess on a held-out body: the 20480-triangle
    ellipsoid (semi-axes 1, 1, 2 m), c dt = 0.02 m, pulses from seeds the
    training never drew (f0 in [50, 150] MHz), FP64 fast method, one field at a
    time.  Per guess (quadratic extrapolation, the trained network, and a
    network with zero weights as the control): GMRES iterations per step over
    steps 201..nt-1, steps/s over the march, the learned guess's share of steps,
    and the relative l2 difference of the marched current from the
    extrapolation run."""
    from paper_2303_05006_amd.inputs import ellipsoid, random_pulses, C0
    from paper_2303_05006_amd.train_guess import DEFAULT_OUT
    v, f = ellipsoid(5)
    dt = 0.02 / C0
    pulses = random_pulses(n_pulses, seed=7777, r_max=2.0)
    trained = np.load(DEFAULT_OUT)
    out, ref = {}, None
    for name, guess, params in (("extrapolation", tdbem.GUESS_EXTRAP, None),
                                ("learned", tdbem.GUESS_LEARNED, trained),
                                ("zero_weights", tdbem.GUESS_LEARNED, np.zeros_like(trained))):
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, nt=nt, mode=tdbem.MODE_IFMM, gmres_rtol=1e-8, gmres_maxit=60,
                                            guess=guess))
        if params is not None:
            S.guess_weights(params)
        its, el, trajs = [], 0.0, []
        for p in pulses:
            S.reset()
            V = torch.zeros((nt - 1, 1, S.ne), dtype=torch.float64, device="cuda")
            for a in range(1, nt):
                S.incident([p], a, V[a - 1])
            J = torch.zeros_like(V)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st, it = S.march(V, J, with_iters=True)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            its.extend(int(x) for x in it[200:])
            trajs.append(J)
        r = {"gmres_iters_per_step": float(np.mean(its)), "steps_per_s": len(pulses) * (nt - 1) / el}
        if guess == tdbem.GUESS_LEARNED:
            r["learned_guess_taken_steps"] = int(S.guess_used())
            r["of_steps"] = len(pulses) * (nt - 1)
        if ref is None:
            ref = trajs
        else:
            num = sum(float(((a - b) ** 2).sum()) for a, b in zip(trajs, ref))
            den = sum(float((b ** 2).sum()) for b in ref)
            r["rel_l2_current_vs_extrapolation_run"] = math.sqrt(num / den)
        out[name] = r
        S.close()
        del trajs
        torch.cuda.empty_cache()
        print(json.dumps({name: r}), flush=True)
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
    ap.add_argument("--batched-steps", type=int, default=48)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, run one 512 MiB device copy (counter calibration)")
    ap.add_argument("--last", type=int, default=NT, help="steps marched in all (untimed after the timed ones)")
    ap.add_argument("--step-loop", action="store_true",
                    help="time the steps as tdbem_step calls (default: one tdbem_march call for the timed steps)")
    ap.add_argument("--no-compare-loop", action="store_true",
                    help="skip the run that times the same steps issued the other way")
    ap.add_argument("--guess-study", action="store_true",
                    help="only the learned initial guess on the held-out 20480-triangle ellipsoid (JSON lines)")
    ap.add_argument("--far-study", action="store_true",
                    help="only the dense vs Fourier-domain M2L study at p = 4, 6, 8 (JSON lines)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_05006_amd import tdbem
    from paper_2303_05006_amd.inputs import workload, C0

    torch.cuda.set_device(0)
    if args.far_study:
        far_study(torch, tdbem)
        return
    if args.guess_study:
        guess_study(torch, tdbem)
        return
    name = "sphere20480" if args.nrhs == 1 else "sphere20480x64"
    w = workload(name, n_rhs=args.nrhs)
    nr = len(w.pulses)
    chosen = not args.no_chosen and nr == 1 and args.form == "fp64" and args.guess == "extrap"

    S, setup_s = make_solver(torch, tdbem, w, args.form, args.guess, args.rtol)
    info = S.info()
    tuned = S.query_array(tdbem.Q_TUNED, 4, np.int32)
    ne = S.ne
    # the pulse reaches the sphere (radius 1 m) after its delay minus the light time to the centre
    arrival = int(math.ceil((w.pulses[0].delay - 1.0 / C0) / w.dt))
    lead, K = steady_window(args.warmup, args.steps, info["Mt"][2], info["window"], arrival)
    last = max(args.last, lead + K)
    # incident fields of every step resident in HBM before timing
    V = torch.zeros((last, nr, ne), dtype=torch.float64, device="cuda")
    for a in range(1, last + 1):
        S.incident(w.pulses, a, V[a - 1])
    traj = torch.zeros((last, nr, ne), dtype=torch.float64, device="cuda") if chosen else None
    # the timed steps without phase timing (its events cost about 4% of a step)
    el, iters, _ = march(torch, S, V, lead, K, last, traj, deferred=not args.step_loop, profile=False)
    # phase pass: the same steps on a fresh context with the same choices, HIP
    # events around each phase (the kernel rates and phase times below)
    Sp, _ = make_solver(torch, tdbem, w, args.form, args.guess, args.rtol, same_as=tuned)
    elp, _, ph = march(torch, Sp, V, lead, K, lead + K, None, deferred=not args.step_loop)
    Sp.close()
    prec_fp64 = args.form == "fp64"
    roof, kernels = kernel_rooflines(info, ph, lead, K, nr, prec_fp64, args.form,
                                     near_leaf=int(tuned[1]) == 0 and int(tuned[0]) > 0)
    d0 = S.d0_nnz()
    res = {
        "metric": METRIC,
        "value": K / el,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": lead,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: PEC sphere r=1 m, 20480 triangles / {ne} RWG edges, c dt = 0.02 m, "
                               f"IFMM p_s=p_t=4, leaves <= 64 edges, {nr} incident field(s); steps {lead + 1}.."
                               f"{lead + K} of {last} timed after a {lead}-step lead-in (M2L windows of every "
                               f"level full, pulse on the sphere from step {arrival})",
                   "form": args.form, "n_rhs": nr, "gmres_rtol": args.rtol, "guess": args.guess,
                   "requested_steps": args.steps, "requested_warmup": args.warmup},
        "roofline": roof,
        "kernels": kernels,
        "rhs_steps_per_s": nr * K / el,
        "d0_nnz": d0,
        "effective_interactions_per_s": d0 * nr * K / el,
        "near_interactions_per_s": info["near_nnz"] * nr * K / el,
        "phase_ms": {k: v[0] for k, v in ph.items()},
        "phase_launches": {k: v[1] for k, v in ph.items()},
        "phase_pass": {"ms_per_step": elp / K * 1e3,
                       "how": "the timed steps again on a fresh context with HIP events around each phase; "
                              "roofline, kernels and phase_ms come from it"},
        "gmres_iters_mean": float(np.mean(iters)),
        "setup_s": setup_s,
        "hierarchy": {k: info[k] for k in ("lmax", "Mt", "ncells", "nilist", "near_nnz", "near_pairs", "z0_nnz",
                                           "windows")},
        "tuned": dict(zip(("near_lag_steps", "near_pair_blocks", "solve_blocks", "autotuned"),
                          (int(x) for x in tuned))),
        "device_gb": info["device_bytes"] / 1e9,
    }
    S.close()
    if not args.no_compare_loop:
        # the other way of issuing the same timed steps, on a fresh context:
        # K tdbem_step calls (a host wait per step) against one tdbem_march
        Sx, _ = make_solver(torch, tdbem, w, args.form, args.guess, args.rtol, same_as=tuned)
        trx = torch.zeros_like(traj) if traj is not None else None
        elx, itx, _ = march(torch, Sx, V, lead, K, lead + K, trx, deferred=args.step_loop, profile=False)
        Sx.close()
        key = "deferred_march" if args.step_loop else "step_loop"
        res[key] = {"steps_per_s": K / elx, "ms_per_step": elx / K * 1e3,
                    "how": "one tdbem_march call" if args.step_loop else f"{K} tdbem_step calls",
                    "gmres_iters_mean": float(np.mean(itx))}
        if traj is not None:
            res[key]["bitwise_equal_currents"] = bool(torch.equal(trx[:lead + K], traj[:lead + K]))
        del trx
    if not args.no_compare_loop and not args.step_loop:
        # the same timed steps issued from captured HIP graphs (graph = 1) on a
        # fresh context, against the plain launches of the run above
        Sg, _ = make_solver(torch, tdbem, w, args.form, args.guess, args.rtol, same_as=tuned, graph=1)
        trg = torch.zeros_like(traj) if traj is not None else None
        elg, _, _ = march(torch, Sg, V, lead, K, lead + K, trg, deferred=True, profile=False)
        built, refreshed = Sg.query_array(tdbem.Q_GRAPHS, 2, np.int64).tolist()
        Sg.close()
        res["graph_march"] = {"steps_per_s": K / elg, "ms_per_step": elg / K * 1e3,
                              "how": "one tdbem_march call with graph = 1 (plain launches: value)",
                              "graphs_built": built, "graph_refreshes": refreshed}
        if traj is not None:
            res["graph_march"]["bitwise_equal_currents"] = bool(torch.equal(trg[:lead + K], traj[:lead + K]))
        del trg
    if chosen:
        # chosen form on the same incident fields: FP32 near values and M2L
        # products, learned initial guess; error of its march against FP64's
        # over every step to the end of the workload
        S2, setup2 = make_solver(torch, tdbem, w, "fp32", "learned", args.rtol)
        traj32 = torch.zeros_like(traj)
        el2, iters2, _ = march(torch, S2, V, lead, K, last, traj32, deferred=not args.step_loop, profile=False)
        tuned2 = S2.query_array(tdbem.Q_TUNED, 4, np.int32)
        S2p, _ = make_solver(torch, tdbem, w, "fp32", "learned", args.rtol, same_as=tuned2)
        _, _, ph2 = march(torch, S2p, V, lead, K, lead + K, None, deferred=not args.step_loop)
        roof2, kernels2 = kernel_rooflines(S2p.info(), ph2, lead, K, nr, False, "fp32")
        S2p.close()
        dn = ((traj32 - traj) ** 2).sum(dim=(1, 2)).sqrt()
        jn = (traj ** 2).sum(dim=(1, 2)).sqrt()
        res["chosen"] = {"form": "fp32 near values and M2L + learned initial guess", "value": K / el2,
                         "unit": "steps/s", "ms_per_step": el2 / K * 1e3, "speedup_vs_fp64": el / el2,
                         "rel_l2_err_vs_fp64": rel_l2(traj32, traj), "err_over_steps": f"1..{last}",
                         "rel_l2_err_vs_fp64_last100": rel_l2(traj32[-100:], traj[-100:]),
                         "max_step_err_over_peak": float(dn.max() / jn.max()),
                         "roofline": roof2, "kernels": kernels2,
                         "phase_ms": {k: v[0] for k, v in ph2.items()},
                         "gmres_iters_mean": float(np.mean(iters2)), "setup_s": setup2}
        S2.close()
        del traj32
    del V, traj
    torch.cuda.empty_cache()
    if chosen and not args.no_batched:
        _, Kb = steady_window(lead, args.batched_steps, info["Mt"][2], info["window"], arrival)
        res["batched"] = batched_runs(torch, tdbem, lead, Kb, args.rtol, K / el, deferred=not args.step_loop)
    if args.copy_probe:
        res["copy_probe"] = copy_probe(torch)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
