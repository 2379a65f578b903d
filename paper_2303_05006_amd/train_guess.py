"""Training of the learned initial guess of the Z0 solve.

The network and its features are defined in include/tdbem.h (tdbem_guess_*).
Training data come from the library itself: marching runs with feature capture
switched on record, for every step and edge, the normalised features x, the
scale s and the extrapolation; the target is the solved current, as the
correction y = (J - extrapolation) / s.  The odd network g(x) = (o(x) - o(-x)) / 2
is fitted to y by Adam in FP32 with the library's own training kernels
(tdbem_guess_grad, tdbem_guess_adam; torch only holds the buffers); the library
rounds W1 and W2 to bf16 when the parameters are loaded for inference.

python -m paper_2303_05006_amd.train_guess [--runs 24] [--rhs 8] [--nt 1000] [--out FILE]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "guess_mlp_icosphere5120.npy")


def collect(S, pulses, nt, first, frac, gen, torch):
    """March one batch of pulses; return sampled (features, target) on the GPU."""
    from . import tdbem
    ne, nr = S.ne, len(pulses)
    V = torch.zeros((nr, ne), dtype=torch.float64, device="cuda")
    J = torch.zeros((nr, ne), dtype=torch.float64, device="cuda")
    F = torch.zeros((nr, ne, tdbem.GUESS_NFEAT), dtype=torch.float32, device="cuda")
    A = torch.zeros((nr, ne, 2), dtype=torch.float64, device="cuda")
    S.reset()
    xs, ys = [], []
    nsamp = max(1, int(frac * nr * ne))
    for a in range(1, nt):
        S.incident(pulses, a, V)
        if a >= first:
            S.guess_capture(F, A)
        S.step(V, J)
        if a >= first:
            S.guess_capture()
            idx = torch.randint(0, nr * ne, (nsamp,), device="cuda", generator=gen)
            f = F.reshape(nr * ne, -1)[idx]
            aux = A.reshape(nr * ne, 2)[idx]
            y = (J.reshape(-1)[idx] - aux[:, 1]) / aux[:, 0]
            xs.append(f)
            ys.append(y.float())
    return torch.cat(xs), torch.cat(ys)


def init_params(seed):
    """He-initialised W1, W2, zero biases and a zero last layer (so that the
    untrained network reproduces the extrapolation)."""
    from . import tdbem
    rng = np.random.default_rng(seed)
    nf, nh = tdbem.GUESS_NFEAT, tdbem.GUESS_NHIDDEN
    p = np.concatenate([rng.standard_normal(nf * nh) * np.sqrt(2.0 / nf), np.zeros(nh),
                        rng.standard_normal(nh * nh) * np.sqrt(2.0 / nh), np.zeros(nh), np.zeros(nh), [0.0]])
    return p.astype(np.float32)


def train(X, Y, torch, epochs=4, batch=8192, lr=1e-3, seed=0, log=print):
    """Adam with a cosine learning-rate schedule; gradients and updates run in
    the library's training kernels (torch only holds the buffers)."""
    from . import tdbem
    P = torch.tensor(init_params(seed), device="cuda")
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed + 1)
    var = float(Y.var())
    # fit y / sigma (unit variance); g is linear in (w3, b3), so scaling them by
    # sigma afterwards gives the network for y itself
    sigma = max(var ** 0.5, 1e-30)
    Y = (Y / sigma).contiguous()
    nb = (n + batch - 1) // batch
    total = epochs * nb
    t = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot = torch.zeros(1, dtype=torch.float64, device="cuda")
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            Xb = X[idx].contiguous()
            Yb = Y[idx].contiguous()
            tdbem.guess_grad(P, Xb, Yb, G, L)
            t += 1
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / total))
            tdbem.guess_adam(P, G, M, V, t, lr=rate)
            tot += L.double() * len(idx)
        log(f"epoch {ep}: mse {float(tot) / n * var:.3e} (target variance {var:.3e})")
    p = P.cpu().numpy()
    nf, nh = tdbem.GUESS_NFEAT, tdbem.GUESS_NHIDDEN
    o = nf * nh + nh + nh * nh + nh
    p[o:] *= sigma                  # w3 and b3
    return p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=3, help="solver runs (each marches --rhs pulses at once)")
    ap.add_argument("--rhs", type=int, default=8)
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--first", type=int, default=100, help="first captured step")
    ap.add_argument("--frac", type=float, default=0.1, help="fraction of (edge, rhs) items sampled per step")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()

    import torch
    from . import tdbem
    from .inputs import icosphere, random_pulses, C0

    torch.cuda.set_device(0)
    v, f = icosphere(4)                  # 5120 triangles, radius 1 m
    dt = 0.02 / C0
    S = tdbem.Solver(v, f, tdbem.Config(dt=dt, nt=args.nt, mode=tdbem.MODE_IFMM, n_rhs=args.rhs,
                                        gmres_rtol=1e-8, gmres_maxit=60))
    gen = torch.Generator(device="cuda").manual_seed(args.seed)
    xs, ys = [], []
    t0 = time.time()
    for run in range(args.runs):
        pulses = random_pulses(args.rhs, seed=args.seed * 1000 + run)
        x, y = collect(S, pulses, args.nt, args.first, args.frac, gen, torch)
        xs.append(x); ys.append(y)
        print(f"run {run}: {x.shape[0]} samples ({time.time() - t0:.1f} s)", flush=True)
    S.close()
    X, Y = torch.cat(xs), torch.cat(ys)
    params = train(X, Y, torch, epochs=args.epochs, seed=args.seed, log=lambda s: print(s, flush=True))
    assert params.size == tdbem.GUESS_NPARAMS
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    print(f"saved {args.out} ({params.size} parameters, {time.time() - t0:.1f} s)")


if __name__ == "__main__":
    sys.exit(main())
