"""Learned initial guess of the Z0 solve, through the C ABI.

* the captured features equal the documented definition computed here from
  the marched history, the right-hand side (V minus the potentials) and the
  diagonal of Z0, with an independent 12-nearest-edge search;
* the network's output equals the oracle's forward pass with the bf16
  roundings of the definition (oracle/guess_mlp.py g_bf16), and the plain FP64
  network within the oracle's first-order bound on those roundings;
* zero parameters reproduce the extrapolation exactly;
* the training kernels (loss gradient, Adam step) equal the FP64 oracle;
* the trained parameters do not need more GMRES iterations than the
  extrapolation on a held-out body and held-out pulses.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from oracle import guess_mlp as GM
from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, ellipsoid, gaussian_pulse, random_pulses, C0

WEIGHTS = os.path.join(os.path.dirname(tdbem.__file__), "weights", "guess_mlp_icosphere5120.npy")
# held-out gain the trained network must reach (GMRES iterations per step);
# the committed weights (200 seeded training runs) measured 13.10 -> 12.13
MIN_GAIN = 0.5
DT = 0.5e-9


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def bf16(a):
    """Round-to-nearest-even to bf16, returned as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def neighbours(m):
    """12 nearest edges by midpoint distance (ties by index) and direction signs."""
    mid = 0.5 * (m.xyz[m.edges[:, 0]] + m.xyz[m.edges[:, 1]])
    cen = lambda t: ((m.xyz[m.tri[t, 0]] / 3.0 + m.xyz[m.tri[t, 1]] / 3.0) + m.xyz[m.tri[t, 2]] / 3.0)
    d = cen(m.etri[:, 1]) - cen(m.etri[:, 0])
    nn = np.zeros((m.ne, 12), int)
    sg = np.zeros((m.ne, 12), np.float32)
    idx = np.arange(m.ne)
    for i in range(m.ne):
        dx = mid[:, 0] - mid[i, 0]
        dy = mid[:, 1] - mid[i, 1]
        dz = mid[:, 2] - mid[i, 2]
        r2 = (dx * dx + dy * dy) + dz * dz
        r2[i] = np.inf
        order = np.lexsort((idx, r2))[:12]
        nn[i] = order
        dot = (d[i, 0] * d[order, 0] + d[i, 1] * d[order, 1]) + d[i, 2] * d[order, 2]
        sg[i] = np.where(dot < 0.0, -1.0, 1.0)
    return nn, sg


def features(Js, a, R, Z0, dinv, nn, sg):
    """Unnormalised FP32 features of step a (J^{a-1} is being solved for)."""
    ne = len(dinv)
    f = np.zeros((ne, 116), np.float32)
    edges = np.concatenate([np.arange(ne)[:, None], nn], axis=1)           # [ne, 13]
    signs = np.concatenate([np.ones((ne, 1), np.float32), sg], axis=1)
    for e in range(13):
        for s in range(1, 9):
            b = a - 1 - s
            if b >= 0:
                f[:, 8 * e + s - 1] = signs[:, e] * Js[b][edges[:, e]].astype(np.float32)
    ext = 3.0 * Js[a - 2] - 3.0 * Js[a - 3] + Js[a - 4]
    res = R - Z0 @ ext
    for e in range(12):
        f[:, 104 + e] = signs[:, e] * (dinv[edges[:, e]] * res[edges[:, e]]).astype(np.float32)
    return f


def normalise(f):
    s = np.abs(f).max(axis=1)
    s = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    inv = (np.float32(1.0) / s).astype(np.float32)
    return bf16(f * inv[:, None]), s


@pytest.fixture(scope="module")
def marched():
    torch = _torch()
    v, f = icosphere(2)
    m = O.Mesh(v, f)
    S = tdbem.Solver(v, f, tdbem.Config(dt=DT, mode=tdbem.MODE_DIRECT, gmres_rtol=1e-12, gmres_maxit=100))
    pulse = gaussian_pulse(60e6, 40e6)
    V = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    Vs, Js = [], []
    for a in range(1, 41):
        S.incident([pulse], a, V)
        S.step(V, J)
        Vs.append(V.cpu().numpy().copy())
        Js.append(J.cpu().numpy().copy())
    Z0 = S.near_rows(np.arange(m.ne), 2)[:, :, 1]
    dinv = 1.0 / np.diag(Z0)
    nn, sg = neighbours(m)
    yield m, S, pulse, Vs, Js, Z0, dinv, nn, sg
    S.close()


def test_captured_features_match_definition(marched):
    torch = _torch()
    m, S, pulse, Vs, Js, Z0, dinv, nn, sg = marched
    a = 35                                  # replay steps 1..a-1, capture step a
    S.reset()
    V = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    F = torch.zeros((1, m.ne, 116), dtype=torch.float32, device="cuda")
    A = torch.zeros((1, m.ne, 2), dtype=torch.float64, device="cuda")
    for b in range(1, a + 1):
        S.incident([pulse], b, V)
        if b == a:
            S.guess_capture(F, A)
        S.step(V, J)
    S.guess_capture()
    hist = torch.tensor(np.stack(Js[:a - 1]), device="cuda")
    pot = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    S.potentials(hist, a - 1, pot)
    R = Vs[a - 1] - pot.cpu().numpy()
    x_ref, s_ref = normalise(features(Js, a, R, Z0, dinv, nn, sg))
    x = F[0].cpu().numpy()
    aux = A[0].cpu().numpy()
    assert np.allclose(aux[:, 0], s_ref, rtol=1e-6, atol=0), np.abs(aux[:, 0] / s_ref - 1).max()
    ext = 3.0 * Js[a - 2] - 3.0 * Js[a - 3] + Js[a - 4]
    assert np.abs(aux[:, 1] - ext).max() <= 1e-14 * np.abs(ext).max()
    d = np.abs(x - x_ref)
    print(f"features: {np.mean(d == 0):.4f} identical, max diff {d.max():.2e}")
    # the residual group carries the rounding of Z0 x (summation order): at most
    # one bf16 unit apart, and only on a few features
    assert d.max() <= 2.0 ** -8 and np.mean(d == 0) > 0.99


@pytest.mark.parametrize("zero", [True, False])
def test_network_output_matches_fp64_forward(marched, zero):
    """Each step starts from the learned guess x_L = extrap + s g(x) when its
    residual ||R - Z0 x_L|| is smaller than the extrapolation's, else from the
    extrapolation; g against the FP64 forward, the choice against the residuals
    computed here (R = V - potentials of the step's history, Z0 from the
    library's coefficients)."""
    torch = _torch()
    m, S0, pulse, Vs, Js, Z0, dinv, nn, sg = marched
    v, f = icosphere(2)
    # a huge tolerance makes the solve return its initial guess unchanged
    S = tdbem.Solver(v, f, tdbem.Config(dt=DT, mode=tdbem.MODE_DIRECT, gmres_rtol=1e30,
                                        guess=tdbem.GUESS_LEARNED))
    rng = np.random.default_rng(7)
    # random network plus one path that makes g(x) contain the edge's own scaled
    # residual (feature 104), i.e. a Jacobi step from the extrapolation, so that
    # the learned guess wins the residual comparison on most steps
    W1 = rng.standard_normal((116, 128)) * np.sqrt(2 / 116)
    b1 = rng.standard_normal(128) * 0.1
    W2 = rng.standard_normal((128, 128)) * np.sqrt(2 / 128)
    b2 = rng.standard_normal(128) * 0.1
    w3 = rng.standard_normal(128) / np.sqrt(128) * 1e-3
    W1[:, 0] = 0.0; W1[104, 0] = 1.0; b1[0] = 0.0
    W2[:, 0] = 0.0; W2[0, 0] = 1.0; b2[0] = 0.0
    w3[0] = 2.0
    p = GM.pack(W1, b1, W2, b2, w3, 0.3).astype(np.float32)
    if zero:
        p[:] = 0.0
    S.guess_weights(p)
    V = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    F = torch.zeros((1, m.ne, 116), dtype=torch.float32, device="cuda")
    A = torch.zeros((1, m.ne, 2), dtype=torch.float64, device="cuda")
    S.guess_capture(F, A)
    worst, taken, checked = 0.0, 0, 0
    hist = []
    for a in range(1, 16):
        S.incident([pulse], a, V)
        S.step(V, J)
        x = F[0].cpu().numpy()
        aux = A[0].cpu().numpy()
        Jn = J.cpu().numpy()
        if zero:
            assert np.array_equal(Jn, aux[:, 1])
            hist.append(Jn)
            continue
        pot = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
        if hist:
            S0.potentials(torch.tensor(np.stack(hist), device="cuda"), len(hist), pot)
        R = V.cpu().numpy() - pot.cpu().numpy()
        xe = aux[:, 1]
        p64 = p.astype(np.float64)
        xl = xe + aux[:, 0] * GM.g_bf16(p64, x)
        xp = xe + aux[:, 0] * GM.g(p64, x)                    # plain FP64 network
        bnd = aux[:, 0] * GM.g_bf16_bound(p64, x)
        re, rl = np.linalg.norm(R - Z0 @ xe), np.linalg.norm(R - Z0 @ xl)
        hist.append(Jn)
        if abs(re - rl) <= 1e-6 * re:
            continue                     # too close to call in FP64 rounding
        checked += 1
        if rl < re:
            taken += 1
            err = np.abs(Jn - xl).max() / max(np.abs(xl - xe).max(), 1e-300)
            worst = max(worst, err)
            # FP32 accumulation on top of the bf16 roundings: 1e-5 of the correction
            slack = 1e-5 * np.abs(xl - xe).max()
            assert np.all(np.abs(Jn - xp) <= 1.01 * bnd + slack), np.abs(Jn - xp).max()
        else:
            assert np.array_equal(Jn, xe)
    S.guess_capture()
    if not zero:
        assert S.guess_used() == taken
    S.close()
    print(f"network: learned guess taken in {taken} of {checked} steps, output vs oracle bf16 forward {worst:.2e}")
    assert zero or (checked >= 10 and taken >= 1 and worst < 2e-3)


def _random_params(rng):
    return GM.pack(rng.standard_normal((116, 128)) * np.sqrt(2 / 116), rng.standard_normal(128) * 0.3,
                   rng.standard_normal((128, 128)) * np.sqrt(2 / 128), rng.standard_normal(128) * 0.3,
                   rng.standard_normal(128) / np.sqrt(128), 0.2).astype(np.float32)


@pytest.mark.parametrize("n", [1, 31, 100, 4099])
def test_training_gradient_matches_oracle(n):
    """n spans one partial block, several blocks and a ragged tail."""
    torch = _torch()
    rng = np.random.default_rng(n)
    p = _random_params(rng)
    x = (rng.standard_normal((n, 116)) * 0.5).astype(np.float32)
    y = (rng.standard_normal(n) * 0.1).astype(np.float32)
    P, X, Y = (torch.tensor(a, device="cuda") for a in (p, x, y))
    G = torch.full((GM.NPARAMS,), 7.0, dtype=torch.float32, device="cuda")
    L = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    tdbem.guess_grad(P, X, Y, G, L)
    torch.cuda.synchronize()
    g_ref = GM.grad(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    l_ref = GM.loss(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    g = G.cpu().numpy().astype(np.float64)
    offs = np.cumsum([0, 116 * 128, 128, 128 * 128, 128, 128, 1])
    for name, a, b in zip(["W1", "b1", "W2", "b2", "w3", "b3"], offs[:-1], offs[1:]):
        scale = max(np.abs(g_ref[a:b]).max(), 1e-30)
        err = np.abs(g[a:b] - g_ref[a:b]).max() / scale
        print(f"n={n} {name}: {err:.2e}")
        assert err < 1e-4 if name != "b3" else np.all(g[a:b] == 0.0)
    assert abs(float(L.item()) - l_ref) <= 1e-5 * l_ref


def test_adam_step_matches_oracle():
    torch = _torch()
    rng = np.random.default_rng(9)
    p = rng.standard_normal(GM.NPARAMS).astype(np.float32)
    g = rng.standard_normal(GM.NPARAMS).astype(np.float32)
    m = (rng.standard_normal(GM.NPARAMS) * 0.1).astype(np.float32)
    v = (rng.random(GM.NPARAMS) * 0.01).astype(np.float32)
    P, G, Mt, Vt = (torch.tensor(a, device="cuda") for a in (p, g, m, v))
    tdbem.guess_adam(P, G, Mt, Vt, 5, lr=1e-3)
    torch.cuda.synchronize()
    # the kernel takes its hyperparameters in FP32: give the oracle the same values
    f32 = lambda z: float(np.float32(z))
    q, m2, v2 = GM.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64), v.astype(np.float64), 5,
                        lr=f32(1e-3), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    assert np.allclose(Mt.cpu().numpy(), m2, rtol=1e-5, atol=1e-7)
    assert np.allclose(Vt.cpu().numpy(), v2, rtol=1e-5, atol=1e-9)
    assert np.abs(P.cpu().numpy() - q).max() <= 1e-5 * 1e-3 + 1e-6 * np.abs(q).max()


def test_trained_guess_reduces_iterations_on_a_held_out_body():
    """Held out: an ellipsoid (semi-axes 1, 1, 2 m; 5120 triangles) and pulses
    from seeds the training never drew.  The trained network must save GMRES
    iterations against the extrapolation and against a zero-weight network
    (the control: its correction is zero, so the residual judge falls back to
    the extrapolation and the counts match), and its guess must be taken in a
    real share of the steps."""
    torch = _torch()
    assert os.path.exists(WEIGHTS), f"{WEIGHTS} missing: run python -m paper_2303_05006_amd.train_guess"
    params = np.load(WEIGHTS)
    v, f = ellipsoid(4)
    dt = 0.02 / C0
    pulses = random_pulses(2, seed=1000)
    res, used = {}, {}
    for name, guess, w in (("extrap", tdbem.GUESS_EXTRAP, None), ("learned", tdbem.GUESS_LEARNED, params),
                           ("zero", tdbem.GUESS_LEARNED, np.zeros_like(params))):
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_IFMM, gmres_rtol=1e-8, guess=guess))
        if w is not None:
            S.guess_weights(w)
        it = []
        for p in pulses:
            S.reset()
            V = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
            J = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
            for a in range(1, 700):
                S.incident([p], a, V)
                S.step(V, J)
                if a > 200:
                    it.append(S.gmres_iters())
        res[name] = float(np.mean(it))
        if guess == tdbem.GUESS_LEARNED:
            used[name] = S.guess_used()
        S.close()
    print(f"GMRES iterations per step: extrapolation {res['extrap']:.2f}, learned {res['learned']:.2f}, "
          f"zero-weight control {res['zero']:.2f} (learned guess taken in {used['learned']} of {2 * 699} steps)")
    assert abs(res["zero"] - res["extrap"]) < 0.02
    assert res["learned"] <= res["extrap"] - MIN_GAIN
    assert res["learned"] <= res["zero"] - MIN_GAIN
    assert used["learned"] >= 700


@pytest.mark.parametrize("prec,tol", [(tdbem.FP64, 1e-9), (tdbem.FP32, 1e-5)])
def test_learned_guess_batched_equals_single_runs(prec, tol):
    """Three incident fields marched in one batch with the learned guess against
    three single runs: the features, the network and the residual judge act
    per right-hand side, so every column reaches the same solution (both solve
    Z0 to 1e-12).  In FP64 the columns agree to the solver tolerance.  The FP32
    form (the chosen configuration) evaluates its batched M2L with another
    kernel and summation order than a single field, and the march amplifies
    that FP32 rounding (6.6e-7 measured)."""
    torch = _torch()
    params = np.load(WEIGHTS)
    v, f = icosphere(3)
    dt = 0.04 / C0
    pulses = [gaussian_pulse(150e6, 100e6, k=(np.sin(0.7 * i), np.cos(0.7 * i), 0.2)) for i in range(3)]
    cfg = dict(dt=dt, mode=tdbem.MODE_IFMM, precision=prec, gmres_rtol=1e-12, gmres_maxit=200,
               guess=tdbem.GUESS_LEARNED)
    nt = 120
    B = tdbem.Solver(v, f, tdbem.Config(n_rhs=3, **cfg))
    B.guess_weights(params)
    V = torch.zeros((3, B.ne), dtype=torch.float64, device="cuda")
    J = torch.zeros((3, B.ne), dtype=torch.float64, device="cuda")
    out = torch.zeros((nt - 1, 3, B.ne), dtype=torch.float64, device="cuda")
    for a in range(1, nt):
        B.incident(pulses, a, V)
        B.step(V, J)
        out[a - 1] = J
    used_b = B.guess_used()
    B.close()
    S = tdbem.Solver(v, f, tdbem.Config(**cfg))
    S.guess_weights(params)
    for r, p in enumerate(pulses):
        S.reset()
        V1 = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
        J1 = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
        ref = torch.zeros((nt - 1, S.ne), dtype=torch.float64, device="cuda")
        for a in range(1, nt):
            S.incident([p], a, V1)
            S.step(V1, J1)
            ref[a - 1] = J1
        rel = float(((out[:, r] - ref) ** 2).sum().sqrt() / (ref ** 2).sum().sqrt())
        print(f"rhs {r}: batched vs single rel l2 {rel:.2e}")
        assert rel < tol
    S.close()
    print(f"learned guess taken in {used_b} of {3 * (nt - 1)} (step, rhs) solves of the batch")
    assert used_b > 0
