"""Edge cases and error paths of the C ABI (no case here faults or hangs: every
invalid input is rejected on the host before any launch).

* empty history: the potentials of step 1 are zero;
* invalid configurations and meshes: EINVAL with a message;
* a time hierarchy without a step per finest interval: EBREAKDOWN;
* 65 right-hand sides (one full group of 64 and a ragged group of 1) against
  single runs, in both precisions' kernels;
* the learned guess: wrong parameter count, missing parameters, empty batch.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, gaussian_pulse, C0

CDT = 0.078


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def _solver(**kw):
    v, f = icosphere(2)
    base = dict(dt=CDT / C0, mode=tdbem.MODE_IFMM, leaf_max=6, gmres_rtol=1e-12, gmres_maxit=200)
    base.update(kw)
    return tdbem.Solver(v, f, tdbem.Config(**base))


def test_empty_history_gives_zero_potentials():
    torch = _torch()
    for mode in (tdbem.MODE_IFMM, tdbem.MODE_DIRECT):
        S = _solver(mode=mode)
        out = torch.full((S.ne,), 7.0, dtype=torch.float64, device="cuda")
        S.potentials(None, 0, out)
        assert torch.count_nonzero(out).item() == 0
        S.close()


@pytest.mark.parametrize("bad", [dict(dt=0.0), dict(dt=-1e-9), dict(precision=7), dict(mode=5), dict(interp=9),
                                 dict(n_rhs=0), dict(leaf_max=0)])
def test_invalid_config_is_rejected(bad):
    _torch()
    with pytest.raises(tdbem.TdbemError) as e:
        _solver(**bad)
    assert e.value.code == tdbem.EINVAL


def test_open_or_broken_meshes_are_rejected():
    _torch()
    v, f = icosphere(1)
    cfg = tdbem.Config(dt=0.25e-9, mode=tdbem.MODE_DIRECT)
    for tris in (f[1:], np.concatenate([f[:1, ::-1], f[1:]]), np.where(f == 3, 200, f)):
        with pytest.raises(tdbem.TdbemError) as e:
            tdbem.Solver(v, tris, cfg)
        assert e.value.code == tdbem.EINVAL, e.value


def test_time_hierarchy_breakdown():
    """c dt larger than the finest cell side: no step per interval (M_t = 0,
    Remark 1) is refused in IFMM mode; the direct path accepts it.  One step
    per interval is accepted (the window grows by the intervals the truncated
    differences reach: 9 + 3 at the finest level)."""
    _torch()
    v, f = icosphere(2)
    with pytest.raises(tdbem.TdbemError) as e:
        tdbem.Solver(v, f, tdbem.Config(dt=0.3 / C0, mode=tdbem.MODE_IFMM, leaf_max=6))
    assert e.value.code == tdbem.EBREAKDOWN
    tdbem.Solver(v, f, tdbem.Config(dt=0.3 / C0, mode=tdbem.MODE_DIRECT)).close()
    S = tdbem.Solver(v, f, tdbem.Config(dt=0.2 / C0, mode=tdbem.MODE_IFMM, leaf_max=6))
    info = S.info()
    assert info["Mt"][3] == 1 and info["windows"][3] == 12 and info["windows"][2] == 11
    S.close()


@pytest.mark.parametrize("prec", [tdbem.FP64, tdbem.FP32])
def test_ragged_rhs_batch_of_65(prec):
    torch = _torch()
    nr = 65
    B = _solver(n_rhs=nr, precision=prec)
    S = _solver(precision=prec)
    n_hist = 40
    rng = np.random.default_rng(65)
    hist = rng.standard_normal((n_hist, nr, B.ne))
    out = torch.zeros((nr, B.ne), dtype=torch.float64, device="cuda")
    B.potentials(torch.tensor(hist, device="cuda"), n_hist, out)
    tol = 1e-12 if prec == tdbem.FP64 else 2e-3
    for r in (0, 31, 63, 64):
        o1 = torch.zeros(B.ne, dtype=torch.float64, device="cuda")
        S.potentials(torch.tensor(np.ascontiguousarray(hist[:, r]), device="cuda"), n_hist, o1)
        ref = o1.cpu().numpy()
        rel = np.abs(out[r].cpu().numpy() - ref).max() / np.abs(ref).max()
        assert rel < tol, (r, rel)
    # one marched step of all 65 fields
    V = torch.zeros((nr, B.ne), dtype=torch.float64, device="cuda")
    J = torch.zeros((nr, B.ne), dtype=torch.float64, device="cuda")
    B.reset()
    pulses = [gaussian_pulse(150e6, 100e6, k=(np.cos(0.1 * i), np.sin(0.1 * i), 0.3)) for i in range(nr)]
    for a in range(1, 6):
        B.incident(pulses, a, V)
        B.step(V, J)
    assert torch.isfinite(J).all()
    B.close()
    S.close()


def test_guess_api_misuse():
    torch = _torch()
    S = _solver(guess=tdbem.GUESS_LEARNED)
    with pytest.raises(tdbem.TdbemError) as e:
        S.guess_weights(np.zeros(10, np.float32))
    assert e.value.code == tdbem.EINVAL
    bad = np.zeros(tdbem.GUESS_NPARAMS, np.float32)
    bad[5] = np.nan
    with pytest.raises(tdbem.TdbemError):
        S.guess_weights(bad)
    V = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
    S.incident([gaussian_pulse(150e6, 100e6)], 1, V)
    with pytest.raises(tdbem.TdbemError) as e:
        S.step(V, J)                     # no parameters loaded
    assert e.value.code == tdbem.EINVAL
    S.close()
    P = torch.zeros(tdbem.GUESS_NPARAMS, dtype=torch.float32, device="cuda")
    X = torch.zeros((0, 116), dtype=torch.float32, device="cuda")
    Y = torch.zeros(0, dtype=torch.float32, device="cuda")
    G = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(tdbem.TdbemError):
        tdbem.guess_grad(P, X, Y, G, L)
