"""Accuracy of the fast method (D1) against the discretised problem (D0).

The direct GPU path computes D0 (it equals the FP64 oracle to 1e-14 on the
parity meshes); the IFMM replaces the far pairs by interpolation (p_s = p_t = 4,
Lagrange), so the difference is interpolation-limited.  Measured here on a
5120-triangle sphere with the benchmark's c dt and pulse, per step (potentials
of a marched history) and for the marched current, as the relative l2 error
sqrt(sum_a |J_a - J_ref,a|^2 / sum_a |J_ref,a|^2) over steps and edges.  The
bounds below are the measured values rounded up (temporal CHI-FD, the default:
2.5e-2 for the potentials, 3.6e-2 for the march; temporal Lagrange: 2.2e-2 and
3.2e-2).  With the causality guard (causal_guard = 1: the interval shrunk so
that no far pair can interact within one interval although basis supports
reach beyond their cells) the error barely moves (1.6e-2 / 2.4e-2): it is the
interpolation's, not the dropped same-interval terms'.  The FP32 form is
measured against the FP64 IFMM on the same march (4.4e-5).
"""
import math
import os

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, gaussian_pulse, C0

NT = 400
CDT = 0.02


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def _march(S, pulse, nt, torch):
    V = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
    out = torch.zeros((nt - 1, S.ne), dtype=torch.float64, device="cuda")
    for a in range(1, nt):
        S.incident([pulse], a, V)
        S.step(V, J)
        out[a - 1] = J
    return out


def _rel(a, b):
    return float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt())


@pytest.fixture(scope="module")
def runs():
    torch = _torch()
    v, f = icosphere(4)
    dt = CDT / C0
    pulse = gaussian_pulse(300e6, 200e6)
    res = {}
    for name, kw in (("direct", dict(mode=tdbem.MODE_DIRECT)), ("ifmm", dict(mode=tdbem.MODE_IFMM)),
                     ("ifmm32", dict(mode=tdbem.MODE_IFMM, precision=tdbem.FP32)),
                     ("guard", dict(mode=tdbem.MODE_IFMM))):
        if name == "guard":
            kw["causal_guard"] = 1
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, nt=NT, gmres_rtol=1e-12, gmres_maxit=100, **kw))
        res[name] = (S, _march(S, pulse, NT, torch))
    yield res
    for S, _ in res.values():
        S.close()


def test_ifmm_potentials_against_direct(runs):
    """History part of the right-hand side for the direct path's own marched
    history, at steps across the pulse."""
    torch = _torch()
    Sd, Jd = runs["direct"]
    for name, bound in (("ifmm", 3e-2), ("guard", 2e-2)):
        Si, _ = runs[name]
        worst = 0.0
        for a in (100, 200, 300, 399):
            hist = Jd[:a - 1].contiguous()
            pd = torch.zeros(Sd.ne, dtype=torch.float64, device="cuda")
            pi = torch.zeros(Sd.ne, dtype=torch.float64, device="cuda")
            Sd.potentials(hist, a - 1, pd)
            Si.potentials(hist, a - 1, pi)
            e = _rel(pi, pd)
            print(f"{name} step {a}: potentials rel l2 {e:.2e}")
            worst = max(worst, e)
        assert worst < bound


def test_ifmm_marched_current_against_direct(runs):
    _, Jd = runs["direct"]
    for name, bound in (("ifmm", 5e-2), ("guard", 3e-2)):
        _, Ji = runs[name]
        e = _rel(Ji, Jd)
        print(f"marched current, {name} vs direct: rel l2 {e:.2e}")
        assert e < bound


def test_fp32_form_marched_current_against_fp64_ifmm(runs):
    _, Ji = runs["ifmm"]
    _, J32 = runs["ifmm32"]
    e = _rel(J32, Ji)
    print(f"marched current, FP32 form vs FP64 IFMM: rel l2 {e:.2e}")
    assert e < 1e-4


def test_precision_forms_on_a_cube():
    """Precision forms on a structured cube of side 2 m (19200 triangles,
    c dt = 0.02 m, 300 / 200 MHz pulse along +z, 400 steps): the marched current
    of the FP32 form and of the BF16 form (bf16 near-field coefficients) against
    the FP64 IFMM.  The cube's finest cells are smaller than its basis
    supports reach, and its march grows after the pulse with cell-sized
    interpolation boxes; the boxes are widened here (box_widen = 1), with
    which the march decays."""
    from paper_2303_05006_amd.inputs import cube
    torch = _torch()
    v, f = cube(40, 2.0)
    dt = CDT / C0
    pulse = gaussian_pulse(300e6, 200e6, r_max=math.sqrt(3.0))
    res = {}
    for name, prec in (("fp64", tdbem.FP64), ("fp32", tdbem.FP32), ("bf16", tdbem.BF16)):
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, nt=NT, mode=tdbem.MODE_IFMM, precision=prec, gmres_rtol=1e-12,
                                            gmres_maxit=200, box_widen=1))
        res[name] = _march(S, pulse, NT, torch)
        S.close()
    e32 = _rel(res["fp32"], res["fp64"])
    e16 = _rel(res["bf16"], res["fp64"])
    print(f"cube 19200 triangles: FP32 form {e32:.2e}, BF16 form {e16:.2e} (relative l2 against FP64)")
    assert e32 < 1e-4
    assert e16 < 1e-2
