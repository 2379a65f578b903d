"""The allocation-free step (tdbem_step_noalloc) through the C ABI.

Its solve takes the Z0 GMRES workspace, status and barrier words from the
library's static array instead of the context's allocations.  Checked against
tdbem_step on the same inputs, to the bar of the direct-march parity tests:

* two contexts in a row on the same device, the second with a smaller system
  (fewer edges and right-hand sides), so the second call reuses the array the
  first left behind;
* a system too large for the array is refused with TDBEM_EINVAL before any
  work, and the host-driven solver is refused too.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, gaussian_pulse, C0


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def _march_both(level, nr, mode, nt):
    torch = _torch()
    v, f = icosphere(level)
    dt = 0.078 / C0 if mode == tdbem.MODE_IFMM else 0.25e-9
    cfg = dict(dt=dt, mode=mode, n_rhs=nr, leaf_max=6, gmres_rtol=1e-12, gmres_maxit=200)
    A = tdbem.Solver(v, f, tdbem.Config(**cfg))
    B = tdbem.Solver(v, f, tdbem.Config(**cfg))
    pulses = [gaussian_pulse(150e6 + 20e6 * r, 100e6) for r in range(nr)]
    shape = (A.ne,) if nr == 1 else (nr, A.ne)
    V = torch.zeros(shape, dtype=torch.float64, device="cuda")
    Ja = torch.zeros(shape, dtype=torch.float64, device="cuda")
    Jb = torch.zeros(shape, dtype=torch.float64, device="cuda")
    worst = 0.0
    for a in range(1, nt):
        A.incident(pulses, a, V)
        A.step(V, Ja)
        B.step_noalloc(V, Jb)
        scale = float(Ja.abs().max())
        if scale > 0:
            worst = max(worst, float((Ja - Jb).abs().max()) / scale)
    A.close()
    B.close()
    return worst


def test_noalloc_step_matches_step_on_two_calls_second_smaller():
    big = _march_both(2, 3, tdbem.MODE_IFMM, 60)          # 480 edges, 3 rhs
    small = _march_both(1, 1, tdbem.MODE_DIRECT, 60)      # 120 edges, 1 rhs
    print(f"allocation-free vs allocating step: {big:.2e} (480 edges, 3 rhs), {small:.2e} (120 edges, 1 rhs)")
    # the same kernels on the same inputs: identical up to the order of the
    # solve's block reductions, which does not depend on the buffer
    assert big < 1e-12 and small < 1e-12


def test_noalloc_step_refuses_what_does_not_fit():
    torch = _torch()
    v, f = icosphere(3)                                     # 1920 edges
    S = tdbem.Solver(v, f, tdbem.Config(dt=0.25e-9, mode=tdbem.MODE_DIRECT, n_rhs=32, gmres_rtol=1e-10))
    V = torch.zeros((32, S.ne), dtype=torch.float64, device="cuda")
    J = torch.zeros_like(V)
    with pytest.raises(tdbem.TdbemError) as e:             # 32 x 1920 x 35 doubles > 16 MiB
        S.step_noalloc(V, J)
    assert e.value.code == tdbem.EINVAL
    S.close()
    v, f = icosphere(1)
    H = tdbem.Solver(v, f, tdbem.Config(dt=0.25e-9, mode=tdbem.MODE_DIRECT, solver=tdbem.SOLVER_HOST))
    V = torch.zeros(H.ne, dtype=torch.float64, device="cuda")
    with pytest.raises(tdbem.TdbemError) as e:
        H.step_noalloc(V, torch.zeros_like(V))
    assert e.value.code == tdbem.EINVAL
    H.close()
