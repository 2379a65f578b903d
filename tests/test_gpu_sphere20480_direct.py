"""The fast method against the direct method on the benchmark sphere itself
(20480 triangles, 30720 RWG edges, c dt = 0.02 m, the benchmark's pulse),
through the C ABI.

The direct path stores every pair's exact J-form coefficients (about 5.3e9
values, 42 GB in FP64, and as many again while the jagged-diagonal store is
built; set-up takes a few minutes) and computes the discretised problem D0;
the fast method (p_s = p_t = 4, leaves of at most 64 edges) computes D1.  Both
march the 1000 steps of the workload; the relative l2 difference of the
currents over all steps and edges is the interpolation-limited error at this
size (3.6e-2 on the 5120-triangle sphere, test_gpu_accuracy.py).

Takes about five minutes on one MI355X (direct set-up 278 s, 58 GB of
device memory): run with TDBEM_LARGE_TESTS=1.
"""
import os

import pytest

pytestmark = pytest.mark.gpu

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import workload

if os.environ.get("TDBEM_LARGE_TESTS") != "1":
    pytest.skip("all-pairs direct method on 30720 edges (about six minutes): set TDBEM_LARGE_TESTS=1",
                allow_module_level=True)


def _march(S, w, torch, name):
    V = torch.zeros((w.nt - 1, S.ne), dtype=torch.float64, device="cuda")
    for a in range(1, w.nt):
        S.incident(w.pulses, a, V[a - 1])
    J = torch.zeros_like(V)
    for k0 in range(0, w.nt - 1, 100):
        k1 = min(w.nt - 1, k0 + 100)
        rc, st = S.march(V[k0:k1], J[k0:k1])
        assert rc == tdbem.OK, (name, k0, rc)
        print(f"{name}: steps {k0 + 1}..{k1} marched", flush=True)
    return J


def test_sphere20480_fast_against_direct():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    os.environ["TDBEM_TRACE"] = "1"        # set-up progress on stderr
    w = workload("sphere20480")
    common = dict(dt=w.dt, nt=w.nt, theta=w.theta, zeta=w.zeta, gmres_rtol=1e-10, gmres_maxit=200)
    D = tdbem.Solver(w.verts, w.tris, tdbem.Config(mode=tdbem.MODE_DIRECT, **common))
    print(f"direct: set up in {D.info()['setup_ms'] / 1e3:.0f} s, {D.info()['device_bytes'] / 1e9:.1f} GB, "
          f"{D.info()['near_nnz']} stored coefficients", flush=True)
    Jd = _march(D, w, torch, "direct")
    D.close()
    torch.cuda.empty_cache()
    F = tdbem.Solver(w.verts, w.tris, tdbem.Config(mode=tdbem.MODE_IFMM, leaf_max=w.leaf_max, **common))
    Jf = _march(F, w, torch, "fast")
    F.close()
    rel = float(((Jf - Jd) ** 2).sum().sqrt() / (Jd ** 2).sum().sqrt())
    dn = ((Jf - Jd) ** 2).sum(dim=1).sqrt()
    peak = float((Jd ** 2).sum(dim=1).sqrt().max())
    print(f"fast against direct, 20480 triangles, steps 1..{w.nt - 1}: relative l2 {rel:.3e}, "
          f"largest step error / peak {float(dn.max()) / peak:.3e}", flush=True)
    # measured: 3.57e-2 (largest step error 4.3e-2 of the peak), as on the
    # 5120-triangle sphere: the interpolation's error does not grow with N
    assert rel < 4e-2
