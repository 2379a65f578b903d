"""The precision forms at the size of the precision workload: a PEC cube of
side 2 m, 83 x 83 squares per face (82668 triangles, 124002 edges), c dt =
0.015 m, 2000 steps, modulated Gaussian 300 / 200 MHz along +z polarised
along x, leaves of at most 128 edges (l_max = 5, M_t(5) = 4), interpolation
boxes widened by the basis supports' reach (the cube's finest cells are not
much larger than its edges' supports).

The FP64 fast method is the reference (no direct solution exists at this
size).  Per form, FP32 (near coefficients and M2L operator / moments in FP32
on the matrix cores), BF16 (near coefficients in bf16 with FP64 sums, the FP32
M2L) and the bf16 M2L (operator and moments in bf16 on the matrix cores with
FP32 accumulation, FP64 near field):

* the relative l2 error of the marched current over all steps and edges;
* the relative l2 error of the far field: the radiation integral of dJ/dt,
  F(r, t) = sum over triangles of A_T (I - r r) dJ/dt(x_T, t + r.x_T / c),
  over 26 directions (the cube's face, edge and corner directions) and all
  steps (a post-processor of this project, not in the paper).

Takes about three minutes on one MI355X: run with TDBEM_LARGE_TESTS=1.
"""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import cube, gaussian_pulse, C0

N_FACE, CDT, NT = 83, 0.015, 2000
N_PHYS = 1000      # steps of the physical response: the pulse has left the cube and the current fallen
                   # below 1e-3 of its peak by about step 900; the FP64 fast march grows again from
                   # about step 1000 on this mesh (x1.6 per 100 steps), and the forms are compared
                   # both over the response and over all steps

if os.environ.get("TDBEM_LARGE_TESTS") != "1":
    pytest.skip("82668-triangle cube over 2000 steps (about 3 minutes): set TDBEM_LARGE_TESTS=1",
                allow_module_level=True)


def _directions():
    d = [np.array(v, float) for v in
         [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1) if (i, j, k) != (0, 0, 0)]]
    return np.array([v / np.linalg.norm(v) for v in d])


class FarField:
    """Radiation integral of dJ/dt from the RWG currents at triangle centroids
    (linear interpolation in time between steps)."""

    def __init__(self, v, f, torch):
        v = np.asarray(v, float)
        f = np.asarray(f, np.int64)
        # the library's RWG convention: T+ traverses the edge from its lower to
        # its higher vertex index, T- the other way; edges sorted by (lo, hi)
        e = {}
        for t, tri in enumerate(f):
            for k in range(3):
                u, w, o = int(tri[k]), int(tri[(k + 1) % 3]), int(tri[(k + 2) % 3])
                key = (min(u, w), max(u, w))
                e.setdefault(key, [None, None])[0 if u < w else 1] = (t, o)
        edges = sorted(e)
        self.nt = len(f)
        cen = v[f].mean(axis=1)
        area = 0.5 * np.linalg.norm(np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]), axis=1)
        rows, cols, vals = [], [], []
        for n, key in enumerate(edges):
            L = np.linalg.norm(v[key[0]] - v[key[1]])
            (t0, o0), (t1, o1) = e[key]
            # RWG at the centroid: (L / 2A)(x - o) on T+, -(L / 2A)(x - o) on T-
            for t, o, s in ((t0, o0, 1.0), (t1, o1, -1.0)):
                fv = s * L / (2 * area[t]) * (cen[t] - v[o])
                for c in range(3):
                    rows.append(3 * t + c)
                    cols.append(n)
                    vals.append(fv[c] * area[t])
        idx = torch.tensor(np.array([rows, cols]), dtype=torch.int64)
        self.B = torch.sparse_coo_tensor(idx, torch.tensor(np.array(vals)), (3 * len(f), len(edges))).to("cuda")
        self.cen = torch.tensor(cen, device="cuda")

    def __call__(self, J, dt, torch):
        """J [steps][edges] on the device -> F [directions][steps][3]."""
        JT = (self.B @ J.T).T.reshape(J.shape[0], self.nt, 3)       # A_T J(x_T) per step
        dJ = torch.zeros_like(JT)
        dJ[1:] = (JT[1:] - JT[:-1]) / dt
        out = []
        for r in _directions():
            rr = torch.tensor(r, device="cuda")
            shift = (self.cen @ rr) / (C0 * dt)                      # steps of advance per triangle
            t = torch.arange(J.shape[0], device="cuda", dtype=torch.float64)[:, None] + shift[None, :]
            i0 = t.floor().clamp(0, J.shape[0] - 2).long()
            w = (t - i0).clamp(0, 1)[..., None]
            tri = torch.arange(self.nt, device="cuda")[None, :].expand_as(i0)
            g = (1 - w) * dJ[i0, tri] + w * dJ[i0 + 1, tri]
            s = g.sum(dim=1)
            out.append(s - (s @ rr)[:, None] * rr[None, :])
        return torch.stack(out)


def test_precision_forms_on_the_82668_triangle_cube():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    v, f = cube(N_FACE, 2.0)
    dt = CDT / C0
    pulse = gaussian_pulse(300e6, 200e6, r_max=math.sqrt(3.0))
    res = {}
    forms = (("fp64", dict(precision=tdbem.FP64)), ("fp32", dict(precision=tdbem.FP32)),
             ("bf16", dict(precision=tdbem.BF16)), ("bf16_m2l", dict(m2l=tdbem.M2L_BF16)))
    for name, kw in forms:
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, nt=NT, mode=tdbem.MODE_IFMM, leaf_max=128, gmres_rtol=1e-10,
                                            gmres_maxit=200, box_widen=1, growth_limit=1e6, **kw))
        info = S.info()
        V = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
        J = torch.zeros(S.ne, dtype=torch.float64, device="cuda")
        out = torch.zeros((NT - 1, S.ne), dtype=torch.float64, device="cuda")
        first_bad = None
        for a in range(1, NT):
            S.incident([pulse], a, V)
            rc = S.step_rc(V, J)
            if rc != tdbem.OK and first_bad is None:
                first_bad = (a, rc)
            out[a - 1] = J
        print(f"{name}: first step not OK: {first_bad}", flush=True)
        if name != "bf16_m2l":
            assert first_bad is None
        torch.cuda.synchronize()
        res[name] = out
        print(f"{name}: l_max {info['lmax']}, M_t {info['Mt']}, windows {info['windows']}, "
              f"peak |J| {float(out.abs().max()):.3e}, |J| at the end / peak {float(out[-1].abs().max() / out.abs().max()):.2e}",
              flush=True)
        S.close()
    ff = FarField(v, f, torch)
    F = {k: ff(res[k], dt, torch) for k in res}
    env = res["fp64"].abs().amax(dim=1).cpu().numpy()
    env = [float(env[i:i + 100].max() / env.max()) for i in range(0, NT - 1, 100)]
    print("fp64 max |J| / peak per 100 steps: " + " ".join(f"{x:.1e}" for x in env), flush=True)

    def rel(a, b):
        return float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt())

    errs = {}
    for name in ("fp32", "bf16", "bf16_m2l"):
        e = (rel(res[name][:N_PHYS], res["fp64"][:N_PHYS]), rel(F[name][:, :N_PHYS], F["fp64"][:, :N_PHYS]),
             rel(res[name], res["fp64"]), rel(F[name], F["fp64"]))
        errs[name] = e
        print(f"{name} against fp64: steps 1..{N_PHYS}: current {e[0]:.3e}, far field {e[1]:.3e}; "
              f"steps 1..{NT - 1}: current {e[2]:.3e}, far field {e[3]:.3e}", flush=True)
    # measured over the response: FP32 1.7e-4 (current) and 1.7e-5 (far field);
    # the BF16 form 2.6e-2 and 1.3e-2 (its march grows earlier); the bf16 M2L
    # diverges (its amplified rounding, about 1 already on the potentials)
    assert errs["fp32"][0] < 3e-4 and errs["fp32"][1] < 5e-5
    assert errs["bf16"][0] < 5e-2 and errs["bf16"][1] < 3e-2
