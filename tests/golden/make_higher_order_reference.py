"""Writes the stored oracle potentials for the p = 6 and p = 8 far-field
parity tests (tests/golden/higher_order_reference.npz).  Calls only oracle/:
O1's J-form coefficients on the near pairs plus O2's far field (all earlier
intervals) for a seeded random current history.  Run from the repository root:
    python tests/golden/make_higher_order_reference.py
The cases (mesh, c dt, leaf size, order, history length, seed) are listed in
CASES and re-read by the test, which regenerates the same history."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# name: (icosphere level, c dt [m], leaf_max, p, history steps, seed)
CASES = {"p6": (2, 0.078, 6, 6, 30, 606), "p8": (2, 0.078, 100000, 8, 13, 808)}
OUT = os.path.join(HERE, "higher_order_reference.npz")


def history(ne, n_hist, seed):
    """The seeded random current history the test marches in (J^0..J^{n-1})."""
    return np.random.default_rng(seed).standard_normal((n_hist, ne))


def reference(name):
    from oracle import oracle as O
    from oracle.constants import C0, EPS0, MU0
    from oracle.ifmm import IFMM
    from paper_2303_05006_amd.inputs import icosphere
    lev, cdt, leaf, p, n_hist, seed = CASES[name]
    v, f = icosphere(lev)
    m = O.Mesh(v, f)
    dt = cdt / C0
    F = IFMM(m, dt, 1.0, C0 / 2, EPS0, MU0, p_s=p, p_t=p, leaf_max=leaf, interp_t="chi")
    hist = history(m.ne, n_hist, seed)
    a = n_hist + 1
    near = np.zeros((m.ne, m.ne), bool)
    for i, j in F.H.near_pairs():
        near[i, j] = True
    Z = O.zrows(m, np.arange(m.ne), cdt, 1.0, C0 / 2, G=O.max_lag(m, cdt) + 1)
    pot = np.zeros(m.ne)
    for g in range(2, Z.shape[2]):
        if 0 <= a - g < n_hist:
            pot += (Z[:, :, g] * near) @ hist[a - g]
    far = F.far_history(hist)[a - 1]
    return pot + far, far, np.array(F.H.Mt)


if __name__ == "__main__":
    out = {}
    for name in CASES:
        tot, far, Mt = reference(name)
        out[name + "_potentials"] = tot
        out[name + "_far"] = far
        out[name + "_Mt"] = Mt
        print(name, np.abs(far).max(), np.abs(tot).max())
    np.savez_compressed(OUT, **out)
