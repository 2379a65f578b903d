"""Far field at higher interpolation orders and the generic M2L, through the C ABI.

* the generic dense M2L (operator entries formed per lane from lattice
  distances, any p) equals the tuned p = 4 kernel (operator tables in LDS) to
  FP64 rounding, for one right-hand side (offset-major) and a batch
  (target-major), and within FP32 rounding in the FP32 form;
* the Fourier-domain M2L (Section 3.6.1, last paragraph) equals the dense one
  to FP64 rounding at p = 4;
* p_s = p_t = 6 and 8 (FAST6 and FAST8 of Section 4.2), dense and Fourier M2L:
  the potentials of a random history equal O1's near pairs plus O2's far field
  over all earlier intervals, stored by
  tests/golden/make_higher_order_reference.py (O2 at p = 8 takes minutes on the
  host).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_higher_order_reference as REF  # noqa: E402

from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, C0

CDT = 0.078
LEAF = 6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def _potentials(v, f, hist, nr=1, **kw):
    torch = _torch()
    S = tdbem.Solver(v, f, tdbem.Config(dt=CDT / C0, mode=tdbem.MODE_IFMM, n_rhs=nr, gmres_rtol=1e-12,
                                        gmres_maxit=200, **kw))
    out = torch.zeros((nr, S.ne) if nr > 1 else (S.ne,), dtype=torch.float64, device="cuda")
    S.potentials(torch.tensor(hist, device="cuda"), hist.shape[0], out)
    info = S.info()
    S.close()
    return out.cpu().numpy(), info


@pytest.mark.parametrize("prec,nr", [(tdbem.FP64, 1), (tdbem.FP64, 3), (tdbem.FP32, 1)])
def test_generic_m2l_equals_tuned_kernel_at_p4(prec, nr):
    v, f = icosphere(2)
    rng = np.random.default_rng(44 + nr)
    ne = 480
    hist = rng.standard_normal((40, ne) if nr == 1 else (40, nr, ne))
    a, _ = _potentials(v, f, hist, nr, leaf_max=LEAF, precision=prec)
    b, _ = _potentials(v, f, hist, nr, leaf_max=LEAF, precision=prec, m2l=tdbem.M2L_GENERIC)
    rel = np.abs(a - b).max() / np.abs(a).max()
    print(f"generic vs tuned M2L, precision {prec}, {nr} rhs: {rel:.2e}")
    # the two kernels sum the same products in different orders
    assert rel < (1e-11 if prec == tdbem.FP64 else 1e-3)


@pytest.mark.parametrize("kindA_dt2,nr", [(tdbem.DT2_SPLIT, 1), (tdbem.DT2_SPLIT, 3), (tdbem.DT2_KERNEL, 1),
                                          (tdbem.DT2_INTERP, 2)])
def test_fourier_m2l_equals_dense_at_p4(kindA_dt2, nr):
    """The Fourier-domain M2L (circulant embedding of the node-lattice
    convolution) against the dense tuned kernel: the same products to FP64
    rounding, for every kernel of the vector-potential group."""
    v, f = icosphere(2)
    rng = np.random.default_rng(7 + nr)
    hist = rng.standard_normal((40, 480) if nr == 1 else (40, nr, 480))
    a, _ = _potentials(v, f, hist, nr, leaf_max=LEAF, dt2=kindA_dt2)
    b, info = _potentials(v, f, hist, nr, leaf_max=LEAF, dt2=kindA_dt2, m2l=tdbem.M2L_FFT)
    rel = np.abs(a - b).max() / np.abs(a).max()
    print(f"Fourier vs dense M2L, dt2 {kindA_dt2}, {nr} rhs: {rel:.2e} (levels {info['lmax']}, M_t {info['Mt']})")
    assert rel < 1e-10


@pytest.mark.parametrize("m2l", [tdbem.M2L_AUTO, tdbem.M2L_FFT])
@pytest.mark.parametrize("name", ["p6", "p8"])
def test_higher_order_potentials_match_oracle(name, m2l):
    lev, cdt, leaf, p, n_hist, seed = REF.CASES[name]
    assert cdt == CDT
    ref = np.load(os.path.join(HERE, "golden", "higher_order_reference.npz"))
    v, f = icosphere(lev)
    hist = REF.history(480, n_hist, seed)
    got, info = _potentials(v, f, hist, leaf_max=leaf, p_s=p, p_t=p, m2l=m2l)
    assert info["Mt"][2:] == ref[name + "_Mt"][2:].tolist()
    tot, far = ref[name + "_potentials"], ref[name + "_far"]
    rel = np.abs(got - tot).max() / np.abs(tot).max()
    rel_far = np.abs(got - tot).max() / np.abs(far).max()
    print(f"{name}: levels {info['lmax']}, rel err {rel:.2e} (relative to the far part {rel_far:.2e})")
    assert rel < 1e-10 and rel_far < 1e-9
