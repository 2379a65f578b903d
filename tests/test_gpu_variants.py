"""Variants of the method and the rest of the boundary, through the C ABI.

* CFIE2 and CFIE3 (Section 4.3.1): the direct march against the oracle's
  (O1, dense LU) to 1e-9, and the IFMM potentials against O1 near + O2 far;
* the three placements of the vector potential's second time derivative
  (Section 4.3.2) against O2;
* the late-time stability monitor: tripped from the host by a tiny limit once
  the excitation has passed, silent with a large one;
* checkpoint / restore: a restored context marches bitwise like the original;
* the all-pairs coefficient count and the configuration in effect.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from oracle.ifmm import IFMM
from oracle.constants import C0, EPS0, MU0
from paper_2303_05006_amd import tdbem
from paper_2303_05006_amd.inputs import icosphere, gaussian_pulse

CDT = 0.078        # 480-edge sphere: d_s(3) = 0.25, M_t = 3
LEAF = 6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return torch


def _march(S, pulses, nt, torch, rc_out=None):
    shape = (S.ne,) if len(pulses) == 1 else (len(pulses), S.ne)
    V = torch.zeros(shape, dtype=torch.float64, device="cuda")
    J = torch.zeros(shape, dtype=torch.float64, device="cuda")
    out = torch.zeros((nt - 1,) + shape, dtype=torch.float64, device="cuda")
    for a in range(1, nt):
        S.incident(pulses, a, V)
        rc = S.step_rc(V, J)
        if rc_out is not None:
            rc_out.append(rc)
        elif rc != tdbem.OK:
            raise tdbem.TdbemError(rc, "step")
        out[a - 1] = J
    return out


@pytest.mark.parametrize("cfie", [tdbem.CFIE2, tdbem.CFIE3])
def test_direct_march_cfie_variant_matches_oracle(cfie):
    torch = _torch()
    v, f = icosphere(1)
    dt, nt = 0.25e-9, 60
    m = O.Mesh(v, f)
    pulse = gaussian_pulse(150e6, 100e6)
    Z = O.zdense(m, dt * C0, 1.0, C0 / 2, cfie=cfie)
    Vref = O.incident_all(m, pulse, dt, nt, 1.0, C0 / 2, cfie=cfie)
    Jref = O.march_dense(Z, Vref)
    S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_DIRECT, cfie=cfie, gmres_rtol=1e-14,
                                        gmres_maxit=100))
    got = _march(S, [pulse], nt, torch).cpu().numpy()
    S.close()
    rel = float(np.linalg.norm(got - Jref) / np.linalg.norm(Jref))
    print(f"CFIE{cfie} direct march vs oracle: {rel:.2e}")
    assert rel < 1e-9


VARIANTS = [(tdbem.CFIE2, tdbem.DT2_SPLIT), (tdbem.CFIE3, tdbem.DT2_SPLIT),
            (tdbem.CFIE1, tdbem.DT2_KERNEL), (tdbem.CFIE1, tdbem.DT2_INTERP)]
DT2 = {tdbem.DT2_SPLIT: "split", tdbem.DT2_KERNEL: "kernel", tdbem.DT2_INTERP: "interp"}


@pytest.fixture(scope="module", params=VARIANTS, ids=lambda p: f"cfie{p[0]}-{DT2[p[1]]}")
def variant(request):
    _torch()
    cfie, dt2 = request.param
    v, f = icosphere(2)
    m = O.Mesh(v, f)
    dt = CDT / C0
    S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_IFMM, leaf_max=LEAF, gmres_rtol=1e-13,
                                        gmres_maxit=200, cfie=cfie, dt2=dt2))
    F = IFMM(m, dt, 1.0, C0 / 2, EPS0, MU0, leaf_max=LEAF, interp_t="chi", cfie=cfie, dt2=DT2[dt2])
    G = O.max_lag(m, CDT) + 1
    Z = O.zrows(m, np.arange(m.ne), CDT, 1.0, C0 / 2, G=G, cfie=cfie)
    near = np.zeros((m.ne, m.ne), bool)
    for i, j in F.H.near_pairs():
        near[i, j] = True
    # one random history; the far field at step a uses J^0..J^{a-2} only, so
    # the potentials after its first n steps are row n of O2's causal march
    hist = np.random.default_rng(50).standard_normal((45, m.ne))
    farh = F.far_history(hist)
    yield m, S, Z, near, hist, farh
    S.close()


@pytest.mark.parametrize("n_hist", [30, 45])
def test_variant_potentials_match_near_plus_all_interval_far(variant, n_hist):
    torch = _torch()
    m, S, Z, near, hist_all, farh = variant
    hist = np.ascontiguousarray(hist_all[:n_hist])
    a = n_hist + 1
    Zn = Z * near[:, :, None]
    ref = np.zeros(m.ne)
    for g in range(2, Z.shape[2]):
        if 0 <= a - g < n_hist:
            ref += Zn[:, :, g] @ hist[a - g]
    far = farh[a - 1]
    ref += far
    out = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
    S.potentials(torch.tensor(hist, device="cuda"), n_hist, out)
    got = out.cpu().numpy()
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    rel_far = np.abs(got - ref).max() / max(np.abs(far).max(), 1e-300)
    print(f"n_hist={n_hist}: rel err {rel:.2e} (relative to the far part {rel_far:.2e})")
    assert rel < 1e-10 and rel_far < 1e-9


def test_monitor_trips_when_forced_and_stays_silent_otherwise():
    """A stable direct march: with growth_limit 1e-30 the first step after the
    excitation has passed returns EUNSTABLE (forced from the host); with 1e6
    no step does.  reset() clears the monitor."""
    torch = _torch()
    v, f = icosphere(1)
    pulse = gaussian_pulse(300e6, 200e6)
    dt, nt = 0.5e-9, 90
    for limit, expect in ((1e-30, True), (1e6, False)):
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_DIRECT, gmres_rtol=1e-12, growth_limit=limit))
        rcs = []
        _march(S, [pulse], nt, torch, rcs)
        tripped = [a + 1 for a, rc in enumerate(rcs) if rc == tdbem.EUNSTABLE]
        assert all(rc in (tdbem.OK, tdbem.EUNSTABLE) for rc in rcs)
        print(f"growth_limit {limit:g}: first EUNSTABLE at step {tripped[0] if tripped else None}")
        if expect:
            # the pulse has passed the 1 m sphere by about t = 10 sigma + 2 R / c = 30 ns = step 60
            assert tripped and 40 <= tripped[0] <= 75
            assert S.unstable()[0] == 1
            S.reset()
            assert S.unstable()[0] == 0
        else:
            assert not tripped
        S.close()


@pytest.mark.parametrize("mode,prec,m2l", [(tdbem.MODE_DIRECT, tdbem.FP64, 0), (tdbem.MODE_IFMM, tdbem.FP64, 0),
                                           (tdbem.MODE_IFMM, tdbem.FP32, 0),
                                           (tdbem.MODE_IFMM, tdbem.FP64, tdbem.M2L_FFT)])
def test_checkpoint_restore_resumes_bitwise(mode, prec, m2l):
    """(With the Fourier-domain M2L the transformed moments are rebuilt from the
    restored moments.)"""
    torch = _torch()
    v, f = icosphere(2)
    dt = CDT / C0
    cfg = dict(dt=dt, mode=mode, precision=prec, leaf_max=LEAF, gmres_rtol=1e-12, gmres_maxit=200, growth_limit=1e9,
               m2l=m2l)
    pulse = gaussian_pulse(150e6, 100e6)
    A = tdbem.Solver(v, f, tdbem.Config(**cfg))
    V = torch.zeros(A.ne, dtype=torch.float64, device="cuda")
    J = torch.zeros(A.ne, dtype=torch.float64, device="cuda")
    for a in range(1, 41):               # stop between time gates of every level
        A.incident([pulse], a, V)
        A.step(V, J)
    state = A.checkpoint()
    ref = []
    for a in range(41, 81):
        A.incident([pulse], a, V)
        A.step(V, J)
        ref.append(J.clone())
    B = tdbem.Solver(v, f, tdbem.Config(**cfg))
    B.restore(state)
    assert B.query_i32(tdbem.Q_STEP) == 41
    for k, a in enumerate(range(41, 81)):
        B.incident([pulse], a, V)
        B.step(V, J)
        assert torch.equal(J, ref[k]), a
    # the same context, rewound
    A.restore(state)
    for k, a in enumerate(range(41, 51)):
        A.incident([pulse], a, V)
        A.step(V, J)
        assert torch.equal(J, ref[k]), a
    # another configuration refuses it
    C = tdbem.Solver(v, f, tdbem.Config(**dict(cfg, gmres_rtol=1e-11)))
    with pytest.raises(tdbem.TdbemError) as e:
        C.restore(state)
    assert e.value.code == tdbem.EINVAL
    with pytest.raises(tdbem.TdbemError):
        B.restore(state[:-8])
    for S in (A, B, C):
        S.close()


def test_all_pairs_count_and_config_in_effect():
    _torch()
    v, f = icosphere(2)
    dt = CDT / C0
    D = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_DIRECT))
    d = D.info()
    # every pair stores its exact lag range; g = 1 entries make up Z0
    assert D.d0_nnz() == d["near_nnz"] + d["z0_nnz"]
    F = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=tdbem.MODE_IFMM, leaf_max=LEAF, box_widen=1, causal_guard=0,
                                        solver=tdbem.SOLVER_HOST, gmres_restart=20, cfie=tdbem.CFIE2))
    assert F.d0_nnz() == D.d0_nnz()
    eff = F.config_in_effect()
    assert (eff["box_widen"], eff["causal_guard"], eff["solver"], eff["gmres_restart"], eff["cfie"]) == \
        (1, 0, tdbem.SOLVER_HOST, 20, tdbem.CFIE2)
    D.close()
    F.close()


@pytest.mark.parametrize("field,value", [("cfie", 0), ("cfie", 4), ("n_quad", 6), ("gmres_restart", 0),
                                         ("gmres_restart", 33), ("dt2", 3), ("solver", 2), ("growth_limit", -1.0),
                                         ("box_widen", 2), ("p_s", 5), ("p_s", 6), ("m2l", 7),
                                         ("m2l+fp32", tdbem.M2L_FFT), ("m2l+p6", tdbem.M2L_BF16),
                                         ("near_kernel", 8), ("near_kernel", 9), ("autotune", 2),
                                         ("graph", 2), ("graph+host", 1), ("near_kernel+rhs", 3)])
def test_invalid_configuration_fields(field, value):
    """(p_s = 6 with p_t = 4: the orders must agree; the Fourier-domain M2L with
    FP32; the graph march needs the device solver; with several right-hand
    sides only near_kernel 1 and 8 exist.)"""
    _torch()
    v, f = icosphere(1)
    cfg = tdbem.Config(dt=0.1 / C0, mode=tdbem.MODE_IFMM, leaf_max=6)
    if field == "m2l+fp32":               # the Fourier-domain M2L is FP64 only
        field, cfg.precision = "m2l", tdbem.FP32
    if field == "m2l+p6":                 # the bf16 M2L is built for p = 4
        field, cfg.p_s, cfg.p_t = "m2l", 6, 6
    if field == "graph+host":             # graphs wrap the device solve's launches
        field, cfg.solver = "graph", tdbem.SOLVER_HOST
    if field == "near_kernel+rhs":        # a one-rhs form with two right-hand sides
        field, cfg.n_rhs = "near_kernel", 2
    setattr(cfg, field, value)
    with pytest.raises(tdbem.TdbemError) as e:
        tdbem.Solver(v, f, cfg)
    assert e.value.code == tdbem.EINVAL


@pytest.mark.parametrize("mode", [tdbem.MODE_DIRECT, tdbem.MODE_IFMM])
def test_autotuned_context_marches_like_the_default(mode):
    """autotune = 1 picks a near-field form and the device solve's blocks per
    system by timing them at set-up (TDBEM_Q_TUNED); the march is the same up
    to the order of FP64 sums."""
    torch = _torch()
    v, f = icosphere(3)
    dt = 0.05 / C0
    cfg = dict(dt=dt, mode=mode, leaf_max=16, gmres_rtol=1e-12, gmres_maxit=200)
    A = tdbem.Solver(v, f, tdbem.Config(**cfg))
    B = tdbem.Solver(v, f, tdbem.Config(**cfg, autotune=1))
    tuned = B.query_array(tdbem.Q_TUNED, 4, np.int32)
    print(f"tuned: near round {tuned[0]} lag steps x {tuned[1]} pair blocks, solve blocks {tuned[2]}")
    assert tuned[3] == 1 and (tuned[0], tuned[1]) in {(2, 1), (1, 1), (3, 1), (2, 2), (1, 2), (2, 0), (1, 0)}
    assert tuned[2] in (0, 64, 96, 128, 160, 192, 256)
    # the default: the per-leaf kernel (2 lag steps, shape (2, 0)) where any
    # leaf's window fits the LDS budget, else the row kernel (2, 1)
    assert A.query_array(tdbem.Q_TUNED, 4, np.int32).tolist() in ([2, 0, 0, 0], [2, 1, 0, 0])
    pulse = gaussian_pulse(300e6, 200e6)
    Ja = _march(A, [pulse], 80, torch).cpu().numpy()
    Jb = _march(B, [pulse], 80, torch).cpu().numpy()
    rel = np.abs(Ja - Jb).max() / np.abs(Ja).max()
    print(f"tuned vs default march: {rel:.2e}")
    assert rel < 1e-10
    A.close()
    B.close()


@pytest.mark.parametrize("mode,prec,level,cdt", [(tdbem.MODE_IFMM, tdbem.FP64, 2, CDT),
                                                 (tdbem.MODE_IFMM, tdbem.FP32, 2, CDT),
                                                 (tdbem.MODE_DIRECT, tdbem.FP64, 3, 0.075),
                                                 (tdbem.MODE_DIRECT, tdbem.FP64, 3, 0.01)])
def test_near_field_forms_agree_bitwise(mode, prec, level, cdt):
    """Every one-rhs near-field form (near_kernel 1..7) on the same history
    agrees with the default row kernel to FP64 rounding (the per-leaf forms 6
    and 7 read the sources' currents from LDS and give each lane other
    (pair, lag) terms, so they sum in another order).  In the direct mode at
    c dt = 0.01 m every pair is near and each leaf's window (all 1920 sources
    over some 30 lags) exceeds the LDS budget, so the per-leaf forms hand all
    rows to the default row kernel's gathers: bitwise equal."""
    torch = _torch()
    v, f = icosphere(level)
    dt = cdt / C0
    ne = 3 * len(f) // 2
    hist = torch.tensor(np.random.default_rng(9).standard_normal((40, ne)), device="cuda")
    outs = {}
    for k in range(1, 8):
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=mode, precision=prec, leaf_max=LEAF, near_kernel=k))
        assert S.query_array(tdbem.Q_TUNED, 4, np.int32)[3] == 0
        o = torch.zeros(ne, dtype=torch.float64, device="cuda")
        S.potentials(hist, 40, o)
        outs[k - 1] = o
        S.close()
    if cdt == 0.01:                       # both hand every row to the row kernel's gathers
        assert torch.equal(outs[5], outs[0]) and torch.equal(outs[6], outs[0])
    ref = outs[0].abs().max()
    for k in range(1, 7):
        assert float((outs[k] - outs[0]).abs().max() / ref) < 1e-13


@pytest.mark.parametrize("mode,prec,nr,level,cdt", [(tdbem.MODE_IFMM, tdbem.FP64, 3, 2, CDT),
                                                    (tdbem.MODE_IFMM, tdbem.FP64, 70, 2, CDT),
                                                    (tdbem.MODE_IFMM, tdbem.FP32, 3, 2, CDT),
                                                    (tdbem.MODE_DIRECT, tdbem.FP64, 2, 2, 0.1),
                                                    (tdbem.MODE_IFMM, tdbem.FP64, 5, 3, 0.01)])
def test_batched_near_field_on_the_matrix_cores(mode, prec, nr, level, cdt):
    """Batched right-hand sides: the per-leaf matrix-core near field
    (near_kernel 8: each leaf's coefficients as a dense block over its window,
    per source the lags its strips reach, times the sources' currents at those
    lags) against the row kernel (near_kernel 1)
    on the same history; 70 rhs spans two groups of 64 with a ragged second.
    FP64 to rounding of the sums; the FP32 form accumulates in FP32 on the
    matrix cores (the row kernel in FP64).  The last case (1280 triangles,
    leaves of 64 edges, c dt = 0.01 m, a history as long as the leaves' lag
    windows) has leaves wider than one column segment of 2048 (source, lag)
    columns, so their rows sum several segments."""
    torch = _torch()
    v, f = icosphere(level)
    dt = cdt / C0
    leaf = LEAF if level == 2 else 64
    nh = 30 if level == 2 else 160
    outs = []
    for k in (1, 8):                      # the row kernel, the matrix-core form
        S = tdbem.Solver(v, f, tdbem.Config(dt=dt, mode=mode, precision=prec, leaf_max=leaf, n_rhs=nr,
                                            near_kernel=k))
        ne = S.ne
        if k == 1:
            hist = torch.tensor(np.random.default_rng(nr).standard_normal((nh, nr, ne)), device="cuda")
        o = torch.zeros((nr, ne), dtype=torch.float64, device="cuda")
        S.potentials(hist, nh, o)
        outs.append(o)
        lb = S.info()["near_leaf_bytes"]
        S.close()
    vb = 8 if prec == tdbem.FP64 else 4
    assert lb > 0
    if level == 3:
        assert lb / vb / ne > 2048, "the leaves are expected to span several column segments"
    rel = float((outs[1] - outs[0]).abs().max() / outs[0].abs().max())
    print(f"mode {mode}, precision {prec}, {nr} rhs, {ne} edges: matrix-core vs row near field {rel:.2e}; "
          f"leaf blocks {lb / 1e6:.1f} MB")
    assert rel < (1e-12 if prec == tdbem.FP64 else 1e-5)
