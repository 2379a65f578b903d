"""Late-time behaviour of the oracle's MOT march (CPU): after the pulse has
passed, the current of the 80-triangle sphere decays window after window, with
no growth over five times the pulse duration."""
import numpy as np

from oracle import oracle as O
from paper_2303_05006_amd.inputs import icosphere, gaussian_pulse, C0


def test_oracle_march_decays_at_late_time():
    v, f = icosphere(1)
    m = O.Mesh(v, f)
    dt = 0.25e-9
    cdt = C0 * dt
    pulse = gaussian_pulse(150e6, 100e6)
    nt = 801                                   # 800 steps; the pulse is over by step ~150
    Z = O.zdense(m, cdt, 1.0, C0 / 2)
    V = O.incident_all(m, pulse, dt, nt, 1.0, C0 / 2)
    J = O.march_dense(Z, V)
    win = np.sqrt((J.reshape(16, 50, -1) ** 2).sum(axis=(1, 2)))
    peak = win.max()
    late = win[6:]
    print("window norms / peak:", " ".join(f"{x / peak:.1e}" for x in win))
    assert late[-1] < 1e-6 * peak
    assert np.all(late[1:] <= late[:-1] * 1.05)
