"""T_c from the Binder cumulant on the GPU path: U_L = 1 - <m^4> / (3 <m^2>^2)
becomes size-independent at the critical point, so the curves U_64(T) and
U_128(T) cross at T_c = 2 / ln(1 + sqrt 2) up to corrections to scaling that
are small on the square lattice.  The samples come from Swendsen-Wang steps
(which decorrelate in a few steps at T_c) of one batch holding 32 replicas per
temperature and size; the crossing is located by linear interpolation of
U_64 - U_128 between the grid temperatures around its sign change (measured: T = 2.2690 against
T_c = 2.2692, U = 0.610 there; the bounds below are several times the
statistical spread).
"""

import numpy as np
import pytest

from oracle import exact

pytestmark = pytest.mark.gpu

TEMPS = np.linspace(2.24, 2.30, 9)
SIZES = (64, 128)
REPS = 32
STEPS, BURN = 3000, 300


def test_binder_crossing_at_tc():
    import torch
    import paper_2404_16990_amd as P
    descs, keys = [], []
    for L in SIZES:
        for ti, T in enumerate(TEMPS):
            for k in range(REPS):
                descs.append(dict(Lx=L, Ly=L, J=1.0, beta=1.0 / T, seed=7000 + len(descs), replica=len(descs), init=0))
                keys.append((L, ti))
    b = P.Batch(descs)
    _, mag = b.cluster(STEPS, "sw", 1)
    torch.cuda.synchronize()
    m = mag.cpu().numpy().astype(np.float64)[:, BURN:]
    b.close()
    keys = np.array(keys)
    U = {}
    for L in SIZES:
        for ti in range(len(TEMPS)):
            sel = (keys[:, 0] == L) & (keys[:, 1] == ti)
            x = m[sel] / (L * L)
            m2, m4 = (x ** 2).mean(), (x ** 4).mean()
            U[L, ti] = 1.0 - m4 / (3.0 * m2 * m2)
    diff = np.array([U[SIZES[0], ti] - U[SIZES[1], ti] for ti in range(len(TEMPS))])
    print("U_64:", [round(float(U[64, ti]), 4) for ti in range(len(TEMPS))], flush=True)
    print("U_128:", [round(float(U[128, ti]), 4) for ti in range(len(TEMPS))], flush=True)
    # below T_c the larger lattice is more ordered (U closer to 2/3), above it less
    assert diff[0] < 0 < diff[-1], diff
    k = int(np.argmax(diff > 0))
    t_cross = TEMPS[k - 1] + (TEMPS[k] - TEMPS[k - 1]) * (-diff[k - 1]) / (diff[k] - diff[k - 1])
    assert abs(t_cross - exact.T_C) < 0.004, (t_cross, exact.T_C)
    u_cross = U[SIZES[0], k - 1] + (U[SIZES[0], k] - U[SIZES[0], k - 1]) * (t_cross - TEMPS[k - 1]) / (TEMPS[k] - TEMPS[k - 1])
    assert 0.59 < u_cross < 0.63, u_cross
    print(f"crossing T = {t_cross:.4f} (T_c = {exact.T_C:.4f}), U = {u_cross:.4f}", flush=True)
