"""The sub-box argument behind the sampled full-size parity tests, checked on
the oracle alone: after k steps a cell depends only on the initial state
within 2k cells (one cell of streaming plus one cell of the force stencil
per step), so a sub-box with walls on its cut faces reproduces the full run
bit for bit on the cells farther than 2k + 2 from every cut face, and does
not near the cut faces."""
import numpy as np

import oracle
from paper_1510_03560_amd import workloads as W

K = 3


def test_subbox_matches_full_run_away_from_cut_faces():
    oracle.set_threads(4)
    case = W.porous_noise(48, 2)
    full = oracle.Sim(case.params, case.solid, case.rho0, case.u0, None)
    full.step(K)
    fr, fu, _, _ = full.moments()
    n = 48
    fr = fr.reshape(2, n, n, n)
    fu = fu.reshape(2, 3, n, n, n)
    m = 2 * K + 2
    for origin in [(0, 0, 0), (16, 16, 16), (16, 0, 16)]:
        sub, art = W.crop(case, origin, (32, 32, 32))
        s = oracle.Sim(sub.params, sub.solid, sub.rho0, sub.u0, None)
        s.step(K)
        sr, su, _, _ = s.moments()
        sr = sr.reshape(2, 32, 32, 32)
        su = su.reshape(2, 3, 32, 32, 32)
        sl = [slice(m if art[2 * d] else 0, 32 - m if art[2 * d + 1] else 32) for d in range(3)]
        g = [slice(origin[d] + sl[d].start, origin[d] + sl[d].stop) for d in range(3)]
        assert np.array_equal(sr[:, sl[2], sl[1], sl[0]], fr[:, g[2], g[1], g[0]])
        assert np.array_equal(su[:, :, sl[2], sl[1], sl[0]], fu[:, :, g[2], g[1], g[0]])
        if any(art):
            # the cut faces do change the cells next to them
            assert not np.array_equal(sr, fr[:, origin[2]:origin[2] + 32, origin[1]:origin[1] + 32,
                                             origin[0]:origin[0] + 32])
