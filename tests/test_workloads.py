"""Host-side checks of the seeded input generators (no method arithmetic)."""
import numpy as np
from scipy import ndimage

from paper_1510_03560_amd import workloads as W


def _components(case):
    p = case.params
    sol = case.solid.reshape(p["nz"], p["ny"], p["nx"])
    lab, n = ndimage.label(sol == 0)
    return sol, lab, n


def test_channel_network_live_and_sealed_tubes():
    """Every live tube runs from the inlet face to the outlet face, every
    sealed tube touches neither, and no two tubes merge."""
    for shape, n_live in [((128, 64, 32), 2), ((256, 256, 64), 4)]:
        c = W.channel_network(*shape, seed=1, n_live=n_live)
        sol, lab, n = _components(c)
        assert n == 2 * n_live
        inlet = set(np.unique(lab[:, :, 0])) - {0}
        outlet = set(np.unique(lab[:, :, -1])) - {0}
        assert inlet == outlet and len(inlet) == n_live
        # the initial mesh is the inlet layer of blocks holding fluid
        B = 16
        nbz, nby, nbx = shape[2] // B, shape[1] // B, shape[0] // B
        act = c.active_blocks.reshape(nbz, nby, nbx)
        fluid_b = (sol == 0).reshape(nbz, B, nby, B, nbx, B).any(axis=(1, 3, 5))
        assert np.array_equal(act[:, :, 0] != 0, fluid_b[:, :, 0]) and act[:, :, 1:].sum() == 0


def test_channel_network_is_seeded():
    a = W.channel_network(128, 64, 32, seed=3, n_live=2)
    b = W.channel_network(128, 64, 32, seed=3, n_live=2)
    c = W.channel_network(128, 64, 32, seed=4, n_live=2)
    assert np.array_equal(a.solid, b.solid) and not np.array_equal(a.solid, c.solid)


def test_crop_keeps_faces_and_fields():
    case = W.porous_noise(64, 0)
    sub, art = W.crop(case, (0, 16, 16), (32, 32, 48))
    assert sub.params["bc"][0] == W.INLET and art == (0, 1, 1, 1, 1, 0)
    full = case.rho0.reshape(2, 64, 64, 64)
    assert np.array_equal(sub.rho0.reshape(2, 48, 32, 32), full[:, 16:64, 16:48, 0:32])
