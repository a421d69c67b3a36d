"""Pins of the oracle's electric force along the local face normal
(elec_normal = 1; an alternative to the electrode direction of the paper's
reading).  CPU only.  What fixes each expected value:
  - on flat walls the local normal is the electrode direction, so the whole
    trajectory equals the elec_normal = 0 one bit for bit;
  - an independent numpy derivation (minimum-image displacements to every
    solid node of the lattice) gives the same direction codes on a rough
    channel;
  - hand-worked nodes next to a step: beside a vertical face the force points
    into the face, at the foot of the step it points diagonally into the
    corner;
  - mirroring the geometry in x mirrors the codes and the trajectory.
"""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
MIRROR_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]


def numpy_codes(p, solid):
    """Direction codes from the definition, by minimum-image displacement to
    every solid node (needs nx, ny > 2 k + 1 so that images do not repeat)."""
    layer, _ = O.electric_layer(p, solid)
    ny, nx = solid.shape
    sy, sx = np.nonzero(solid)
    code = np.zeros_like(solid)
    for y, x in zip(*np.nonzero(layer)):
        dx = (sx - x + nx // 2) % nx - nx // 2
        dy = (sy - y + ny // 2) % ny - ny // 2
        d = np.maximum(np.abs(dx), np.abs(dy))
        sel = d == d.min()
        v = np.array([dx[sel].sum(), dy[sel].sum()])
        s = np.sign(v)
        if s.any():
            code[y, x] = int(np.nonzero((E == s).all(1))[0][0])
    return code


def test_flat_walls_give_the_electrode_direction_bitwise():
    c = I.channel_case(48, 24, I.flat_channel(48, 24), f_elec=2e-3, accel=1e-6, seed=1, layers=2)
    p1 = c.params.replace(elec_normal=1)
    code = O.electric_normal(p1, c.solid)
    layer, top = O.electric_layer(c.params, c.solid)
    assert np.all(code[(layer == 1) & (top == 0)] == 4)      # e_4 = (0, -1) at the bottom
    assert np.all(code[(layer == 1) & (top == 1)] == 2)      # e_2 = (0, +1) at the top
    assert np.all(code[layer == 0] == 0)
    f0 = O.init(c.params, c.solid, c.rho)
    f1 = f0.copy()
    O.step(c.params, c.solid, f0, 300)
    O.step(p1, c.solid, f1, 300)
    assert np.array_equal(f0, f1)


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_codes_match_independent_derivation(layers):
    c = I.rough_channel_case(nx=64, ny=40, f_elec=1e-3, seed=2, layers=layers)
    p = c.params.replace(elec_normal=1)
    np.testing.assert_array_equal(O.electric_normal(p, c.solid), numpy_codes(p, c.solid))
    assert np.all(O.electric_normal(c.params, c.solid) == 0)   # elec_normal = 0: no codes


def test_hand_worked_step():
    """Bottom wall (row 0) with one step of width 4 and height 3 at x = 10..13."""
    nx, ny = 32, 20
    s = np.zeros((ny, nx), np.uint8)
    s[0, :] = 1
    s[ny - 1, :] = 1
    s[1:4, 10:14] = 1
    p = I.Params(nx=nx, ny=ny, elec_layers=1, elec_normal=1)
    code = O.electric_normal(p, s)
    assert code[2, 9] == 1      # beside the left face, mid height: towards +x (into the step)
    assert code[2, 14] == 3     # beside the right face: towards -x
    assert code[1, 9] == 8      # foot of the left face: wall below, step to the right: (1, -1)
    assert code[4, 11] == 4     # on top of the step: towards -y
    assert code[4, 9] == 8      # above the left edge of the step, diagonal neighbour only: (1, -1)
    assert code[1, 5] == 4      # flat floor away from the step
    flags = O.flags(p, s)
    assert (flags[2, 9] >> 11) & 15 == 1 and (flags[1, 9] >> 11) & 15 == 8


def test_mirror_covariance():
    c = I.rough_channel_case(nx=64, ny=40, f_elec=2e-3, accel=0.0, seed=4, layers=2)
    p = c.params.replace(elec_normal=1)
    sm = c.solid[:, ::-1].copy()
    code = O.electric_normal(p, c.solid)
    code_m = O.electric_normal(p, sm)
    np.testing.assert_array_equal(code_m, np.array(MIRROR_X)[code[:, ::-1]])
    rho = c.rho
    f = O.init(p, c.solid, rho)
    fm = O.init(p, sm, rho[:, ::-1].copy())
    O.step(p, c.solid, f, 200)
    O.step(p, sm, fm, 200)
    mirrored = f[MIRROR_X][:, :, ::-1]
    np.testing.assert_allclose(fm, mirrored, rtol=0, atol=1e-13)
