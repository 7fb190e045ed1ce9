"""Pins of the oracle's learned-correction training targets (mean of the 4 fine faces covering a coarse
face minus the coarse face value): exact on linear face data, where the mean is the value at the coarse
face's centre, and the coarse value enters with a minus sign."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk


def face_slot(d, x, y, z):
    return ((z * 8 + y) * 9 + x) if d == 0 else (((z * 9 + y) * 8 + x) if d == 1 else ((z * 8 + y) * 8 + x))


def faces_of(ijk, fn):
    """Face data [n * 1728, 8] of blocks ijk: component v of face (d, x, y, z) of block b is
    fn(d, X, Y, Z) + v at the face's global coordinates (X along d at the face, the others cell indices)."""
    ijk = np.asarray(ijk).reshape(-1, 3)
    out = np.zeros((ijk.shape[0], 3, 576, 8))
    for b in range(ijk.shape[0]):
        for d in range(3):
            ext = [8, 8, 8]
            ext[d] = 9
            for z in range(ext[2]):
                for y in range(ext[1]):
                    for x in range(ext[0]):
                        val = fn(d, 8 * ijk[b, 0] + x, 8 * ijk[b, 1] + y, 8 * ijk[b, 2] + z)
                        out[b, d, face_slot(d, x, y, z)] = val + np.arange(8)
    return out.reshape(-1, 8).astype(np.float32)


def grids(nroot):
    lv, ijk, _ = wk.uniform_blocks(nroot)
    lvf, ijkf, _ = wk.two_level_blocks(nroot, np.ones(nroot[::-1], bool))
    return ijkf, ijk


@pytest.mark.parametrize("nroot", [(2, 1, 1), (1, 2, 2)])
def test_linear_fine_faces_average_to_the_coarse_face_centre(oracle_mod, nroot):
    fine_ijk, coarse_ijk = grids(nroot)
    fn = lambda d, X, Y, Z: 1000.0 * d + X + 32.0 * Y + 1024.0 * Z
    Ff = faces_of(fine_ijk, fn)
    Fc = np.zeros((len(coarse_ijk) * 1728, 8), np.float32)
    T = oracle_mod.face_targets(Ff, fine_ijk, Fc, coarse_ijk).reshape(len(coarse_ijk), 3, 576, 8)
    for c, cijk in enumerate(np.asarray(coarse_ijk).reshape(-1, 3)):
        for d in range(3):
            ext = [8, 8, 8]
            ext[d] = 9
            for z in range(ext[2]):
                for y in range(ext[1]):
                    for x in range(ext[0]):
                        q = [8 * cijk[0] + x, 8 * cijk[1] + y, 8 * cijk[2] + z]
                        # fine coordinates: the face plane at twice the coarse position, the two fine rows
                        # across it centred at twice the coarse index plus a half
                        g = [2.0 * q[a] + (0.0 if a == d else 0.5) for a in range(3)]
                        want = fn(d, *g) + np.arange(8)
                        assert np.array_equal(T[c, d, face_slot(d, x, y, z)], want.astype(np.float32)), (c, d, x, y, z)


def test_coarse_value_is_subtracted(oracle_mod):
    fine_ijk, coarse_ijk = grids((1, 1, 1))
    rng = np.random.default_rng(3)
    Ff = rng.normal(size=(len(fine_ijk) * 1728, 8)).astype(np.float32)
    Fc = rng.normal(size=(len(coarse_ijk) * 1728, 8)).astype(np.float32)
    T0 = oracle_mod.face_targets(Ff, fine_ijk, np.zeros_like(Fc), coarse_ijk)
    T1 = oracle_mod.face_targets(Ff, fine_ijk, Fc, coarse_ijk)
    assert np.array_equal(T1, (T0.astype(np.float64) - Fc.astype(np.float64)).astype(np.float32)) or \
        np.max(np.abs(T1 - (T0 - Fc))) <= 2.0 ** -22 * (np.abs(T0).max() + np.abs(Fc).max())
