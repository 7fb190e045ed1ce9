"""Pins of the oracle's learned flux correction and its face features (CPU only).

The learned form is not in the paper: F = F_plain + dF on every face not next to a body cell; a cell
whose provisional state is not positive or leaves the tau-widened range of its old 7-point
neighbourhood in density or pressure is flagged, every face of a flagged cell takes the plain flux again
on both sides, and the stage is recomputed once. These tests tie that definition to exact consequences:
the zero correction is the plain method, consistent corrections conserve, hand-built single-face cases
have closed-form results, and the stencil features are the primitives at known cell centres.
"""
import math

import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

GAMMA = 5.0 / 3.0
NO_STATS = np.concatenate([np.zeros(8), np.ones(8)])  # out_mean = 0, out_std = 1


def _plain(oracle_mod, wl, W, n_stages, **kw):
    g = oracle_mod.Grid.from_workload(wl)
    U0 = g.set_state(W)
    U1 = np.zeros_like(U0)
    dt, f = g.advance(U0, U1, np.zeros(len(wl.sims)), n_stages, **kw)
    return U0, U1, dt, f


def _learned(oracle_mod, wl, W, n_stages, y, ystats, **kw):
    g = oracle_mod.Grid.from_workload(wl)
    U0 = g.set_state(W)
    U1 = np.zeros_like(U0)
    dt, f, nflag = g.advance_learned(U0, U1, np.zeros(len(wl.sims)), n_stages, y, ystats, **kw)
    return U0, U1, dt, f, nflag


def total(wl, U):
    return np.array([math.fsum(U[v].ravel()) for v in range(8)])


@pytest.mark.parametrize("case", ["magnetosphere", "random_box"])
@pytest.mark.parametrize("n_stages", [1, 4])
def test_zero_correction_is_the_plain_method_bitwise(oracle_mod, case, n_stages):
    wl = wk.magnetosphere_cut(16) if case == "magnetosphere" else wk.odd_box()
    y = np.zeros((wl.n_blocks * 1728, 8))
    kw = dict(flux="hlle", powell=True)
    a0, a1, adt, af = _plain(oracle_mod, wl, wl.W, n_stages, **kw)
    b0, b1, bdt, bf, _ = _learned(oracle_mod, wl, wl.W, n_stages, y, NO_STATS, **kw)
    assert np.array_equal(adt, bdt) and af == bf
    assert np.array_equal(a0, b0) and np.array_equal(a1, b1)


@pytest.mark.parametrize("flux", ["rusanov", "hlle"])
def test_consistent_corrections_conserve(oracle_mod, flux):
    """A correction that is the same for both owners of each face moves conserved quantities between
    cells only; the fallback restores the plain flux on both sides of a face, so the totals of all eight
    conserved variables stay constant to round-off (periodic box, Powell off) while some cells fall back
    and others keep their correction."""
    wl = wk.uniform_state((2, 2, 2))
    W = wk.random_positive_state(wl, seed=3)
    y = wk.face_corrections(wl, seed=8, scale=1.0)
    ystats = np.concatenate([np.full(8, 1e-3), np.full(8, 4e-3)])
    U, _, _, f, nflag = _learned(oracle_mod, wl, W, 4, y, ystats, flux=flux, powell=False)
    g = oracle_mod.Grid.from_workload(wl)
    U0 = g.set_state(W)
    t0, t1 = total(wl, U0), total(wl, U)
    scale = np.array([math.fsum(np.abs(U0[v]).ravel()) for v in range(8)])
    assert f == 0
    assert 0 < nflag < 2 * wl.n_cells, nflag
    assert np.all(np.abs(t1 - t0) <= 1e-14 * scale), (t1 - t0) / scale
    Up, _, _, _ = _plain(oracle_mod, wl, W, 4, flux=flux, powell=False)
    assert np.abs(U - Up).max() > 1e-6  # the correction changed the result


def _one_face_case(face_axis, comp, value, W0, floor_rel):
    """Uniform periodic 2x1x1-block state; one face of axis face_axis (between cells (3,4,5) and its
    upper neighbour along that axis, in block 0) carries the normalised correction `value` in
    face-normal component `comp`; every other face none. One forward-Euler stage with dt = 0.01."""
    wl = wk.uniform_state((2, 1, 1), W0=W0)
    y = np.zeros((wl.n_blocks, 3, 576, 8))
    f, t1, t2 = wk.face_slots()
    cell = [3, 4, 5]
    fpos = cell[face_axis] + 1
    others = [a for a in range(3) if a != face_axis]
    s = int(np.where((f[face_axis] == fpos) & (t1[face_axis] == cell[others[0]]) &
                     (t2[face_axis] == cell[others[1]]))[0][0])
    y[0, face_axis, s, comp] = value
    return wl, y.reshape(-1, 8), cell


@pytest.mark.parametrize("face_axis", [0, 1, 2])
def test_single_face_correction_closed_form(oracle_mod, face_axis):
    """With a range floor wide enough to accept it, a correction dF on one face changes exactly its two
    cells, by -dt dF / dx (the lower cell) and +dt dF / dx (the upper one), with dF de-normalised
    (y * out_std + out_mean) and rotated from the face-normal frame: the normal component goes to the
    face's own axis, the first transverse one to the next axis (cyclically)."""
    W0 = (1.0, 0.2, -0.1, 0.3, 0.5, -0.4, 0.3, 0.7)
    dt = 0.01
    ystats = np.concatenate([np.full(8, 0.0), np.full(8, 0.5)])  # dF = 0.5 * 0.3 = 0.15
    for comp in range(8):
        wl, y, cell = _one_face_case(face_axis, comp, 0.3, W0, 1.0)
        g = oracle_mod.Grid.from_workload(wl)
        U0 = g.set_state(wl.W)
        ref = U0.copy()
        U1 = np.zeros_like(U0)
        _, _, nflag = g.advance_learned(U0, U1, [dt], 1, y, ystats, tau=0.1, floor_rel=10.0, flux="hlle",
                                        powell=True, recompute_dt=False)
        assert nflag == 0
        lab = comp if comp in (0, 7) else (1 + (face_axis + comp - 1) % 3 if comp < 4 else 4 + (face_axis + comp - 4) % 3)
        up = list(cell)
        up[face_axis] += 1
        exp = ref.copy()
        exp[lab, 0, cell[2], cell[1], cell[0]] = ref[lab, 0, cell[2], cell[1], cell[0]] + dt * (0.0 - 0.15)
        exp[lab, 0, up[2], up[1], up[0]] = ref[lab, 0, up[2], up[1], up[0]] + dt * (0.15 - 0.0)
        diff = np.argwhere(np.abs(U1 - exp) > 1e-15 * np.abs(ref).max())
        assert diff.size == 0, (comp, diff[:4])


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_single_face_fallback_reverts_both_cells(oracle_mod, sign):
    """A momentum correction dF on one x face of a uniform state moving along x changes the pressure of
    the lower cell by (gamma-1)(u0 d - d^2/(2 rho)) and that of the upper one by
    -(gamma-1)(u0 d + d^2/(2 rho)), d = dt dF / dx. With the band tau * floor * p0 between the two
    magnitudes, only one cell is flagged (the upper one for dF > 0, the lower one for dF < 0); its faces,
    including the corrected one, take the plain flux for both cells, so both cells return to the uniform
    state exactly and one cell is counted."""
    rho0, u0, p0 = 1.0, 0.5, 1.0
    W0 = (rho0, u0, 0.0, 0.0, 0.3, 0.2, -0.1, p0)
    dt, dF = 0.01, 0.3 * sign
    d = abs(dt * dF)
    rise = (GAMMA - 1) * (u0 * d - d * d / (2 * rho0))
    fall = (GAMMA - 1) * (u0 * d + d * d / (2 * rho0))
    tau, floor_rel = 0.1, 1e-2
    band = tau * floor_rel * p0
    assert rise < band < fall
    wl, y, cell = _one_face_case(0, 1, dF, W0, floor_rel)
    g = oracle_mod.Grid.from_workload(wl)
    U0 = g.set_state(wl.W)
    ref = U0.copy()
    U1 = np.zeros_like(U0)
    _, _, nflag = g.advance_learned(U0, U1, [dt], 1, y, NO_STATS, tau=tau, floor_rel=floor_rel, flux="hlle",
                                    powell=True, recompute_dt=False)
    assert nflag == 1
    assert np.array_equal(U1, ref)
    # with no floor the range of a uniform neighbourhood is zero: both cells are flagged
    U0 = g.set_state(wl.W)
    U1 = np.zeros_like(U0)
    _, _, nflag = g.advance_learned(U0, U1, [dt], 1, y, NO_STATS, tau=tau, floor_rel=0.0, flux="hlle",
                                    powell=True, recompute_dt=False)
    assert nflag == 2
    assert np.array_equal(U1, ref)


def test_faces_next_to_the_body_keep_the_plain_flux(oracle_mod):
    """Corrections on faces that touch a body cell are ignored: with corrections only on such faces the
    learned result is the plain result bitwise."""
    wl = wk.magnetosphere_cut(16)
    g = oracle_mod.Grid.from_workload(wl)
    # body membership from the cell centres, as the paper's masked body (a cell is in the body when its
    # centre lies strictly inside the sphere)
    x, yy, z = wk.cell_centres(wl.sims[0], wl.level, wl.ijk)
    c, r = wl.sims[0].body_c, wl.sims[0].body_r
    body = (x - c[0]) ** 2 + (yy - c[1]) ** 2 + (z - c[2]) ** 2 < r * r
    assert body.sum() > 0
    f, t1, t2 = wk.face_slots()
    y = np.zeros((wl.n_blocks, 3, 576, 8))
    rng = np.random.default_rng(0)
    for b in range(wl.n_blocks):
        for d in range(3):
            a1, a2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
            for s in range(576):
                lo = [0, 0, 0]
                lo[d], lo[a1], lo[a2] = f[d, s] - 1, t1[d, s], t2[d, s]
                hi = list(lo)
                hi[d] += 1
                touch = False
                for cc in (lo, hi):
                    if all(0 <= v < 8 for v in cc) and body[b, cc[2], cc[1], cc[0]]:
                        touch = True
                if touch:
                    y[b, d, s] = rng.standard_normal(8)
    assert np.abs(y).sum() > 0
    a0, _, _, _ = _plain(oracle_mod, wl, wl.W, 2, flux="hlle", powell=True)
    b0, _, _, _, _ = _learned(oracle_mod, wl, wl.W, 2, y.reshape(-1, 8), NO_STATS, flux="hlle", powell=True)
    assert np.array_equal(a0, b0)


# ------------------------------------------------------------------------------------------------
# features

def _linear_primitives(wl):
    """Primitives that are affine in the cell centre with a different gradient per variable."""
    x, y, z = wk.cell_centres(wl.sims[0], wl.level, wl.ijk)
    W = np.empty((8,) + x.shape)
    for v in range(8):
        W[v] = (1.0 + v) + (0.01 * (v + 1)) * x + (0.002 * (v + 3)) * y + (0.0003 * (v + 5)) * z
    W[0] += 2.0
    W[7] += 2.0
    return W


def _expected_features(wl, d, b, f, t1, t2):
    """Features of one interior face from the analytic primitives at the four stencil centres."""
    sim = wl.sims[0]
    a1, a2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
    out = np.empty(32)
    for q in range(4):
        idx = [0, 0, 0]
        idx[d], idx[a1], idx[a2] = f - 2 + q, t1, t2
        pos = [sim.origin[a] + (wl.ijk[b][a] * 8 + idx[a] + 0.5) * sim.dx0 for a in range(3)]
        w = [(1.0 + v) + (0.01 * (v + 1)) * pos[0] + (0.002 * (v + 3)) * pos[1] + (0.0003 * (v + 5)) * pos[2]
             for v in range(8)]
        w[0] += 2.0
        w[7] += 2.0
        rot = [w[0], w[1 + d], w[1 + (d + 1) % 3], w[1 + (d + 2) % 3], w[4 + d], w[4 + (d + 1) % 3],
               w[4 + (d + 2) % 3], w[7]]
        out[q * 8:(q + 1) * 8] = rot
    return out


def test_features_are_the_rotated_stencil_primitives(oracle_mod):
    """Interior faces of a large-enough grid (outflow boundaries copy, so stay two cells inside): the
    32 features are the primitives at the four stencil centres, in the face-normal frame, z-scored."""
    wl = wk.uniform_state((2, 2, 2), bc=(1,) * 6)
    W = _linear_primitives(wl)
    g = oracle_mod.Grid.from_workload(wl)
    U = g.set_state(W)
    rng = np.random.default_rng(1)
    stats = np.concatenate([rng.uniform(-1, 1, 32), rng.uniform(0.5, 2, 32)])
    X = g.face_features(U).reshape(wl.n_blocks, 3, 576, 32)
    Xz = g.face_features(U, stats).reshape(wl.n_blocks, 3, 576, 32)
    f, t1, t2 = wk.face_slots()
    checked = 0
    for b in range(wl.n_blocks):
        for d in range(3):
            for s in range(0, 576, 7):
                gl = wl.ijk[b][d] * 8 + f[d, s]
                if gl < 2 or gl > 14:
                    continue
                a1, a2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
                e = _expected_features(wl, d, b, f[d, s], t1[d, s], t2[d, s])
                assert np.allclose(X[b, d, s], e, rtol=1e-13, atol=1e-13), (b, d, s)
                assert np.allclose(Xz[b, d, s], (e - stats[:32]) / stats[32:], rtol=1e-12, atol=1e-12)
                checked += 1
    assert checked > 500


def test_features_follow_a_cyclic_axis_permutation(oracle_mod):
    """Permuting the data cyclically (x -> y -> z -> x, vectors likewise) maps the features of x faces
    onto those of y faces: the face-normal frame is the cyclic one."""
    wl = wk.uniform_state((1, 1, 1))
    W = wk.random_positive_state(wl, seed=9)
    G = W[:, 0]                                # [v][z][y][x]
    P = np.moveaxis(G, 1, 3).copy()            # new (z, y, x) = old (y, x, z): x -> y -> z -> x
    P[1], P[2], P[3] = np.moveaxis(G[3], 0, 2), np.moveaxis(G[1], 0, 2), np.moveaxis(G[2], 0, 2)
    P[4], P[5], P[6] = np.moveaxis(G[6], 0, 2), np.moveaxis(G[4], 0, 2), np.moveaxis(G[5], 0, 2)
    g = oracle_mod.Grid.from_workload(wl)
    X = g.face_features(g.set_state(W)).reshape(3, 576, 32)
    Xp = g.face_features(g.set_state(P[:, None])).reshape(3, 576, 32)
    f, t1, t2 = wk.face_slots()
    # old x face (f, t1 = y, t2 = z) is new y face (f, t1 = x' = old z, t2 = z' = old y)
    for s in range(576):
        sp = int(np.where((f[1] == f[0, s]) & (t1[1] == t2[0, s]) & (t2[1] == t1[0, s]))[0][0])
        assert np.allclose(Xp[1, sp], X[0, s], rtol=1e-14, atol=1e-14), s
