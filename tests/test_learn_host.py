"""Host tests of the learned-correction data plumbing (index bookkeeping only, CPU tensors)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2501_06717_amd import learn


def face_index(d, i, j, z):
    return ((z * 8 + j) * 9 + i) if d == 0 else (((z * 9 + j) * 8 + i) if d == 1 else ((z * 8 + j) * 8 + i))


def per_block_faces(nb, fn):
    """Per-block face arrays [nb^3 * 3 * 576, 1] with value fn(d, X, Y, Z) at global face positions."""
    out = np.zeros((nb, nb, nb, 3, 576, 1))
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                for d in range(3):
                    ext = [8, 8, 8]
                    ext[d] = 9
                    for z in range(ext[2]):
                        for y in range(ext[1]):
                            for x in range(ext[0]):
                                out[bz, by, bx, d, face_index(d, x, y, z), 0] = fn(d, 8 * bx + x, 8 * by + y, 8 * bz + z)
    return torch.from_numpy(out.reshape(-1, 1))


def test_global_roundtrip_and_restriction_by_k():
    nb = 2
    U = torch.arange(8 * nb ** 3 * 512, dtype=torch.float64).reshape(8, nb ** 3, 8, 8, 8)
    G = learn.to_global(U, nb)
    assert torch.equal(learn.from_global(G, nb), U)
    # block 1 is bx = 1: its cell (k, j, i) is global (z=k, y=j, x=8+i)
    assert G[3, 2, 5, 8 + 4] == U[3, 1, 2, 5, 4]
    R = learn.restrict_by(U, nb, 2)
    Gr = learn.to_global(R, 1)
    assert torch.isclose(Gr[0, 1, 2, 3], G[0, 2:4, 4:6, 6:8].mean())


@pytest.mark.parametrize("d", [0, 1, 2])
def test_low_faces_cover_each_face_once(d):
    """Per-block faces of direction d at positions 0..7 along d: 512 per block, and together with the
    domain's high-side faces every global face position exactly once."""
    nb = 2
    F = per_block_faces(nb, lambda dd, X, Y, Z: X + 100.0 * Y + 10000.0 * Z).reshape(-1)
    rows = learn.low_faces(nb ** 3, d)
    assert rows.numel() == nb ** 3 * 512
    vals = F[rows].numpy()
    assert len(np.unique(vals)) == len(vals)
    N = 8 * nb
    pos = [np.arange(N)] * 3
    X, Y, Z = np.meshgrid(*pos, indexing="ij")
    assert set(vals.tolist()) == set((X + 100.0 * Y + 10000.0 * Z).reshape(-1).tolist())


@pytest.mark.parametrize("d", [0, 1, 2])
def test_face_pairs_are_the_two_faces_of_a_cell(d):
    nb = 2
    fn = lambda dd, X, Y, Z: X + 100.0 * Y + 10000.0 * Z
    F = per_block_faces(nb, fn).reshape(-1)
    lo, hi = learn.face_pairs(nb ** 3, d)
    assert lo.numel() == hi.numel() == nb ** 3 * 512
    step = [1.0, 100.0, 10000.0][d]
    assert torch.equal(F[hi] - F[lo], torch.full((lo.numel(),), step, dtype=F.dtype))
    assert len(np.unique(F[lo].numpy())) == lo.numel()


def test_strength_scales_only_the_output_statistics():
    stats = torch.arange(80, dtype=torch.float32) + 1.0
    s = learn.with_strength(stats, 0.25)
    assert torch.equal(s[:64], stats[:64])
    assert torch.equal(s[64:], 0.25 * stats[64:])
    assert torch.equal(stats, torch.arange(80, dtype=torch.float32) + 1.0)  # the input is not modified


def test_saved_network_is_plain_arrays(tmp_path):
    class Net:
        p = torch.linspace(-1.0, 1.0, 11)
    cfg = learn.Config(hidden=32, strength=0.5)
    path = str(tmp_path / "net.npz")
    learn.save(path, Net(), torch.ones(80), cfg, {"gain_mean": 1.03})
    d = np.load(path, allow_pickle=False)
    assert np.array_equal(d["params"], Net.p.numpy()) and d["params"].dtype == np.float32
    assert int(d["hidden"]) == 32 and float(d["strength"]) == 0.5
    assert '"gain_mean": 1.03' in str(d["summary"])


def test_shipped_network_file():
    import os
    path = os.path.join(os.path.dirname(learn.__file__), "trained", "flux_mlp_h128.npz")
    d = np.load(path, allow_pickle=False)
    assert int(d["hidden"]) == 128 and d["params"].shape == (38280,) and d["stats"].shape == (80,)
    assert np.all(np.isfinite(d["params"])) and np.all(d["stats"][32:64] > 0) and np.all(d["stats"][72:80] > 0)
