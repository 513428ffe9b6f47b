"""The seeded workload generators: determinism, shapes and distributions
(CPU only)."""
import numpy as np

from synth import scenes


def test_c0_deterministic_and_distributed():
    a = scenes.make_c0()
    b = scenes.make_c0()
    assert scenes.digest(a.scene.arrays()) == scenes.digest(b.scene.arrays())
    sc = a.scene
    assert sc.means.shape == (2000, 3) and sc.means.dtype == np.float32
    assert np.all(np.abs(sc.means) <= 0.5)
    ls = np.log(sc.scales.astype(np.float64))
    assert abs(ls.mean() + 4.0) < 0.05 and abs(ls.std() - 0.5) < 0.03
    np.testing.assert_allclose(np.linalg.norm(sc.quats, axis=1), 1.0, atol=1e-6)
    assert np.all((sc.opacity > 0) & (sc.opacity < 1))
    rgb = sc.sh[:, 0, :] * (0.5 / np.sqrt(np.pi)) + 0.5
    assert rgb.min() > -1e-6 and rgb.max() < 1 + 1e-6
    v = a.views[0]
    assert (v.width, v.height) == (128, 128)
    np.testing.assert_allclose(v.fx, 64 / np.tan(np.pi / 6), rtol=1e-12)
    np.testing.assert_allclose(-v.R.T @ v.t, [0, 0, -3], atol=1e-6)
    assert a.targets["rgb"][0].shape == (3, 128 * 128)


def test_c2_anchor_structure():
    wl = scenes.make_c2()
    sc = wl.scene
    assert sc.n == 200_000
    counts = np.bincount(sc.level, minlength=4)
    assert counts.tolist() == [2352, 9411, 37647, 150590]     # 1:4:16:64 split, floor + remainder
    assert np.all(counts[1:] > counts[:-1])
    size = 6.4 / 2.0 ** sc.level
    np.testing.assert_allclose(sc.l[:, 0], size, rtol=1e-6)
    # anchors sit on their level's grid (Eq. 2)
    g = sc.x / size[:, None]
    np.testing.assert_allclose(g, np.round(g), atol=1e-3)
    assert sc.F.shape == (200_000, 32) and sc.O.shape == (200_000, 10, 3)
    assert sc.W1_bits.shape == (36, 32) and sc.W2_bits.shape == (32, 110)
    assert len(wl.views) == 8
    for v in wl.views:
        assert 960 <= v.width <= 1920 and 540 <= v.height <= 1080
        assert v.width % 2 == 0 and v.height % 2 == 0
    b = scenes.make_c2()
    assert scenes.digest(sc.arrays()) == scenes.digest(b.scene.arrays())


def test_small_scenes_deterministic():
    a = scenes.make_small_anchor(3)
    b = scenes.make_small_anchor(3)
    assert scenes.digest(a.scene.arrays()) == scenes.digest(b.scene.arrays())
    c = scenes.make_small_explicit(4, sh_degree=3)
    assert c.scene.sh.shape == (40, 16, 3)


def test_bf16_bits_roundtrip():
    x = np.array([1.0, -2.5, 0.1, 3.0e-3], np.float32)
    v = scenes.bf16_value(scenes.bf16_bits(x))
    np.testing.assert_allclose(v, x, rtol=2 ** -8)
    exact = np.array([1.0, -2.5, 0.15625], np.float32)
    np.testing.assert_array_equal(scenes.bf16_value(scenes.bf16_bits(exact)), exact)
