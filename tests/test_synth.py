"""The seeded input generator: deterministic, counter-based, right statistics."""
import numpy as np

import synth

M64 = (1 << 64) - 1


def smix(x):
    """splitmix64 finaliser (Steele, Lea, Flood 2014), written out in Python."""
    x = (x + 0x9E3779B97F4A7C15) & M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M64
    return x ^ (x >> 31)


def test_draw_matches_published_splitmix():
    for seed, g, i, j in [(1, 0, 0, 1), (3, 7, 32767, 5), (2, 0, 8191, 8190)]:
        key = smix(seed ^ ((g * 0x9E3779B97F4A7C15) & M64))
        assert synth.draw(seed, g, i, j) == smix(key ^ ((i << 32) | j))


def test_graph_entries_follow_the_draw():
    W = synth.graph_i32(50, 3, 0.8, 1, 10000)
    thr = int(0.8 * 2 ** 32)
    for i, j in [(0, 1), (7, 3), (49, 0), (12, 40)]:
        x = synth.draw(3, 0, i, j)
        exp = 1 + (((x >> 32) * 10000) >> 32) if (x & 0xFFFFFFFF) < thr else synth.INF_I32
        assert W[i, j] == exp
    assert (np.diag(W) == 0).all()


def test_statistics_and_determinism():
    W = synth.graph_i32(600, 1, 0.5, 1, 1000)
    off = ~np.eye(600, dtype=bool)
    present = (W < synth.INF_I32) & off
    assert abs(present.sum() / off.sum() - 0.5) < 0.01
    assert W[present].min() >= 1 and W[present].max() <= 1000
    np.testing.assert_array_equal(W, synth.graph_i32(600, 1, 0.5, 1, 1000))
    assert not np.array_equal(W, synth.graph_i32(600, 2, 0.5, 1, 1000))
    F = synth.graph_f32(300, 2, 1.0, 0.0, 1.0)
    assert np.isfinite(F).all() and F.min() >= 0 and F.max() < 1
    L = synth.graph_f32(64, 1, 0.5, 0.0, 1.0, ld=80)
    np.testing.assert_array_equal(L[:, :64], synth.graph_f32(64, 1, 0.5, 0.0, 1.0))
    s = synth.batch_sizes()
    assert s.min() >= 16 and s.max() <= 256 and len(s) == 4096
    z = synth.normal_f32(200, 200, 5)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
