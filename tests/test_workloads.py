"""Seeded input generators: determinism, recipe statistics, load totals."""
import numpy as np

import workloads as W


def test_density_recipes_deterministic_and_bounded():
    a = W.density_uniform_noise((120, 40), 1)
    b = W.density_uniform_noise((120, 40), 1)
    assert np.array_equal(a, b) and a.shape == (4800,)
    assert a.min() >= W.RHO_MIN and a.max() <= 1.0
    assert abs(a.mean() - 0.5) < 0.01


def test_volume_fraction_recipe():
    x = W.density_volume_fraction((48, 16, 16), 3, 0.3, 4.0)
    assert abs(x.mean() - 0.3) < 1e-12
    assert x.min() >= W.RHO_MIN and x.max() == 1.0
    xs = x.reshape(16, 16, 48)
    assert np.all(xs[..., :2] == 1.0) and np.all(xs[..., -2:] == 1.0)


def test_loads_and_masks():
    for nel in [(8, 4), (4, 2, 6)]:
        d = len(nel)
        f = W.axial_load(nel)
        assert abs(f.sum() + 1.0) < 1e-15
        assert np.all(f[1::d] == 0)
        m = W.clamp_mask(nel)
        assert m.sum() == d * np.prod([v + 1 for v in nel[1:]])
        assert np.all(f[m != 0] == 0)
    nel = (4, 4, 6)
    t = W.torsion_load(nel)
    nodes = np.flatnonzero(np.abs(t[1::3]) + np.abs(t[2::3]))
    j = (nodes // 5) % 5
    k = nodes // 25
    mom = np.sum((j - 2.0) * t[3 * nodes + 2] - (k - 3.0) * t[3 * nodes + 1])
    assert abs(mom - 1.0) < 1e-14 and abs(t.sum()) < 1e-14


def test_instances_2d():
    inst = W.small_instances_2d()
    assert len(inst) == 32
    assert inst[0]["nel"] == (64, 32) and inst[1]["nel"] == (512, 128)
    for p in inst:
        nx, ny = p["nel"]
        assert ny <= nx // 2
