"""Host-side checks of the seeded workload generators against their recipes (CPU)."""

import numpy as np

from paper_2509_24742_amd import workloads as wl


def test_uneven_batch_follows_its_recipe():
    systems = wl.uneven_batch(place=False)
    assert len(systems) == 32
    N = np.array([w["n_total"] for w in systems])
    assert N.min() >= 2000 and N.max() <= 200000
    for w in systems:
        p = w["params"]
        n_ele, n_ion = len(w["ele_side"]), len(w["ion_q"])
        n = int(round(np.sqrt(n_ele / 2)))
        assert n_ele == 2 * n * n and n == int(round(np.sqrt(0.075 * w["n_total"])))
        assert n_ion % 2 == 0 and abs(np.sum(w["ion_q"])) < 1e-12 * np.sum(np.abs(w["ion_q"]))
        aspect = 3.0 * p["H"] / p["Lx"]
        assert 3.0 <= aspect <= 12.0 and p["M"] == int(np.ceil(aspect))
        assert np.isclose(n_ion / (p["Lx"] * p["Ly"] * p["H"]), 10.0, rtol=1e-12)
        assert p["P"] == int(round(100 * np.sqrt(w["n_total"] / 1e4)))
        # two complete square walls at z = 0 and z = H, spacing Lx / n
        z = w["ele_pos"][:, 2]
        assert np.all((z == 0.0) | (z == p["H"])) and np.sum(z == 0.0) == n * n
        xs = np.unique(np.round(w["ele_pos"][z == 0.0, 0] / (p["Lx"] / n) - 0.5, 9))
        assert np.array_equal(xs, np.arange(n))


def test_uneven_batch_places_systems_independently():
    a = wl.uneven_batch(place={10})[10]
    b = wl.uneven_batch(place={10, 16})[10]
    assert np.array_equal(a["ion_pos"], b["ion_pos"])
    p = a["params"]
    z = a["ion_pos"][:, 2]
    assert z.min() >= 0.4 and z.max() <= p["H"] - 0.4


def test_large_slab_recipe_at_small_size():
    w = wl.large_slab(n_side=16, n_ion=2000, Lx=3.2, H=20.0, M=8, P=50)
    assert len(w["ele_side"]) == 512 and len(w["ion_q"]) == 2000 and abs(np.sum(w["ion_q"])) < 1e-12
    from scipy.spatial import cKDTree
    d, _ = cKDTree(w["ion_pos"], boxsize=(3.2, 3.2, 1e3)).query(w["ion_pos"], k=2)
    assert d[:, 1].min() >= 0.3
