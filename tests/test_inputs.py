"""The seeded input recipes: determinism, ranges, and agreement of the
device-side (torch) evaluation with the numpy one."""
import numpy as np
import torch

from paper_1110_0740_amd import inputs as I


def test_splitmix64_reference_values():
    # SplitMix64 outputs for seed 0 (Steele, Lea & Flood 2014 reference stream)
    r = I.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_recipes_deterministic_and_in_range():
    V1, _ = I.mhd3d_fields(n=8, ng=4, seed=2000)
    V2, _ = I.mhd3d_fields(n=8, ng=4, seed=2000)
    assert np.array_equal(V1, V2)
    assert V1[0].min() >= 0.5 - 1e-12 and V1[0].max() <= 1.5 + 1e-12
    V, _ = I.mhd2d_fields(n=16, ng=4, seed=1000)
    assert np.abs(V[5:7]).max() <= 0.5 + 1e-12
    Vr, _ = I.rmhd3d_fields(n=16, ng=4, seed=4000)
    v2 = (Vr[1:4] ** 2).sum(0)
    assert v2.max() < 1.0
    lor = 1 / np.sqrt(1 - v2)
    assert lor.max() <= 10.0 + 1e-9


def test_torch_evaluation_matches_numpy():
    Vn, _ = I.mhd3d_fields(n=10, ng=4, seed=2000)
    Vt, _ = I.mhd3d_fields_torch(n=10, ng=4, seed=2000, device="cpu")
    assert np.max(np.abs(Vt.numpy() - Vn)) < 1e-12


def test_periodic_ghosts_equal_images():
    V, _ = I.mhd3d_fields(n=8, ng=4, seed=2000)
    W = V.copy()
    I.fill_periodic(W, 4, 3)
    assert np.max(np.abs(W - V)) < 1e-12


def test_amr_fields_torch_matches_numpy():
    h = I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16))
    for lev in (0, 1, 2):
        if not h.levels[lev]:
            continue
        B = h.levels[lev][0]
        Vn = I.amr_fields(h, B, 4)
        Vt = I.amr_fields_torch(h, B, 4, device="cpu")
        assert np.max(np.abs(Vt.numpy() - Vn)) < 1e-12


def test_amr_level_fields_torch_matches_numpy():
    """the level-at-once generator packs every box's amr_fields block in box
    order"""
    h = I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16))
    for lev in range(len(h.levels)):
        flat = I.amr_level_fields_torch(h, lev, 4, device="cpu").numpy()
        o = 0
        for B in h.levels[lev]:
            Vn = I.amr_fields(h, B, 4)
            assert np.max(np.abs(flat[o:o + Vn.size].reshape(Vn.shape) - Vn)) < 1e-12
            o += Vn.size
        assert o == flat.size


def test_cooling_time_torch_matches_numpy():
    import torch

    n, ng = 12, 4
    X, Y, Z = I.cell_centres(I.Box((0, 0, 0), (n, n, n)), ng, (1.0 / n,) * 3, 3)
    a = I.cooling_time_field(5002, X, Y, Z, 0.25)
    b = I.cooling_time_field_torch(5002, n, ng, 0.25, device="cpu").numpy()
    assert np.allclose(a, b, rtol=1e-12, atol=0)
    assert a.min() >= 0.25e-3 * (1 - 1e-12) and a.max() <= 0.25e3 * (1 + 1e-12)


def test_white_cooling_times_follow_splitmix64_and_periodicity():
    """the vectorised draw is the SplitMix64 sequence; the cooling times span
    [1e-3, 1e3] dt0 and the ghosts repeat their periodic images"""
    rng = I.SplitMix64(77)
    seq = [rng.uniform() for _ in range(20)]
    assert np.array_equal(I.splitmix64_uniform(77, np.arange(20)), np.array(seq))
    n, ng = 10, 4
    tc = I.cooling_time_white(5003, n, ng, 2.0)
    assert tc.min() >= 2e-3 and tc.max() <= 2e3 and tc.min() < 2e-2 and tc.max() > 2e2
    W = tc[None].copy()
    I.fill_periodic(W, ng, 3)
    assert np.array_equal(W[0], tc)
    # a sub-box sees the same cells as the whole box
    sub = I.cooling_time_white(5003, n, ng, 2.0, box=I.Box((2, 3, 1), (4, 5, 6)), level_n=n)
    assert np.array_equal(sub, tc[1:1 + 6 + 2 * ng, 3:3 + 5 + 2 * ng, 2:2 + 4 + 2 * ng])
