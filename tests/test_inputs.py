"""Seeded input generators: reproducible, mean density 1, the requested spread, and AMR
layouts that satisfy the library's patch rules (CPU only)."""
import numpy as np

from paper_1110_1379_amd import inputs


def test_gaussian_field_moments_and_seed():
    g = inputs.gaussian_field(32, 2.0, -1.5, seed=7)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 2.0) < 1e-12
    assert np.array_equal(g, inputs.gaussian_field(32, 2.0, -1.5, seed=7))
    assert not np.array_equal(g, inputs.gaussian_field(32, 2.0, -1.5, seed=8))


def test_workload_densities_have_unit_mean():
    for rho in (inputs.small_box(16, 0), inputs.tophat_box(32, 1, count=3), inputs.halo_box(32, 2, count=2)):
        assert abs(rho.mean() - 1.0) < 1e-12
        assert np.isfinite(rho).all() and rho.min() > 0


def test_halos_reach_their_peak_amplitude():
    base = inputs.lognormal(64, 3.0, -1.5, 2)
    rho = inputs.add_nfw_halos(base.copy(), 3, seed=2, peak_min=5e3, peak_max=5e3)
    assert (rho - base).max() > 0.5 * 5e3


def _check_layout(N0, patches, rho_packed):
    by_level = {}
    ends = []
    for i, p in enumerate(patches):
        n, o = p["n"], p["origin"]
        assert n & (n - 1) == 0 and 8 <= n <= 64
        assert all(x % 2 == 0 for x in o)
        side = N0 * 2 ** p["level"]
        assert all(0 <= x and x + n <= side for x in o)
        if p["level"] == 1:
            assert p["parent"] == -1
        else:
            q = patches[p["parent"]]
            assert q["level"] == p["level"] - 1
            for d in range(3):
                assert o[d] // 2 - 1 >= q["origin"][d]
                assert (o[d] + n) // 2 <= q["origin"][d] + q["n"] - 1
        by_level.setdefault(p["level"], []).append(p)
        ends.append((p["offset"], p["offset"] + n ** 3))
    ends.sort()
    assert ends[0][0] == 0 and ends[-1][1] == rho_packed.size
    assert all(a[1] <= b[0] for a, b in zip(ends, ends[1:]))
    for ps in by_level.values():
        for a in range(len(ps)):
            for b in range(a + 1, len(ps)):
                A, B = ps[a], ps[b]
                assert any(A["origin"][d] + A["n"] <= B["origin"][d] or B["origin"][d] + B["n"] <= A["origin"][d]
                           for d in range(3))


def test_amr_layout_follows_the_patch_rules():
    rho0, patches, rho_packed = inputs.amr_workload(64, seed=3, thresholds=(10.0, 40.0, 150.0), sizes=(16, 8, 4))
    assert len(patches) > 5 and max(p["level"] for p in patches) >= 2
    _check_layout(64, patches, rho_packed)
    assert np.isfinite(rho_packed).all() and rho_packed.min() > 0


def test_patch_density_samples_the_same_field():
    """The patch density is the domain recipe evaluated at the finer cell centres: its 2x2x2
    block means track the parent cells it refines."""
    rho0, patches, rho_packed = inputs.amr_workload(32, seed=3, thresholds=(3.0,), sizes=(4,))
    p = patches[0]
    n = p["n"]
    blk = rho_packed[p["offset"]:p["offset"] + n ** 3].reshape((n,) * 3)
    means = blk.reshape(n // 2, 2, n // 2, 2, n // 2, 2).mean(axis=(1, 3, 5))
    o = [x // 2 for x in p["origin"]]
    parent = rho0[o[0]:o[0] + n // 2, o[1]:o[1] + n // 2, o[2]:o[2] + n // 2]
    assert np.corrcoef(means.ravel(), parent.ravel())[0, 1] > 0.9


def test_batch_boxes_parameters():
    boxes = inputs.batch_boxes(n64=3, n128=1)
    assert [b[0] for b in boxes] == [64, 64, 64, 128]
    for N, B, fr0, sigma, seed, rho in boxes:
        assert 1e-6 <= fr0 <= 1e-4 and 1.0 <= sigma <= 3.0 and B == float(N)
        assert abs(rho.mean() - 1.0) < 1e-12


def test_oct_mask_is_oct_aligned_and_buffered():
    rho = inputs.small_box(32, 4)
    od = rho.reshape(16, 2, 16, 2, 16, 2).mean(axis=(1, 3, 5))
    thr = float(np.quantile(od, 0.95))
    m0 = inputs.oct_mask(rho, thr, expand=0)
    m1 = inputs.oct_mask(rho, thr, expand=1)
    for m in (m0, m1):
        assert set(np.unique(m)) <= {-1.0, 1.0}
        blocks = m.reshape(16, 2, 16, 2, 16, 2)
        assert np.all(blocks.min(axis=(1, 3, 5)) == blocks.max(axis=(1, 3, 5)))
    # without the buffer exactly the octs above the threshold; the buffer only adds cells,
    # and every added oct touches a refined one
    assert np.array_equal(m0[::2, ::2, ::2] > 0, od > thr)
    assert np.all(m1[m0 > 0] > 0) and (m1 > 0).sum() > (m0 > 0).sum()
    o0, o1 = m0[::2, ::2, ::2] > 0, m1[::2, ::2, ::2] > 0
    near = np.zeros_like(o0)
    for s in np.ndindex(3, 3, 3):
        near |= np.roll(o0, tuple(x - 1 for x in s), axis=(0, 1, 2))
    assert np.array_equal(o1, near)
