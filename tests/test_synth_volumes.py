"""The served workload's large-volume generator (synth.volumes), on the CPU.

It is input generation, not the method, so it is pinned against what the recipe fixes: any box
generated on its own equals the same cut of a larger box (tiles are reproducible), the counter-based
Poisson draws have the Poisson distribution (moments and a chi-square fit against scipy's pmf), the
SplitMix64 stream matches its published reference values, the per-block densities stay in range,
and the packing keeps bounding spheres within the overlap limit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth.volumes import LargeVolume, counter_bits, counter_poisson, counter_uniform, fast_subvolume_batch, pack_block


def test_splitmix64_reference_values():
    """SplitMix64 seeded with 1234567 (state advanced by the golden gamma before each output):
    the first outputs of the reference generator, computed here with Python integers."""
    M = (1 << 64) - 1

    def ref(state, n):
        out = []
        for _ in range(n):
            state = (state + 0x9E3779B97F4A7C15) & M
            z = state
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            out.append(z ^ (z >> 31))
        return out

    want = ref(1234567, 5)
    # counter i (1-based) is the state after i advances
    got = [v & M for v in counter_bits(1234567, torch.arange(1, 6, dtype=torch.int64)).tolist()]
    assert got == want
    u = counter_uniform(1234567, torch.arange(1, 6, dtype=torch.int64))
    assert torch.equal(u, torch.tensor([((w >> 11) + 0.5) * 2.0 ** -53 for w in want], dtype=torch.float64))
    # the check values published with the generator's reference implementation for seed 1234567
    assert want == [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
                    16408922859458223821]


@pytest.mark.parametrize("lam", [10.0, 70.0, 100.0, 530.0, 1000.0])
def test_counter_poisson_distribution(lam):
    from scipy.stats import poisson
    n = 400_000
    k = counter_poisson(torch.full((n,), lam, dtype=torch.float64), torch.arange(n), 0xC0FFEE).numpy()
    assert abs(k.mean() - lam) < 5.0 * np.sqrt(lam / n)
    assert abs(k.var() / lam - 1.0) < 5.0 * np.sqrt(2.0 / n) + 0.01
    # chi-square over the central bins (expected count >= 50 each), tails pooled
    lo, hi = int(poisson.ppf(1e-3, lam)), int(poisson.ppf(1 - 1e-3, lam))
    obs = np.array([np.sum(k < lo)] + [np.sum(k == v) for v in range(lo, hi + 1)] + [np.sum(k > hi)], np.float64)
    exp = n * np.concatenate([[poisson.cdf(lo - 1, lam)], poisson.pmf(np.arange(lo, hi + 1), lam),
                              [poisson.sf(hi, lam)]])
    ok = exp >= 50
    chi2 = float(np.sum((obs[ok] - exp[ok]) ** 2 / exp[ok]))
    dof = int(ok.sum()) - 1
    assert chi2 < dof + 5.0 * np.sqrt(2.0 * dof), (chi2, dof)


def test_counter_poisson_refuses_small_means():
    with pytest.raises(ValueError):
        counter_poisson(torch.full((4,), 5.0, dtype=torch.float64), torch.arange(4), 1)


def test_box_equals_cut_of_larger_box():
    V = LargeVolume(0x1804063040000005, shape_xyz=(160, 144, 96))
    whole = V.box((0, 0, 0), (160, 144, 96))
    assert whole.dtype == torch.uint16 and tuple(whole.shape) == (96, 144, 160)
    for lo, hi in (((17, 3, 40), (90, 77, 96)), ((0, 0, 0), (31, 29, 7)), ((120, 100, 50), (160, 144, 96))):
        sub = V.box(lo, hi)
        assert torch.equal(sub, whole[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]), (lo, hi)


def test_objects_density_and_packing():
    V = LargeVolume(7, shape_xyz=(256, 256, 256), block=128)
    ol = V.objects()
    counts = np.diff(ol.block_start)
    assert len(counts) == 8
    assert np.all(counts >= 20) and np.all(counts <= 400)
    assert len(set(counts.tolist())) > 1                     # density varies from block to block
    # the object list is a pure function of the seed
    ol2 = LargeVolume(7, shape_xyz=(256, 256, 256), block=128).objects()
    assert np.array_equal(ol.centers, ol2.centers) and np.array_equal(ol.rots, ol2.rots)
    # within a block bounding spheres overlap by at most 10%
    for b in range(8):
        s, e = ol.block_start[b], ol.block_start[b + 1]
        c = ol.centers[s:e]
        r = ol.axes[s:e].max(axis=1)
        d = np.linalg.norm(c[:, None] - c[None], axis=2)
        np.fill_diagonal(d, np.inf)
        assert np.all(d >= 0.9 * (r[:, None] + r[None]) - 1e-9)
    rot = ol.rots
    assert np.allclose(np.einsum("nij,nik->njk", rot, rot), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(rot), 1.0)


def test_tile_requests():
    V = LargeVolume(11, shape_xyz=(300, 280, 200))
    rng = np.random.default_rng(3)
    for _ in range(20):
        lo, hi, clo, chi, idx = V.tile(rng, 40, 120, 16)
        assert np.all(lo >= 0) and np.all(hi <= np.array(V.shape))
        assert np.all(clo - lo <= 16) and np.all(hi - chi <= 16)
        assert np.all((clo - lo == 16) | (lo == 0)) and np.all((hi - chi == 16) | (hi == np.array(V.shape)))
        c = V.objects().centers[idx]
        assert np.all(c >= clo * V.h) and np.all(c <= (chi - 1) * V.h)
        # every object whose centre lies in the core is found
        allc = V.objects().centers
        inside = np.all((allc >= clo * V.h) & (allc <= (chi - 1) * V.h), axis=1)
        assert set(np.where(inside)[0]) == set(idx.tolist())


def test_nuclei_are_bright():
    """Voxels at nucleus centres are brighter than the background on average (the recipe's
    mean is (100 + 900 * blurred coverage) * gain with gain in [0.7, 1])."""
    V = LargeVolume(5, shape_xyz=(128, 128, 64))
    vol = V.box((0, 0, 0), (128, 128, 64)).to(torch.int32).numpy()
    c = V.objects().centers
    ijk = np.rint(c / V.h).astype(int)
    ok = np.all((ijk >= 0) & (ijk < np.array(V.shape)), axis=1)
    at_centres = vol[ijk[ok, 2], ijk[ok, 1], ijk[ok, 0]]
    assert at_centres.mean() > 500.0
    assert np.median(vol) < 400.0


def test_fast_subvolumes():
    vols = list(fast_subvolume_batch(99, n_vol=3, edge_lo=32, edge_hi=48))
    assert len(vols) == 3
    for e, raw, c, a, r, small in vols:
        assert tuple(raw.shape) == (e, e, e) and raw.dtype == torch.uint16
        assert len(c) >= 1
        rad = a.max(axis=1)
        ext = (e - 1) * np.array([1.0, 1.0, 2.0])
        assert np.all(c - rad[:, None] >= 0.0) and np.all(c + rad[:, None] <= ext)
    again = list(fast_subvolume_batch(99, n_vol=3, edge_lo=32, edge_hi=48))
    for x, y in zip(vols, again):
        assert torch.equal(x[1], y[1])


def test_pack_block_respects_target():
    rng = np.random.default_rng(1)
    c, a, r = pack_block(rng, 50, np.zeros(3), np.array([100.0, 100.0, 100.0]))
    assert len(c) == 50
    assert np.all(a >= 3.0) and np.all(a <= 10.0)
