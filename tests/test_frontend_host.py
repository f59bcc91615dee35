"""The automatic frequency grid (host logic): the grid the paper's benchmarks
use (Sec. 2: the Astropy default, N_f ~ 12 N_d), checked against its
definition -- step 1 / (samples_per_peak * baseline), start at half a step,
end at nyquist_factor times the average Nyquist frequency N / (2 baseline)."""
import numpy as np
import pytest

from paper_2409_08090_amd import mils


@pytest.mark.parametrize("nd", [100, 1000, 10_000, 1_000_000])
def test_default_grid_has_about_twelve_frequencies_per_point(nd):
    rng = np.random.default_rng(nd)
    t = np.sort(rng.uniform(0.0, 3650.0, nd))
    T = t.max() - t.min()
    f0, df, nf = mils.autofrequency(t)
    assert df * 5.0 * T == pytest.approx(1.0, rel=1e-15)
    assert f0 == 0.5 * df
    fmax = 5.0 * 0.5 * nd / T
    assert abs(f0 + (nf - 1) * df - fmax) <= 0.5 * df + 1e-12 * fmax
    assert 12 * nd <= nf <= 13 * nd  # the paper's N_f ~ 12 N_d


def test_explicit_limits_and_factors():
    t = np.linspace(10.0, 110.0, 501)  # baseline 100
    f0, df, nf = mils.autofrequency(t, samples_per_peak=10, minimum_frequency=0.2,
                                    maximum_frequency=1.0)
    assert df == pytest.approx(1e-3) and f0 == 0.2
    assert nf == 801 and f0 + (nf - 1) * df == pytest.approx(1.0)
    f0, df, nf = mils.autofrequency(t, nyquist_factor=1.0)
    assert f0 + (nf - 1) * df == pytest.approx(0.5 * 501 / 100.0, abs=df / 2)


def test_shift_invariance_and_tensor_input():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0.0, 50.0, 300))
    a = mils.autofrequency(t)
    b = mils.autofrequency(t + 1e4)
    assert a[2] == b[2] and a[1] == pytest.approx(b[1], rel=1e-9)
    assert mils.autofrequency(torch.from_numpy(t)) == a


@pytest.mark.parametrize("t,kw", [([1.0], {}), ([2.0, 2.0, 2.0], {}), ([0.0, np.inf], {}),
                                  ([0.0, 1.0], {"samples_per_peak": 0}),
                                  ([0.0, 1.0], {"minimum_frequency": 2.0,
                                                "maximum_frequency": 1.0})])
def test_invalid_inputs(t, kw):
    with pytest.raises(ValueError):
        mils.autofrequency(np.asarray(t), **kw)
