"""Host checks of the figures of merit (Sec. 4.2-4.3, eqs. (11)-(13))."""
import numpy as np

from paper_2106_01275_amd import analysis


def test_sample_variance_real_and_complex():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(50)
    assert np.isclose(analysis.sample_variance(x), np.var(x, ddof=1))
    z = x + 1j * rng.standard_normal(50)
    assert np.isclose(analysis.sample_variance(z), np.var(z.real, ddof=1) + np.var(z.imag, ddof=1))


def test_speedups_are_cost_normalised_variance_ratios():
    # one probed sample costs m solves: equal variance per solve means speed-up 1
    assert np.isclose(analysis.speedup_over_hutchinson(8.0, 1.0, 8), 1.0)
    assert np.isclose(analysis.speedup_over_cp(2.0, 16, 1.0, 32), 1.0)
    # eq. (13) is invariant under (var, m_p) -> (var * c, m_p / c): same variance per unit of work
    a = analysis.normalized_relative_error(0.5, 100, 815, 2.0)
    assert np.isclose(a, analysis.normalized_relative_error(5.0, 10, 815, 2.0))
    assert np.isclose(a, np.sqrt(0.5 * 100 / 815) / 2.0)
