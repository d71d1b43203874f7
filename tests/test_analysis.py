"""Host analysis: tau_int and the automatic equilibration detection."""
import numpy as np

from paper_2404_16990_amd import analysis


def _ar1(rng, n, phi):
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


def test_statistical_inefficiency_of_ar1():
    # AR(1): g = (1 + phi) / (1 - phi)
    rng = np.random.default_rng(0)
    phi = 0.8
    x = _ar1(rng, 200000, phi)
    g = analysis.statistical_inefficiency(x)
    assert abs(g - (1 + phi) / (1 - phi)) < 0.5, g


def test_equilibration_finds_the_transient():
    rng = np.random.default_rng(1)
    n = 4000
    x = _ar1(rng, n, 0.5) + 20.0 * np.exp(-np.arange(n) / 150.0)
    t0, g, ne = analysis.equilibration(x)
    # the transient is below the noise after ~150 ln 20 = 450 samples
    assert 250 <= t0 <= 1200, t0
    assert ne > 0.5 * (n - t0) / 3.0


def test_equilibration_keeps_a_stationary_series():
    rng = np.random.default_rng(2)
    x = _ar1(rng, 4000, 0.5)
    t0, g, ne = analysis.equilibration(x)
    assert t0 <= 400, t0


def test_equilibration_of_a_constant_series():
    t0, g, ne = analysis.equilibration(np.ones(100))
    assert t0 == 0 and g == 1.0


def test_batch_means_error_of_ar1():
    """For AR(1) with coefficient phi the error of the mean of n samples is
    sqrt(var * 2 tau / n), tau = (1 + phi) / (2 (1 - phi)); with bins much
    longer than tau the batch-means estimate agrees with it (mean over many
    independent series, so the check is sharp)."""
    rng = np.random.default_rng(5)
    phi, n, bins = 0.9, 40000, 10
    tau = (1 + phi) / (2 * (1 - phi))
    var = 1.0 / (1 - phi * phi)
    want = np.sqrt(var * 2 * tau / n)
    errs = [analysis.batch_means_error(_ar1(rng, n, phi), bins)[1] for _ in range(40)]
    assert abs(np.mean(errs) / want - 1) < 0.1, (np.mean(errs), want)
    # uncorrelated samples: the plain standard error
    x = rng.normal(size=n)
    assert abs(analysis.batch_means_error(x, 20)[1] / (1 / np.sqrt(n)) - 1) < 0.45


def test_replica_agreement_z_follows_its_reference_distribution():
    """Two samplers of the same AR(1) process (tau ~ 50 steps, runs only ~10 tau
    long, where per-chain tau estimates are poor): z from the spread of 8
    independent replicas per group has the spread of Student's t with ~14
    degrees of freedom (variance 14/12), and a shifted sampler is caught."""
    from paper_2404_16990_amd import learned
    rng = np.random.default_rng(2024)
    n_groups, per, n = 400, 8, 500
    phi = 0.96

    def chains(shift):
        x = np.zeros((n_groups * per, n))
        e = rng.standard_normal((n_groups * per, n))
        x[:, 0] = e[:, 0] / np.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[:, t] = phi * x[:, t - 1] + e[:, t]
        return x + shift

    groups = [list(range(g * per, (g + 1) * per)) for g in range(n_groups)]
    z = learned.replica_agreement(chains(0.0), chains(0.0), groups)
    assert 0.85 < np.var(z) < 1.5, np.var(z)
    assert 0.9 < np.mean(np.abs(z) < 2) < 0.97, np.mean(np.abs(z) < 2)
    z_shift = learned.replica_agreement(chains(0.0), chains(3.0), groups)
    assert np.mean(np.abs(z_shift) > 2) > 0.9
