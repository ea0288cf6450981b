"""Statistical pin of the oracle (two-Gaussian example of the Background section).

With A and B drawn from the same distribution, d(x, a) and d(x, b) are
exchangeable, so E[D] = 1/2 exactly.  As the second Gaussian moves away the
error must fall.  The figure's own values are not printed in the paper, so
the curve itself stays "parity unpinned"; only these two properties are.
"""
import numpy as np

import oracle
import workloads


def _error(mu, seed, n=24):
    w = workloads.gaussians_2d(mu, n, seed)
    res = oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across)
    return oracle.error_rate(res)


def test_same_distribution_is_chance():
    errs = np.array([_error(0.0, s) for s in range(60)])
    mean, sem = errs.mean(), errs.std(ddof=1) / np.sqrt(len(errs))
    assert abs(mean - 0.5) < 2.58 * sem + 1e-12      # 99% interval


def test_error_falls_with_shift():
    mus = [0.0, 0.5, 1.0, 2.0, 4.0]
    means = [np.mean([_error(mu, 1000 + s) for s in range(30)]) for mu in mus]
    assert all(b < a for a, b in zip(means, means[1:])), means
    # class 0 is isotropic around the origin, so under the angular distance the
    # error levels off well above 0 (about 0.27 at mu = 4); it must still be far below chance
    assert means[-1] < 0.35
