"""The CPU oracle against its pins (no GPU)."""
import numpy as np
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc.default())


def test_determinism_and_permutation(orc):
    import workloads

    W = workloads.make(2, N=3000, M=8)
    o = orc.default()
    a = o.lagp(W.X, W.Y, W.XX, 6, 20, 200, W.d, W.g, threads=1)
    b = o.lagp(W.X, W.Y, W.XX, 6, 20, 200, W.d, W.g, threads=4)
    perm = np.random.default_rng(1).permutation(W.M)
    c = o.lagp(W.X, W.Y, W.XX[perm], 6, 20, 200, W.d, W.g, threads=3)
    for k in ("pool", "sel", "mean", "s2", "var", "dsel"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
        assert np.array_equal(a[k][perm], c[k], equal_nan=True), k


def test_bad_forced_sequence(orc):
    import workloads

    W = workloads.make(2, N=500, M=2)
    o = orc.default()
    a = o.lagp(W.X, W.Y, W.XX, 6, 12, 60, W.d, W.g)
    f = a["sel"].copy()
    f[0, 8] = f[0, 7]  # repeats a design point
    f[1, 9] = int(np.setdiff1d(np.arange(W.N), a["pool"][1])[0])  # outside the pool
    b = o.alc(W.X, W.Y, W.XX, a["pool"], 6, 12, W.d, W.g, forced=f)
    assert list(b["status"]) == [4, 4]
    assert np.all(np.isnan(b["mean"]))


def test_bad_args(orc):
    import workloads

    W = workloads.make(2, N=500, M=2)
    o = orc.default()
    with pytest.raises(ValueError):
        o.nn_pool(W.X, W.XX, W.N + 1)
    with pytest.raises(ValueError):
        o.lagp(W.X, W.Y, W.XX, 6, 12, 60, -1.0, W.g)
