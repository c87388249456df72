"""Host logic of the training driver (no GPU): early stopping and datasets."""
import numpy as np

from paper_2304_12745_amd import train as T
from paper_2304_12745_amd import workloads as WL


def test_early_stopping_keeps_the_lowest_and_stops_after_patience():
    es = T.EarlyStopping(3)
    costs = [5.0, 4.0, 4.5, 3.0, 3.0, 3.2, 3.1, 2.0]
    best_flags = []
    stopped_at = None
    for ep, c in enumerate(costs):
        best_flags.append(es.update(ep, c))
        if es.stop:
            stopped_at = ep
            break
    assert best_flags == [True, True, False, True, False, False, False]
    assert stopped_at == 6 and es.best_epoch == 3 and es.best_cost == 3.0


def test_early_stopping_never_stops_while_improving():
    es = T.EarlyStopping(1)
    for ep in range(50):
        assert es.update(ep, 100.0 - ep)
        assert not es.stop


def test_datasets_are_seeded_independent_rayleigh_draws():
    a = WL.ufpgd_datasets(64, 16, 16, seed=3)
    b = WL.ufpgd_datasets(64, 16, 16, seed=3)
    c = WL.ufpgd_datasets(64, 16, 16, seed=4)
    np.testing.assert_array_equal(a.train, b.train)
    assert not np.array_equal(a.train, c.train)
    assert a.train.dtype == np.complex64 and a.train.shape == (64, 8, 64)
    assert not np.array_equal(a.val[:1], a.test[:1])
    np.testing.assert_allclose(a.gamma_lin, 10.0)
    big = WL.ufpgd_datasets(4000, 1, 1, seed=0).train
    assert abs(np.mean(np.abs(big) ** 2) - 1.0) < 0.01        # CN(0, 1)
