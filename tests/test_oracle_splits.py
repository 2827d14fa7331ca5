"""Pins of the oracle's stopping rule and split handling."""
import numpy as np

from oracle import oracle as O
from paper_2602_02759_amd import datagen


def test_rule_on_hand_made_sequences():
    L = [10.0, 9.0, 8.0, 7.9, 7.8, 7.7, 7.6]
    V = [5.0, 4.0, 4.1, 4.2, 4.3, 4.4, 4.5]  # rises from t = 2 on
    assert O.stop_reason(5, L, V, 5, 1e-6, 100) is None   # four rises so far
    assert O.stop_reason(6, L, V, 5, 1e-6, 100) == O.STOP_VALIDATION
    assert O.stop_reason(6, L, None, 5, 1e-6, 100) is None
    assert O.stop_reason(6, L, V, 0, 1e-6, 100) is None   # patience 0 disables
    assert O.stop_reason(3, L, V, 5, 0.05, 100) == O.STOP_TRAIN_TOL  # 0.1 / 8 < 5 %
    assert O.stop_reason(2, L, V, 5, 0.05, 100) is None             # 1 / 9 > 5 %
    assert O.stop_reason(6, L, V, 7, 1e-6, 6) == O.STOP_MAX
    assert O.stop_reason(0, [1.0], [1.0], 5, 1e-6, 0) == O.STOP_MAX
    # a rising training loss also stops on the tolerance rule
    assert O.stop_reason(1, [1.0, 1.1], None, 5, 1e-6, 10) == O.STOP_TRAIN_TOL


def test_split_mask_fractions():
    m = datagen.split_mask((200, 300), seed=3)
    n = m.size
    assert abs((m == 3).sum() / n - 0.10) < 0.01
    assert abs((m == 2).sum() / n - 0.9 * 0.05) < 0.005
    assert set(np.unique(m)) == {1, 2, 3}


def test_fit_uses_training_entries_only():
    """Values at validation and heldout entries never change the fit; the
    returned losses are those of the returned state."""
    p = datagen.cp3(1.0, 0.0, sizes=dict(i=9, j=8, k=7), R=3, seed=5, missing=0.0)
    M = datagen.split_mask(p.Y.shape, seed=5)
    Y2 = p.Y.copy()
    Y2[M != 1] = 1e6
    a = O.fit_early_stopping(p.model_str, p.init, p.Y, M, 1.0, 0.0, max_sweeps=8, val_value=0)
    b = O.fit_early_stopping(p.model_str, p.init, Y2, M, 1.0, 0.0, max_sweeps=8, val_value=0)
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    assert a[1] == 8 and a[2] == O.STOP_MAX
    Mt = (M == 1).astype(np.uint8)
    assert a[3][-1] == O.loss(p.model_str, a[0], p.Y, Mt, 1.0, 0.0)


def test_fit_stops_on_tolerance_and_on_validation():
    p = datagen.cp3(1.0, 0.0, sizes=dict(i=10, j=9, k=8), R=4, seed=6, missing=0.0)
    M = datagen.split_mask(p.Y.shape, seed=6, validation=0.2)
    f, t, r, L, V = O.fit_early_stopping(p.model_str, p.init, p.Y, M, 1.0, 0.0, max_sweeps=500,
                                         patience=0, rel_tol=1e-3)
    assert r == O.STOP_TRAIN_TOL and (L[t - 1] - L[t]) < 1e-3 * L[t - 1]
    assert all((L[s - 1] - L[s]) >= 1e-3 * L[s - 1] for s in range(1, t))
    # an overfitting model (rank 4 on noisy counts) eventually raises the
    # validation loss; with patience 1 the first rise stops the fit
    f, t, r, L, V = O.fit_early_stopping(p.model_str, p.init, p.Y, M, 1.0, 0.0, max_sweeps=500,
                                         patience=1, rel_tol=0.0)
    assert r in (O.STOP_VALIDATION, O.STOP_MAX)
    if r == O.STOP_VALIDATION:
        assert V[t] > V[t - 1] and all(V[s] <= V[s - 1] for s in range(1, t))
