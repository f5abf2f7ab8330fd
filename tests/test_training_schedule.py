"""Host logic of the training loop (App. B.1, Tab. 7: plateau schedule; Sec. 3.3: best validation
model kept; Sec. 4.2: seed ensembles), on scripted validation sequences."""
import numpy as np

from paper_2606_19251_amd.train import Plateau, best_run


def test_plateau_halves_after_patience_stale_evaluations():
    s = Plateau(1e-3, patience=2, factor=0.5, min_lr=1e-5)
    seq = [-0.1, -0.2, -0.15, -0.18, -0.19, -0.3, -0.3, -0.25, -0.1, -0.31]
    lrs, best = [], []
    for v in seq:
        best.append(s.update(v))
        lrs.append(s.lr)
    # new bests at -0.1, -0.2, -0.3 and -0.31 (an equal value is not an improvement)
    assert best == [True, True, False, False, False, True, False, False, False, True]
    # stale runs: (-0.15, -0.18) -> halve after the second; -0.19 then starts a new count;
    # (-0.3 equal, -0.25) -> halve; -0.1 stale once; then a new best
    assert lrs == [1e-3, 1e-3, 1e-3, 5e-4, 5e-4, 5e-4, 5e-4, 2.5e-4, 2.5e-4, 2.5e-4]
    assert s.best == -0.31


def test_plateau_respects_min_lr():
    s = Plateau(1e-3, patience=1, factor=0.1, min_lr=2e-5)
    s.update(0.0)
    for _ in range(5):
        s.update(1.0)
    assert s.lr == 2e-5


def test_best_run_is_argmin_first_among_equals():
    assert best_run([-0.2, -0.5, -0.1]) == 1
    assert best_run(np.array([-0.5, -0.5, -0.4])) == 0
