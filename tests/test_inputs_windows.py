"""Host checks of the training-window inputs (no GPU): `inputs.window` and
`precond_train.window_configs`, which cut the learned correction's training
configurations out of larger placements."""
import numpy as np

from paper_1707_06551_amd.inputs import box_side, place_spheres, window


def test_window_is_the_nearest_spheres_of_one_centre():
    c = place_spheres(128, box_side(128, 0.2), 0.02, np.random.default_rng(3))
    w = window(c, 16, np.random.default_rng(4))
    assert w.shape == (16, 3)
    # every window centre is a placement centre, all distinct
    idx = [int(np.argmin(np.linalg.norm(c - x, axis=1))) for x in w]
    assert len(set(idx)) == 16 and all(np.allclose(c[i], x) for i, x in zip(idx, w))
    # the window is the 16 spheres nearest to its first one (centre distance)
    d = np.linalg.norm(c - w[0], axis=1)
    assert np.max(np.linalg.norm(w - w[0], axis=1)) <= np.sort(d)[15] + 1e-12
    # the gap constraint of the placement carries over
    dd = np.linalg.norm(w[:, None] - w[None], axis=2) + 10 * np.eye(16)
    assert dd.min() >= 2.02 - 1e-12


def test_window_configs_do_not_depend_on_the_process_count():
    from paper_1707_06551_amd.precond_train import window_configs
    a = window_configs(5, 2, seed0=11, n=16, big=96, phi=0.2, procs=1)
    b = window_configs(5, 2, seed0=11, n=16, big=96, phi=0.2, procs=3)
    assert len(a) == len(b) == 5
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # windows of one placement differ, placements differ
    assert not np.array_equal(a[0], a[1]) and not np.array_equal(a[0], a[2])
